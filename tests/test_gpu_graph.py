"""A SNAP step captured in a hipGraph (torch.cuda.CUDAGraph around the
library call): every replay, with eager work and synchronisations between
replays, gives bit-for-bit the result of the eager call."""
import numpy as np
import pytest

from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_graph_replays_match_eager(name):
    import torch
    from paper_2011_12875_amd import snapmi
    pos, box, beta, tj = wl.make(name)
    n = len(pos)
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    tpos = torch.as_tensor(pos, device="cuda")
    tbeta = torch.as_tensor(beta, device="cuda")
    out = {"energy": torch.empty(n, dtype=torch.float64, device="cuda"),
           "force": torch.empty((n, 3), dtype=torch.float64, device="cuda")}
    ref = pot.compute(tpos, box, nl, tbeta)          # eager, own outputs
    torch.cuda.synchronize()
    e_ref, f_ref = ref["energy"].cpu().numpy(), ref["force"].cpu().numpy()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pot.compute(tpos, box, nl, tbeta, out=out)   # warm the workspace outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pot.compute(tpos, box, nl, tbeta, out=out)
    other = torch.as_tensor(wl.bcc(4, 0.2, 5)[0], device="cuda")
    onl = snapmi.NeighborList.build(other.cpu().numpy(), wl.bcc(4, 0.2, 5)[1], wl.RCUT)
    for rep in range(4):
        out["energy"].zero_()
        out["force"].zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out["energy"].cpu().numpy(), e_ref), rep
        assert np.array_equal(out["force"].cpu().numpy(), f_ref), rep
        # eager work on the same context between replays
        pot.compute(other, wl.bcc(4, 0.2, 5)[1], onl, torch.as_tensor(
            wl.beta(pot.ncoeff, 6), device="cuda"))
        torch.cuda.synchronize()
    pot.sync_status()
