"""The allocation-free entry point, snap_compute_noalloc (through the C ABI),
against snap_compute on the same inputs: two calls in a row on the static
workspace, the second with a smaller system, so that the second runs on the
first one's leftovers.  Bar: energies within 1e-11 relative, forces, pair
derivatives and bispectra within 1e-10 (the kernels are the same, so the
results are expected to be identical)."""
import numpy as np
import pytest

from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

E_REL = 1e-11
F_ABS = 1e-10


def _case(pot, pos, box, beta):
    import torch
    from paper_2011_12875_amd import snapmi
    nl = snapmi.NeighborList.build(pos, box, pot.rcut)
    tpos = torch.as_tensor(pos, device="cuda")
    tbeta = torch.as_tensor(beta, device="cuda")
    ref = pot.compute(tpos, box, nl, tbeta, bispectrum=True, pair_derivs=True)
    n = len(pos)
    out = {"energy": torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
           "force": torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda"),
           "bispectrum": torch.full((n, pot.ncoeff), float("nan"), dtype=torch.float64,
                                    device="cuda"),
           "dE": torch.full((max(nl.npairs, 1), 3), float("nan"), dtype=torch.float64,
                            device="cuda")}
    torch.cuda.synchronize()
    pot.compute_noalloc(tpos, box, nl, tbeta, out, bispectrum=True, pair_derivs=True)
    pot.sync_status()
    r = {k: v.cpu().numpy() for k, v in ref.items()}
    o = {k: v.cpu().numpy() for k, v in out.items()}
    scale = np.maximum(np.abs(r["energy"]), np.abs(r["energy"]).mean())
    assert (np.abs(o["energy"] - r["energy"]) / scale).max() <= E_REL
    assert np.abs(o["force"] - r["force"]).max() <= F_ABS
    assert np.abs(o["dE"] - r["dE"]).max() <= F_ABS
    assert np.abs(o["bispectrum"] - r["bispectrum"]).max() <= F_ABS
    return max(float(np.abs(o[k] - r[k]).max()) for k in o)


def test_noalloc_two_calls_second_smaller():
    from paper_2011_12875_amd import snapmi
    pot = snapmi.SnapPotential(8, wl.RCUT)
    pos, box, beta, tj = wl.make("bcc2000_2j8")
    print("case noalloc bcc2000_2j8", flush=True)
    d1 = _case(pot, pos, box, beta)
    pos2, box2 = wl.bcc(4, 0.1, 17)
    print("case noalloc 128 atoms, 2J = 8, after the 2000-atom call", flush=True)
    d2 = _case(pot, pos2, box2, beta)
    print("max differences", d1, d2)


def test_noalloc_refusals():
    import ctypes
    import torch
    from paper_2011_12875_amd import snapmi
    lib = snapmi.load()
    pot = snapmi.SnapPotential(14, wl.RCUT)
    dummy = ctypes.c_void_p(256)  # never dereferenced: the calls fail their checks first
    box = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    # the context's tables are not on the device yet
    rc = lib.snap_compute_noalloc(pot._ctx, 64, 0, dummy, box, dummy, dummy, dummy, dummy, 0,
                                  dummy, dummy, None, None, None)
    assert rc == -1 and b"tables" in lib.snap_last_error()
    # after one allocating call, sizes beyond the static array are refused
    pos, box_np = wl.bcc(3, 0.05, 3)
    nl = snapmi.NeighborList.build(pos, box_np, wl.RCUT)
    pot.compute(torch.as_tensor(pos, device="cuda"), box_np, nl,
                torch.as_tensor(wl.beta(pot.ncoeff, 4), device="cuda"))
    torch.cuda.synchronize()
    rc = lib.snap_compute_noalloc(pot._ctx, 100000, 0, dummy, box, dummy, dummy, dummy, dummy, 0,
                                  dummy, dummy, None, None, None)
    assert rc == -1 and b"static workspace" in lib.snap_last_error()
