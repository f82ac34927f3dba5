"""Quadratic SNAP on the GPU (E_i = beta . B_i + B_i^T alpha B_i / 2, forces
through the adjoint with per-atom coefficients) against the oracle's
quadratic energy and literal dB/dr forces: every atom and every pair."""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

E_REL = 1e-11
F_ABS = 1e-10


def _run(pos, box, beta, alpha, tj):
    import torch
    from paper_2011_12875_amd import snapmi
    pot = snapmi.SnapPotential(tj, wl.RCUT)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    out = pot.compute_quadratic(torch.as_tensor(pos, device="cuda"), box, nl,
                                torch.as_tensor(beta, device="cuda"),
                                torch.as_tensor(alpha, device="cuda"), bispectrum=True,
                                pair_derivs=True)
    pot.sync_status()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["off"], res["nbr"] = nl.off.cpu().numpy(), nl.nbr.cpu().numpy()[:nl.npairs]
    res["pot"], res["nl"] = pot, nl
    return res


@pytest.mark.parametrize("name,scale", [("bcc128_2j4", 1e-2), ("bcc2000_2j8", 1e-4)])
def test_quadratic_matches_oracle(name, scale):
    pos, box, beta, tj = wl.make(name)
    alpha = wl.quadratic_alpha(len(beta), 90, scale)
    print("case", name, flush=True)
    g = _run(pos, box, beta, alpha, tj)
    o = oracle.snap_quadratic(pos, box, tj, wl.RCUT, beta, alpha)
    esc = np.maximum(np.abs(o["E"]), np.abs(o["E"]).mean())
    assert (np.abs(g["energy"] - o["E"]) / esc).max() <= E_REL
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    bsc = np.maximum(np.abs(o["B"]), 1.0)
    assert (np.abs(g["bispectrum"] - o["B"]) / bsc).max() <= E_REL
    # same neighbour order on both sides (sorted CSR lists of the same pairs)
    assert np.array_equal(g["off"], o["off"])
    assert np.abs(g["dE"] - o["dE"]).max() <= F_ABS
    # the quadratic part is a real share of the energy here
    lin = o["B"] @ beta
    assert np.abs(o["E"] - lin).mean() > 0.1 * np.abs(lin).mean()


def test_alpha_zero_equals_linear():
    import torch
    pos, box, beta, tj = wl.make("bcc128_2j4")
    g = _run(pos, box, beta, np.zeros((len(beta), len(beta))), tj)
    lin = g["pot"].compute(torch.as_tensor(pos, device="cuda"), box, g["nl"],
                           torch.as_tensor(beta, device="cuda"))
    # same per-atom coefficients in compute_Y: identical forces
    assert np.array_equal(lin["force"].cpu().numpy(), g["force"])
    e = lin["energy"].cpu().numpy()
    assert np.abs(e - g["energy"]).max() <= 1e-12 * np.abs(e).max()
