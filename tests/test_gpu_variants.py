"""GPU parity of the selectable kernel variants (snap_params.y_kernel,
dedr_dirs, dedr_kernel, dedr_waves, u_kernel) against the CPU oracle, on
every atom and pair.

Tolerances as in test_gpu_parity: energies within 1e-11 relative to
max(|E_i|, mean |E_i|), forces and pair derivatives within 1e-10 eV/A.
"""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

E_REL = 1e-11
F_ABS = 1e-10


def _compare(pos, box, beta, tj, **kw):
    import torch
    from paper_2011_12875_amd import snapmi
    pot = snapmi.SnapPotential(tj, wl.RCUT, **kw)
    nl = snapmi.NeighborList.build(pos, box, wl.RCUT)
    tpos = torch.as_tensor(pos, device="cuda")
    tbeta = torch.as_tensor(beta, device="cuda")
    out = pot.compute(tpos, box, nl, tbeta, bispectrum=False, pair_derivs=True)
    pot.sync_status()
    E = out["energy"].cpu().numpy()
    F = out["force"].cpu().numpy()
    dE = out["dE"].cpu().numpy()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta)
    scale = np.maximum(np.abs(o["E"]), np.abs(o["E"]).mean())
    assert (np.abs(E - o["E"]) / scale).max() <= E_REL
    assert np.abs(F - o["F"]).max() <= F_ABS
    off, nbr = nl.off.cpu().numpy(), nl.nbr.cpu().numpy()[:nl.npairs]
    gm = {(i, int(nbr[t])): t for i in range(len(off) - 1) for t in range(off[i], off[i + 1])}
    om = {(i, int(o["nbr"][t])): t for i in range(len(o["off"]) - 1)
          for t in range(o["off"][i], o["off"][i + 1])}
    assert gm.keys() == om.keys()
    keys = list(om)
    assert np.abs(dE[[gm[k] for k in keys]] - o["dE"][[om[k] for k in keys]]).max() <= F_ABS


@pytest.mark.parametrize("y_kernel", [1, 2])
@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_y_kernel_variants(name, y_kernel):
    pos, box, beta, tj = wl.make(name)
    print("case", name, "y_kernel", y_kernel, flush=True)
    _compare(pos, box, beta, tj, y_kernel=y_kernel)


@pytest.mark.parametrize("tj", [2, 3, 5, 6, 7])
def test_y_lds_small(tj):
    pos, box = wl.bcc(3, 0.1, 40 + tj)
    beta = wl.beta(wl.ncoeff(tj), 50 + tj)
    print("case twojmax", tj, "y_kernel 2", flush=True)
    _compare(pos, box, beta, tj, y_kernel=2)


@pytest.mark.parametrize("dirs", [1, 3])
@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_dedr_dirs_variants(name, dirs):
    pos, box, beta, tj = wl.make(name)
    print("case", name, "dedr_dirs", dirs, flush=True)
    _compare(pos, box, beta, tj, dedr_dirs=dirs)


@pytest.mark.parametrize("kern", [1, 2, 3, 4])
@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_dedr_kernel_variants(name, kern):
    pos, box, beta, tj = wl.make(name)
    print("case", name, "dedr_kernel", kern, flush=True)
    _compare(pos, box, beta, tj, dedr_kernel=kern)


@pytest.mark.parametrize("kern", [2, 3, 4])
@pytest.mark.parametrize("tj", [0, 1, 2, 3, 5, 6, 7, 9, 10, 11, 12, 13, 14])
def test_dedr_generator_every_twojmax(tj, kern):
    """Every template instance of the generator form (straight-line and looped
    levels, one and two wavefronts per block, staged and unstaged Y~)."""
    pos, box = wl.bcc(3, 0.1, 60 + tj)
    beta = wl.beta(wl.ncoeff(tj), 70 + tj)
    print("case twojmax", tj, "dedr_kernel", kern, flush=True)
    _compare(pos, box, beta, tj, dedr_kernel=kern)


@pytest.mark.parametrize("waves", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("tj", [7, 8])
def test_dedr_waves_every_split(tj, waves):
    """The generator form with its columns split over 1 .. 4 wavefronts, and
    the automatic choice (0: three at 2J = 7 and 8 on a system this small)."""
    pos, box = wl.bcc(3, 0.1, 110 + tj)
    beta = wl.beta(wl.ncoeff(tj), 120 + tj)
    print("case twojmax", tj, "dedr_waves", waves, flush=True)
    _compare(pos, box, beta, tj, dedr_waves=waves)


@pytest.mark.parametrize("waves", [2, 3])
def test_dedr_waves_2000_atoms(waves):
    pos, box, beta, tj = wl.make("bcc2000_2j8")
    print("case bcc2000_2j8 dedr_waves", waves, flush=True)
    _compare(pos, box, beta, tj, dedr_waves=waves)


@pytest.mark.parametrize("kern", [1, 2, 3])
@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_u_kernel_variants(name, kern):
    pos, box, beta, tj = wl.make(name)
    print("case", name, "u_kernel", kern, flush=True)
    _compare(pos, box, beta, tj, u_kernel=kern)


@pytest.mark.parametrize("kern", [2, 3])
@pytest.mark.parametrize("tj", [0, 1, 2, 3, 5, 6, 7, 9, 10, 11, 12, 13, 14])
def test_u_lane_every_twojmax(tj, kern):
    pos, box = wl.bcc(3, 0.1, 80 + tj)
    beta = wl.beta(wl.ncoeff(tj), 90 + tj)
    print("case twojmax", tj, "u_kernel", kern, flush=True)
    _compare(pos, box, beta, tj, u_kernel=kern)


@pytest.mark.parametrize("kern", [1, 2, 3])
def test_u_long_neighbour_lists(kern):
    """More than 32 neighbours per atom (several chunks of lanes per atom;
    more than 64 for the lanes-over-elements variant): a dense cluster with a
    cutoff that takes in up to 75 neighbours."""
    rng = np.random.default_rng(7)
    n = 150
    pos = rng.uniform(0.0, 9.0, (n, 3))
    box = np.array([0.0, 0.0, 0.0])
    tj = 6
    beta = wl.beta(wl.ncoeff(tj), 11)
    import torch
    from paper_2011_12875_amd import snapmi
    rcut = 4.5
    pot = snapmi.SnapPotential(tj, rcut, u_kernel=kern)
    nl = snapmi.NeighborList.build(pos, box, rcut)
    counts = np.diff(nl.off.cpu().numpy())
    assert counts.max() > 32, counts.max()
    out = pot.compute(torch.as_tensor(pos, device="cuda"), box, nl,
                      torch.as_tensor(beta, device="cuda"))
    pot.sync_status()
    o = oracle.snap(pos, box, tj, rcut, beta=beta, want_dE=False)
    E, F = out["energy"].cpu().numpy(), out["force"].cpu().numpy()
    scale = np.maximum(np.abs(o["E"]), np.abs(o["E"]).mean())
    assert (np.abs(E - o["E"]) / scale).max() <= E_REL
    assert np.abs(F - o["F"]).max() <= F_ABS


@pytest.mark.parametrize("waves", [1, 2, 3, 4])
@pytest.mark.parametrize("tj", [4, 8, 14])
def test_dedr_waves(tj, waves):
    """The generator form with the columns split over 1 .. 4 wavefronts."""
    pos, box = wl.bcc(3, 0.1, 100 + tj)
    beta = wl.beta(wl.ncoeff(tj), 110 + tj)
    print("case twojmax", tj, "dedr_waves", waves, flush=True)
    _compare(pos, box, beta, tj, dedr_kernel=2, dedr_waves=waves)
