"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (stated by the target of this work, FP64): energies within
1e-11 relative, per atom, relative to max(|E_i|, mean_i |E_i|) so that
random-sign coefficients cannot make a near-zero E_i fail on rounding alone;
forces and pair derivatives within 1e-10 eV/A absolute.  Bispectrum
components and U follow the energy tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

pytestmark = pytest.mark.gpu

E_REL = 1e-11
F_ABS = 1e-10


def _torch():
    import torch
    return torch


def _pot(tj, **kw):
    from paper_2011_12875_amd import snapmi
    return snapmi.SnapPotential(tj, kw.pop("rcut", wl.RCUT), **kw)


def _run(pos, box, beta, tj, want_b=True, want_de=True, **kw):
    torch = _torch()
    from paper_2011_12875_amd import snapmi
    pot = _pot(tj, **kw)
    nl = snapmi.NeighborList.build(pos, box, pot.rcut)
    tpos = torch.as_tensor(pos, dtype=torch.float64, device="cuda")
    tbeta = torch.as_tensor(beta, dtype=torch.float64, device="cuda")
    out = pot.compute(tpos, box, nl, tbeta, bispectrum=want_b, pair_derivs=want_de)
    pot.sync_status()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["off"] = nl.off.cpu().numpy()
    res["nbr"] = nl.nbr.cpu().numpy()[:nl.npairs]
    res["pot"], res["nl"], res["tpos"], res["tbeta"] = pot, nl, tpos, tbeta
    return res


def _check_energy(E, Eref, idx=None):
    if idx is not None:
        E, Eref = E[idx], Eref[idx]
    scale = np.maximum(np.abs(Eref), np.abs(Eref).mean())
    err = np.abs(E - Eref) / scale
    assert err.max() <= E_REL, ("energy", err.max(), int(err.argmax()))


def _pair_map(off, nbr):
    keys = {}
    for i in range(len(off) - 1):
        for t in range(off[i], off[i + 1]):
            keys[(i, int(nbr[t]))] = t
    return keys


def _full(name):
    pos, box, beta, tj = wl.make(name)
    return pos, box, beta, tj


@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_full_parity(name):
    """Every atom, every pair: E, F, B and dE against the oracle."""
    pos, box, beta, tj = _full(name)
    print("case", name, flush=True)
    g = _run(pos, box, beta, tj)
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta)
    _check_energy(g["energy"], o["E"])
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    bscale = np.maximum(np.abs(o["B"]), 1.0)
    assert (np.abs(g["bispectrum"] - o["B"]) / bscale).max() <= E_REL
    om = _pair_map(o["off"], o["nbr"])
    gm = _pair_map(g["off"], g["nbr"])
    assert om.keys() == gm.keys()
    go = np.array([gm[k] for k in om])
    oo = np.array([om[k] for k in om])
    assert np.abs(g["dE"][go] - o["dE"][oo]).max() <= F_ABS


def test_u_and_y_workspace():
    """U_j against the oracle's explicit sum, and the Euler identity
    E_i = (1/3) Re sum_j Y_j : U_j^* (B is cubic in U), which pins Y."""
    pos, box, beta, tj = _full("bcc128_2j4")
    g = _run(pos, box, beta, tj)
    pot = g["pot"]
    n = len(pos)
    U = pot.workspace(0, n).cpu().numpy()   # [nhalf, n]
    Y = pot.workspace(1, n).cpu().numpy()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta, want_utot=True)
    offs, _ = oracle.ufull_offsets(tj)
    helem = pot.table(1)
    ref = np.stack([o["U"][:, offs[J] + p * (J + 1) + q] for J, p, q in helem])
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(ref).max()
    w = np.array([2.0 if 2 * q < J else 1.0 for J, p, q in helem])
    Ee = (w[:, None] * (Y * np.conj(U)).real).sum(0) / 3.0
    _check_energy(Ee, o["E"])


@pytest.mark.parametrize("tj", [0, 1, 2, 3, 5, 6, 7, 9, 10, 11, 12, 13])
def test_all_twojmax_small(tj):
    """Every template instance, on a small periodic crystal."""
    pos, box = wl.bcc(3, 0.1, 20 + tj)
    nb = wl.ncoeff(tj)
    beta = wl.beta(nb, 30 + tj)
    print("case twojmax", tj, flush=True)
    g = _run(pos, box, beta, tj)
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta)
    _check_energy(g["energy"], o["E"])
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    bscale = np.maximum(np.abs(o["B"]), 1.0)
    assert (np.abs(g["bispectrum"] - o["B"]) / bscale).max() <= E_REL


def _full_check(pos, box, beta, tj, label, ocall=None, **kw):
    """E, B and F of every atom and dE of every pair against the oracle."""
    print("case", label, flush=True)
    g = _run(pos, box, beta, tj, **kw)
    okw = {k: v for k, v in kw.items() if k in ("rcut", "rfac0", "rmin0", "switch_flag", "wself")}
    rcut = okw.pop("rcut", wl.RCUT)
    o = ocall() if ocall else oracle.snap(pos, box, tj, rcut, beta=beta, **okw)
    _check_energy(g["energy"], o["E"])
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    bscale = np.maximum(np.abs(o["B"]), 1.0)
    assert (np.abs(g["bispectrum"] - o["B"]) / bscale).max() <= E_REL
    om = _pair_map(o["off"], o["nbr"])
    gm = _pair_map(g["off"], g["nbr"])
    for key, t in gm.items():   # listed pairs the oracle leaves out contribute nothing
        if key not in om:
            assert np.all(g["dE"][t] == 0.0), key
    go = np.array([gm[k] for k in om], dtype=np.int64)
    oo = np.array([om[k] for k in om], dtype=np.int64)
    if len(oo):
        assert np.abs(g["dE"][go] - o["dE"][oo]).max() <= F_ABS
    return g, o


def test_2j14_full():
    """2J = 14 (204 components) at the benchmark size: every atom and pair."""
    pos, box, beta, tj = _full("bcc2000_2j14")
    _full_check(pos, box, beta, tj, "bcc2000_2j14")


def test_uneven_neighbours_full():
    """15 200 atoms with vacancies (16-30 neighbours) in one launch: every
    atom and pair (several blocks per XCD in compute_Y's walk)."""
    pos, box, beta, tj = _full("bcc15200vac_2j8")
    g, _ = _full_check(pos, box, beta, tj, "bcc15200vac_2j8")
    counts = np.diff(g["off"])
    assert counts.min() <= 20 and counts.max() >= 28
    assert np.abs(g["force"].sum(0)).max() < 1e-8


@pytest.mark.parametrize("tj", [4, 8])
def test_inner_radius(tj):
    """rmin0 = 2.9 A between the first and second BCC shells: pairs on both
    sides of the inner radius (f_c = 1 inside, theta0 offset)."""
    pos, box = wl.bcc(4, 0.1, 70 + tj)
    beta = wl.beta(wl.ncoeff(tj), 71 + tj)
    _full_check(pos, box, beta, tj, "rmin0 2.9 twojmax %d" % tj, rmin0=2.9)


def test_strict_cutoff_without_switching():
    """Switching off (f_c = 1 up to rcut): neighbours at rcut (1 - 1e-12)
    count, at rcut (1 + 1e-12) they do not, also when the list holds them
    (built to a longer cutoff, a skin)."""
    torch = _torch()
    from paper_2011_12875_amd import snapmi
    rng = np.random.default_rng(75)
    tj = 6
    beta = wl.beta(wl.ncoeff(tj), 76)
    dirs = rng.normal(size=(6, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    rc = wl.RCUT
    pos = np.concatenate([np.zeros((1, 3)),
                          rc * (1 - 1e-12) * dirs[:3], rc * (1 + 1e-12) * dirs[3:]])
    pos = np.concatenate([pos, pos + np.array([30.0, 0.0, 0.0])])
    pos[7:] += rng.normal(0.0, 0.3, size=(7, 3))   # a second, distorted copy
    box = np.zeros(3)
    g, o = _full_check(pos, box, beta, tj, "switching off at rcut", switch_flag=0)
    assert np.diff(o["off"])[0] == 3
    # the same system with a skin: pairs beyond rcut listed, still no contribution
    pot = _pot(tj, switch_flag=0)
    nl = snapmi.NeighborList.build(pos, box, rc + 0.5)
    assert nl.npairs > len(o["nbr"])
    out = pot.compute(torch.as_tensor(pos, device="cuda"), box, nl,
                      torch.as_tensor(beta, device="cuda"), pair_derivs=True)
    pot.sync_status()
    _check_energy(out["energy"].cpu().numpy(), o["E"])
    assert np.abs(out["force"].cpu().numpy() - o["F"]).max() <= F_ABS


def test_orthorhombic_box():
    """Three different periodic edges."""
    pos, box = wl.bcc((4, 5, 6), 0.1, 77)
    tj = 6
    _full_check(pos, box, wl.beta(wl.ncoeff(tj), 78), tj, "orthorhombic 4x5x6")


@pytest.mark.parametrize("open_axes", [(2,), (0, 1)])
def test_partly_open_box(open_axes):
    """A slab (z open) and a wire (x, y open): surfaces with fewer neighbours."""
    pos, box = wl.bcc((5, 4, 6), 0.1, 79, open_axes=open_axes)
    tj = 6
    g, _ = _full_check(pos, box, wl.beta(wl.ncoeff(tj), 80), tj, "open axes %s" % (open_axes,))
    assert np.diff(g["off"]).min() < 20


def test_wide_open_cluster():
    """An open cluster several cut-offs wide (each open axis holds more than
    two cells of the neighbour builder)."""
    pos, box = wl.cluster(300, 9.0, 0)
    tj = 6
    _full_check(pos, box, wl.beta(wl.ncoeff(tj), 81), tj, "cluster 300 atoms radius 9 A")


def test_many_neighbours_and_open_box():
    """More than 32 neighbours per atom (several slot chunks), open box."""
    pos, box = wl.cluster(70, 4.2, 5, min_dist=1.6)
    tj = 6
    beta = wl.beta(wl.ncoeff(tj), 6)
    g = _run(pos, box, beta, tj, rcut=6.5)
    assert np.diff(g["off"]).max() > 40
    o = oracle.snap(pos, box, tj, 6.5, beta=beta)
    _check_energy(g["energy"], o["E"])
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    assert np.abs(g["force"].sum(0)).max() < 1e-10


def test_isolated_and_lonely_atoms():
    """An isolated atom (no neighbour) and a dimer, with w_self != 1 and the
    switching function off."""
    tj = 4
    beta = wl.beta(wl.ncoeff(tj), 7)
    pos = np.array([[0.0, 0.0, 0.0], [20.0, 0.0, 0.0], [21.5, 1.0, -0.5]])
    g = _run(pos, np.zeros(3), beta, tj, wself=1.3, switch_flag=0)
    o = oracle.snap(pos, np.zeros(3), tj, wl.RCUT, beta=beta, wself=1.3, switch_flag=0)
    _check_energy(g["energy"], o["E"])
    assert np.abs(g["force"] - o["F"]).max() <= F_ABS
    assert np.all(g["force"][0] == 0.0)


def test_per_atom_beta_and_directions():
    """Per-atom coefficients, and the one- and three-direction dE kernels."""
    pos, box = wl.bcc(3, 0.1, 40)
    tj = 4
    B = wl.beta(wl.ncoeff(tj), 41, natoms=len(pos))
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=B)
    for dirs in (1, 3):
        g = _run(pos, box, B, tj, dedr_dirs=dirs)
        _check_energy(g["energy"], o["E"])
        assert np.abs(g["force"] - o["F"]).max() <= F_ABS


def test_deterministic():
    """No atomics anywhere: two evaluations are bit-identical."""
    pos, box, beta, tj = _full("bcc2000_2j8")
    g1 = _run(pos, box, beta, tj)
    torch = _torch()
    out = g1["pot"].compute(g1["tpos"], box, g1["nl"], g1["tbeta"])
    torch.cuda.synchronize()
    assert np.array_equal(out["energy"].cpu().numpy(), g1["energy"])
    assert np.array_equal(out["force"].cpu().numpy(), g1["force"])


def test_coincident_atoms_flagged():
    from paper_2011_12875_amd import snapmi
    torch = _torch()
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    tj = 2
    pot = _pot(tj)
    off = np.array([0, 2, 4, 6], dtype=np.int32)
    nbr = np.array([1, 2, 0, 2, 0, 1], dtype=np.int32)
    rev = np.array([2, 4, 0, 5, 1, 3], dtype=np.int32)
    snapmi.check_neighbors(off, nbr, rev)
    nl = snapmi.NeighborList(off, nbr, rev)
    tpos = torch.as_tensor(pos, device="cuda")
    beta = torch.as_tensor(wl.beta(wl.ncoeff(tj), 1), device="cuda")
    pot.compute(tpos, np.zeros(3), nl, beta)
    with pytest.raises(snapmi.SnapError) as e:
        pot.sync_status()
    assert e.value.code == -4
    pot.sync_status()  # cleared


def test_backward_matches_weighted_forces():
    """snap_backward with g_i gives -d(sum g_i E_i)/dr: compare with the
    oracle's forces for per-atom coefficients g_i * beta."""
    pos, box = wl.bcc(3, 0.1, 50)
    tj = 6
    beta = wl.beta(wl.ncoeff(tj), 51)
    gvec = np.random.default_rng(52).normal(size=len(pos))
    torch = _torch()
    from paper_2011_12875_amd import snapmi
    pot = _pot(tj)
    nl = snapmi.NeighborList.build(pos, box, pot.rcut)
    tpos = torch.as_tensor(pos, device="cuda")
    tbeta = torch.as_tensor(beta, device="cuda")
    E, B = pot.forward(tpos, box, nl, tbeta)
    F = pot.backward(tpos, box, nl, tbeta, torch.as_tensor(gvec, device="cuda"))
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=gvec[:, None] * beta[None, :])
    ob = oracle.snap(pos, box, tj, wl.RCUT, beta=beta)
    _check_energy(E.cpu().numpy(), ob["E"])
    assert np.abs(F.cpu().numpy() - o["F"]).max() <= F_ABS
    assert np.abs(B.cpu().numpy() - ob["B"]).max() <= E_REL * max(1.0, np.abs(ob["B"]).max())


@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_virial_matches_oracle(name):
    """W = sum_p dE_p (x) r_ik from the GPU pair derivatives against the
    oracle's (its own dE and minimum image); per-atom shares sum to W; W is
    symmetric (rotational invariance)."""
    pos, box, beta, tj = _full(name)
    g = _run(pos, box, beta, tj)
    W, Wa = g["pot"].virial(g["tpos"], box, g["nl"], _torch().as_tensor(g["dE"], device="cuda"),
                            per_atom=True)
    W, Wa = W.cpu().numpy(), Wa.cpu().numpy()
    o = oracle.snap(pos, box, tj, wl.RCUT, beta=beta)
    Wo, Wao = oracle.virial(pos, box, o["off"], o["nbr"], o["dE"])
    scale = np.abs(Wao).max()
    assert np.abs(Wa - Wao).max() <= 1e-10 * scale
    assert np.abs(W - Wo).max() <= 1e-10 * np.abs(Wo).max()
    assert np.abs(Wa.sum(0) - W).max() <= 1e-12 * np.abs(W).max() * len(pos)
    assert np.abs(W - W.T).max() <= 1e-9 * np.abs(W).max()
