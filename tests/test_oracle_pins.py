"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it does not compute the same
way: sympy's exact Clebsch-Gordan values, a polynomial expansion done by
numpy convolution, group-theory identities (unitarity, homomorphism, the
Clebsch-Gordan series), closed forms for an isolated atom and a single
neighbour, invariances, and finite differences of the energy.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RC, RF, RM = wl.RCUT, wl.RFAC0, wl.RMIN0


# --------------------------------------------------------------------------
# component enumeration (Sec. II.A; counts printed in Sec. II.C / III)
# --------------------------------------------------------------------------

def test_component_counts_golden():
    gold = json.load(open(os.path.join(GOLD, "component_counts.json")))["counts"]
    for tj, n in gold.items():
        assert len(oracle.components(int(tj))) == n


def test_component_rules():
    for tj in (2, 4, 8):
        tri = oracle.components(tj)
        assert len({tuple(t) for t in tri}) == len(tri)
        for J1, J2, J in tri:
            assert 0 <= J2 <= J1 <= J <= tj
            assert abs(J1 - J2) <= J <= J1 + J2 and (J1 + J2 + J) % 2 == 0


# --------------------------------------------------------------------------
# Clebsch-Gordan coefficients
# --------------------------------------------------------------------------

def _sympy_cg(J1, M1, J2, M2, J, M):
    from sympy import Rational
    from sympy.physics.quantum.cg import CG
    h = lambda x: Rational(x, 2)
    return float(CG(h(J1), h(M1), h(J2), h(M2), h(J), h(M)).doit())


def test_cg_matches_sympy_small():
    worst = 0.0
    for J1 in range(0, 5):
        for J2 in range(0, 5):
            for J in range(abs(J1 - J2), J1 + J2 + 1, 2):
                for M1 in range(-J1, J1 + 1, 2):
                    for M2 in range(-J2, J2 + 1, 2):
                        M = M1 + M2
                        if abs(M) > J:
                            continue
                        ref = _sympy_cg(J1, M1, J2, M2, J, M)
                        worst = max(worst, abs(ref - oracle.cg(J1, M1, J2, M2, J, M)))
    assert worst < 1e-14


def test_cg_matches_sympy_sampled_large():
    rng = np.random.default_rng(0)
    for _ in range(120):
        J1 = int(rng.integers(0, 15))
        J2 = int(rng.integers(0, 15))
        Js = list(range(abs(J1 - J2), min(J1 + J2, 14) + 1, 2))
        if not Js:
            continue
        J = int(rng.choice(Js))
        M1 = int(rng.choice(range(-J1, J1 + 1, 2)))
        M2c = [m for m in range(-J2, J2 + 1, 2) if abs(M1 + m) <= J]
        if not M2c:
            continue
        M2 = int(rng.choice(M2c))
        ref = _sympy_cg(J1, M1, J2, M2, J, M1 + M2)
        assert abs(ref - oracle.cg(J1, M1, J2, M2, J, M1 + M2)) < 1e-13


def test_cg_orthogonality():
    for J1, J2 in [(3, 2), (4, 4), (6, 3), (8, 8)]:
        Js = list(range(abs(J1 - J2), J1 + J2 + 1, 2))
        for M in range(-(J1 + J2), J1 + J1 + 1, 2):
            rows = [(M1, M - M1) for M1 in range(-J1, J1 + 1, 2) if abs(M - M1) <= J2]
            cols = [J for J in Js if abs(M) <= J]
            if not rows:
                continue
            C = np.array([[oracle.cg(J1, m1, J2, m2, J, M) for J in cols] for m1, m2 in rows])
            assert np.allclose(C.T @ C, np.eye(len(cols)), atol=1e-13)
            assert np.allclose(C @ C.T, np.eye(len(rows)), atol=1e-13)


# --------------------------------------------------------------------------
# hyperspherical harmonics u^J (the SU(2) representation matrices)
# --------------------------------------------------------------------------

def _random_su2(rng):
    v = rng.normal(size=4)
    v /= np.linalg.norm(v)
    return v[0] + 1j * v[1], v[2] + 1j * v[3]


def _sym_power_by_convolution(J, a, b):
    """Matrix of x -> a x + b y, y -> -b* x + a* y on degree-J polynomials in
    the basis x^p y^(J-p)/sqrt(p!(J-p)!), by multiplying coefficient arrays."""
    from math import factorial
    gx = np.array([b, a])             # coefficients in powers of x: b*y + a*x (y^1 x^0, x^1)
    gy = np.array([np.conj(a), -np.conj(b)])
    U = np.zeros((J + 1, J + 1), dtype=complex)
    for q in range(J + 1):
        poly = np.array([1.0 + 0j])
        for _ in range(q):
            poly = np.convolve(poly, gx)
        for _ in range(J - q):
            poly = np.convolve(poly, gy)
        # poly[p] is the coefficient of x^p y^(J-p)
        for p in range(J + 1):
            U[p, q] = poly[p] * np.sqrt(factorial(p) * factorial(J - p) /
                                        (factorial(q) * factorial(J - q)))
    return U


def test_wigner_j1_closed_form():
    rng = np.random.default_rng(1)
    a, b = _random_su2(rng)
    u = oracle.wigner(1, a, b)
    assert np.allclose(u, [[np.conj(a), b], [-np.conj(b), a]], atol=1e-15)


def test_wigner_matches_polynomial_expansion():
    rng = np.random.default_rng(2)
    for J in range(0, 15):
        a, b = _random_su2(rng)
        assert np.allclose(oracle.wigner(J, a, b), _sym_power_by_convolution(J, a, b), atol=1e-13)


def test_wigner_unitary_homomorphism_symmetry():
    rng = np.random.default_rng(3)
    for J in (1, 2, 5, 8, 14):
        a1, b1 = _random_su2(rng)
        a2, b2 = _random_su2(rng)
        u1, u2 = oracle.wigner(J, a1, b1), oracle.wigner(J, a2, b2)
        assert np.allclose(u1 @ u1.conj().T, np.eye(J + 1), atol=1e-13)
        # the 2x2 matrix with columns the images of x and y
        M1 = np.array([[a1, -np.conj(b1)], [b1, np.conj(a1)]])
        M2 = np.array([[a2, -np.conj(b2)], [b2, np.conj(a2)]])
        M12 = M1 @ M2
        u12 = oracle.wigner(J, M12[0, 0], M12[1, 0])
        assert np.allclose(u12, u1 @ u2, atol=1e-12)
        # u_{J-p,J-q} = (-1)^(p-q) conj(u_{pq})
        p, q = np.meshgrid(np.arange(J + 1), np.arange(J + 1), indexing="ij")
        assert np.allclose(u1[::-1, ::-1], ((-1.0) ** (p - q)) * np.conj(u1), atol=1e-13)


# --------------------------------------------------------------------------
# 3-sphere map and switching function derivatives
# --------------------------------------------------------------------------

def test_geometry_unit_norm_and_fd():
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(20):
        rv = rng.normal(size=3)
        rv *= rng.uniform(1.5, 4.6) / np.linalg.norm(rv)
        g = oracle.geometry(rv, RC, RF, RM)
        assert abs(abs(g["a"]) ** 2 + abs(g["b"]) ** 2 - 1.0) < 1e-15
        for al in range(3):
            e = np.zeros(3)
            e[al] = h
            gp, gm = oracle.geometry(rv + e, RC, RF, RM), oracle.geometry(rv - e, RC, RF, RM)
            assert abs((gp["a"] - gm["a"]) / (2 * h) - g["da"][al]) < 1e-8
            assert abs((gp["b"] - gm["b"]) / (2 * h) - g["db"][al]) < 1e-8
            assert abs((gp["fc"] - gm["fc"]) / (2 * h) - g["dfc"][al]) < 1e-8


def test_switching_values():
    g = oracle.geometry(np.array([0.0, 0.0, RC * (1 - 1e-12)]), RC, RF, RM)
    assert abs(g["fc"]) < 1e-20
    g = oracle.geometry(np.array([0.0, 0.0, 0.5 * RC]), RC, RF, RM)
    assert abs(g["fc"] - 0.5) < 1e-15
    g = oracle.geometry(np.array([0.0, 0.0, 0.5 * RC]), RC, RF, RM, switch_flag=0)
    assert g["fc"] == 1.0 and np.all(g["dfc"] == 0.0)


# --------------------------------------------------------------------------
# closed forms of the bispectrum
# --------------------------------------------------------------------------

def _beta(nb, seed=0):
    return np.random.default_rng(seed).normal(0, 0.1, nb)


@pytest.mark.parametrize("tj", [4, 8])
@pytest.mark.parametrize("wself", [1.0, 1.7])
def test_isolated_atom(tj, wself):
    """Utot^J = w_self I  =>  Z = w_self^2 I (orthogonality)  =>  B = w_self^3 (J+1)."""
    tri = oracle.components(tj)
    out = oracle.snap(np.zeros((1, 3)), np.zeros(3), tj, RC, wself=wself, beta=_beta(len(tri)))
    ref = wself ** 3 * (tri[:, 2] + 1.0)
    assert np.allclose(out["B"][0], ref, rtol=1e-14, atol=0)
    assert np.all(out["F"] == 0)


@pytest.mark.parametrize("tj", [4, 8, 14])
def test_single_neighbour_clebsch_gordan_series(tj):
    """w_self = 0 and one neighbour: U^J = f_c u^J, the Clebsch-Gordan series
    gives Z^J_{J1J2} = f_c^2 u^J, and unitarity gives B = f_c^3 (J+1)."""
    tri = oracle.components(tj)
    pos = np.array([[0.0, 0.0, 0.0], [1.3, -2.1, 1.7]])
    out = oracle.snap(pos, np.zeros(3), tj, RC, wself=0.0, beta=_beta(len(tri)))
    fc = oracle.geometry(pos[1] - pos[0], RC, RF, RM)["fc"]
    assert np.allclose(out["B"][0], fc ** 3 * (tri[:, 2] + 1.0), rtol=1e-12, atol=1e-14)


def test_energy_is_linear_in_beta():
    tj = 4
    pos, box = wl.bcc(3, 0.1, 11)
    nb = len(oracle.components(tj))
    rng = np.random.default_rng(5)
    b1, b2 = rng.normal(size=nb), rng.normal(size=nb)
    o1 = oracle.snap(pos, box, tj, RC, beta=b1)
    o2 = oracle.snap(pos, box, tj, RC, beta=b2)
    o12 = oracle.snap(pos, box, tj, RC, beta=b1 + 2 * b2)
    assert np.allclose(o12["E"], o1["E"] + 2 * o2["E"], rtol=1e-12, atol=1e-12)
    assert np.allclose(o1["E"], o1["B"] @ b1, rtol=1e-13, atol=1e-13)
    assert np.allclose(o12["F"], o1["F"] + 2 * o2["F"], atol=1e-11)


# --------------------------------------------------------------------------
# invariances
# --------------------------------------------------------------------------

def _rotation(seed):
    from scipy.spatial.transform import Rotation
    return Rotation.random(random_state=seed).as_matrix()


@pytest.mark.parametrize("tj", [4, 8])
def test_rotation_invariance_cluster(tj):
    pos, box = wl.cluster(12, 3.2, seed=7)
    nb = len(oracle.components(tj))
    beta = _beta(nb, 3)
    R = _rotation(8)
    o = oracle.snap(pos, box, tj, RC, beta=beta)
    orot = oracle.snap(pos @ R.T, box, tj, RC, beta=beta)
    scale = np.abs(o["B"]).max()
    assert np.abs(orot["B"] - o["B"]).max() < 1e-12 * scale
    assert np.allclose(orot["F"], o["F"] @ R.T, atol=1e-11)
    # net force and net torque vanish for an isolated cluster
    assert np.abs(o["F"].sum(0)).max() < 1e-12
    assert np.abs(np.cross(pos, o["F"]).sum(0)).max() < 1e-11


def test_permutation_and_translation_invariance():
    tj = 6
    pos, box = wl.bcc(3, 0.1, 12)
    nb = len(oracle.components(tj))
    beta = _beta(nb, 4)
    o = oracle.snap(pos, box, tj, RC, beta=beta)
    perm = np.random.default_rng(9).permutation(len(pos))
    op = oracle.snap(pos[perm], box, tj, RC, beta=beta)
    assert np.allclose(op["E"], o["E"][perm], rtol=1e-12, atol=1e-13)
    assert np.allclose(op["F"], o["F"][perm], atol=1e-12)
    ot = oracle.snap(np.mod(pos + np.array([1.1, -2.3, 0.7]), box[0]), box, tj, RC, beta=beta)
    assert np.allclose(ot["E"], o["E"], rtol=1e-12, atol=1e-13)
    assert np.allclose(ot["F"], o["F"], atol=1e-12)
    # periodic crystal: forces sum to zero (Newton's third law pair by pair)
    assert np.abs(o["F"].sum(0)).max() < 1e-12


# --------------------------------------------------------------------------
# finite differences
# --------------------------------------------------------------------------

def _local_energy(pos, box, tj, beta, k, centres):
    o = oracle.snap(pos, box, tj, RC, beta=beta, centers=centres, want_dE=False)
    return o["E"][centres].sum()


@pytest.mark.parametrize("tj", [4, 8])
def test_forces_match_finite_differences(tj):
    """F_k = -d(sum_i E_i)/dr_k by central differences (h = 1e-5 A) on the
    local energy of k and its neighbours."""
    pos, box = wl.bcc(3, 0.1, 13)
    nb = len(oracle.components(tj))
    beta = _beta(nb, 6)
    full = oracle.snap(pos, box, tj, RC, beta=beta)
    off, nbr = full["off"], full["nbr"]
    h = 1e-5
    for k in (0, 17, 40):
        centres = np.unique(np.concatenate([[k], nbr[off[k]:off[k + 1]]]))
        for al in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, al] += h
            pm[k, al] -= h
            fd = -(_local_energy(pp, box, tj, beta, k, centres) -
                   _local_energy(pm, box, tj, beta, k, centres)) / (2 * h)
            assert abs(fd - full["F"][k, al]) < 1e-7, (k, al, fd, full["F"][k, al])


def test_pair_derivative_matches_finite_differences():
    """dE_p = dE_i/dr_ik for p = (i -> k): move k only, watch E_i only."""
    tj = 6
    pos, box = wl.bcc(3, 0.1, 14)
    nb = len(oracle.components(tj))
    beta = _beta(nb, 7)
    full = oracle.snap(pos, box, tj, RC, beta=beta)
    off, nbr, dE = full["off"], full["nbr"], full["dE"]
    i = 5
    h = 1e-5
    for t in (off[i], off[i] + 3, off[i + 1] - 1):
        k = nbr[t]
        for al in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, al] += h
            pm[k, al] -= h
            ep = oracle.snap(pp, box, tj, RC, beta=beta, centers=[i], want_dE=False)["E"][i]
            em = oracle.snap(pm, box, tj, RC, beta=beta, centers=[i], want_dE=False)["E"][i]
            assert abs((ep - em) / (2 * h) - dE[t, al]) < 1e-8


def test_per_atom_beta():
    tj = 4
    pos, box = wl.bcc(3, 0.1, 15)
    nb = len(oracle.components(tj))
    B = np.random.default_rng(16).normal(0, 0.1, (len(pos), nb))
    o = oracle.snap(pos, box, tj, RC, beta=B)
    assert np.allclose(o["E"], np.einsum("il,il->i", o["B"], B), rtol=1e-13, atol=1e-14)
    # forces are the sum of per-atom contributions: compare with scaling one row
    B2 = B.copy()
    B2[3] *= 2.0
    o2 = oracle.snap(pos, box, tj, RC, beta=B2)
    B3 = np.zeros_like(B)
    B3[3] = B[3]
    o3 = oracle.snap(pos, box, tj, RC, beta=B3)
    assert np.allclose(o2["F"], o["F"] + o3["F"], atol=1e-12)


# --------------------------------------------------------------------------
# neighbour list shape of the benchmark
# --------------------------------------------------------------------------

def test_bcc_has_26_neighbours():
    gold = json.load(open(os.path.join(GOLD, "bcc_shells.json")))
    pos, box = wl.bcc(3, 0.0, 0)
    off, nbr = oracle.neighbors(pos, box, gold["rcut"])
    assert np.all(np.diff(off) == gold["neighbours_per_atom"])


def test_cutoff_is_strict_without_switching():
    """r == rcut is outside (strict inequality of eq. (u)); just inside counts."""
    tj = 2
    nb = len(oracle.components(tj))
    beta = _beta(nb, 1)
    for r, expect in ((RC, 0), (RC * (1 - 1e-12), 1)):
        pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
        o = oracle.snap(pos, np.zeros(3), tj, RC, switch_flag=0, beta=beta)
        assert np.diff(o["off"])[0] == expect
