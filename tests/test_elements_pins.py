"""Pins of the oracle's several-element SNAP (CPU only).

The paper's eq. (u) leaves out the density weights and per-element radii of
multi-element SNAP (Sec. II.A defers them to the SNAP reference); the reading
used here: element e has a radius R_e and weight w_e, the pair (i, k) has the
cutoff R_ik = rcutfac (R_t(i) + R_t(k)) and enters U_i as w_t(k) f_c u, and
E_i uses the coefficients of the centre's element.  Each pin ties that
reading to something other than the oracle's own element code: the
one-element special case, closed-form scalings (B is cubic in U), dimers and
trimers that reduce to one-element evaluations with a chosen cutoff, and
central finite differences of the total energy.
"""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

TJ = 4


def _beta(nelem, seed):
    return np.stack([wl.beta(wl.ncoeff(TJ), seed + e) for e in range(nelem)])


def test_one_element_is_plain_snap():
    """One element of radius R with rcutfac = 1/2 is plain SNAP with rcut = R."""
    pos, box = wl.bcc(3, 0.1, 31)
    b = _beta(1, 32)
    o = oracle.snap(pos, box, TJ, wl.RCUT, beta=b[0])
    m = oracle.snap_elements(pos, box, TJ, np.zeros(len(pos), int), [wl.RCUT], [1.0], 0.5, b)
    for k in ("E", "F", "B", "dE"):
        np.testing.assert_allclose(m[k], o[k], rtol=0, atol=1e-13)


def test_uniform_weight_scales_cubically():
    """w_self = 0 and every weight lambda: U -> lambda U, so B, E and F scale
    by lambda^3 (eq. (z) is cubic in U)."""
    pos, box = wl.cluster(12, 3.2, seed=33)
    types = np.random.default_rng(34).integers(0, 2, len(pos))
    rad, b = [2.4, 2.7], _beta(2, 35)
    lam = 1.7
    a = oracle.snap_elements(pos, box, TJ, types, rad, [1.0, 1.0], 1.0, b, wself=0.0)
    c = oracle.snap_elements(pos, box, TJ, types, rad, [lam, lam], 1.0, b, wself=0.0)
    for k in ("E", "B", "F"):
        np.testing.assert_allclose(c[k], lam ** 3 * a[k], rtol=1e-12, atol=1e-12)


def test_weight_is_the_neighbours():
    """Dimer A-B with w_self = 0: U_A holds w_B u(r_AB) only and U_B holds
    w_A u(r_BA), so B_A = w_B^3 B_plain(A) and B_B = w_A^3 B_plain(B)."""
    pos = np.array([[0.0, 0.0, 0.0], [1.3, -0.4, 2.1]])
    box = np.zeros(3)
    rc = 3.0
    plain = oracle.snap(pos, box, TJ, rc, beta=np.zeros(wl.ncoeff(TJ)), wself=0.0)
    wA, wB = 0.6, 1.9
    m = oracle.snap_elements(pos, box, TJ, [0, 1], [rc / 2, rc / 2], [wA, wB], 1.0,
                             np.zeros((2, wl.ncoeff(TJ))), wself=0.0)
    np.testing.assert_allclose(m["B"][0], wB ** 3 * plain["B"][0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m["B"][1], wA ** 3 * plain["B"][1], rtol=1e-12, atol=1e-14)


def test_pair_cutoff_combines_both_radii():
    """Centre A with an A neighbour and a B neighbour at the same distance d,
    2 rcutfac R_A < d < rcutfac (R_A + R_B): only the B neighbour counts, with
    the cutoff rcutfac (R_A + R_B) in its 3-sphere map and switching."""
    d = 2.5
    pos = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0], [0.0, 0.6 * d, 0.8 * d]])
    box = np.zeros(3)
    rA, rB, f = 1.1, 1.9, 1.0   # A-A cutoff 2.2 < d < A-B cutoff 3.0
    nb = wl.ncoeff(TJ)
    b = _beta(2, 36)
    m = oracle.snap_elements(pos, box, TJ, [0, 0, 1], [rA, rB], [1.0, 1.4], f, b, want_utot=True)
    # centre 0 alone with its B neighbour, plain SNAP with the A-B cutoff
    two = oracle.snap(pos[[0, 2]], box, TJ, f * (rA + rB), beta=b[0], want_utot=True)
    Uw = two["U"][0].copy()
    # the B neighbour's weight scales the neighbour part of U (w_self stays)
    offs, _ = oracle.ufull_offsets(TJ)
    eye = np.zeros_like(Uw)
    for J in range(TJ + 1):
        for p in range(J + 1):
            eye[offs[J] + p * (J + 1) + p] = 1.0
    np.testing.assert_allclose(m["U"][0], eye + 1.4 * (Uw - eye), rtol=0, atol=1e-13)
    # atom 1 (A) sees atom 0 (A) at d: beyond 2.2, and atom 2 (B) at
    # sqrt(d^2 + d^2) > 3.0: nothing but w_self
    np.testing.assert_allclose(m["U"][1], eye, rtol=0, atol=0)
    assert np.all(m["dE"][m["off"][1]:m["off"][2]] == 0.0)


def test_forces_are_energy_gradients():
    """Three elements with different radii and weights, per-element
    coefficients: F = -dE_total/dr by central differences."""
    pos, box = wl.cluster(10, 3.0, seed=37)
    types = np.random.default_rng(38).integers(0, 3, len(pos))
    rad, w, f = [2.2, 2.6, 2.9], [0.8, 1.3, 1.1], 0.9
    b = _beta(3, 39)
    m = oracle.snap_elements(pos, box, TJ, types, rad, w, f, b)
    h = 1e-5
    for i in (0, 3, 7):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            ep = oracle.snap_elements(pp, box, TJ, types, rad, w, f, b)["E"].sum()
            em = oracle.snap_elements(pm, box, TJ, types, rad, w, f, b)["E"].sum()
            assert abs(-(ep - em) / (2 * h) - m["F"][i, a]) < 2e-7, (i, a)


def test_energy_uses_the_centre_elements_coefficients():
    """eq. (snapatomenergy) per element: E_i = beta[t_i] . B_i."""
    pos, box = wl.cluster(9, 3.0, seed=40)
    types = np.random.default_rng(41).integers(0, 2, len(pos))
    b = _beta(2, 42)
    m = oracle.snap_elements(pos, box, TJ, types, [2.3, 2.6], [1.0, 0.7], 1.0, b)
    np.testing.assert_allclose(m["E"], (b[types] * m["B"]).sum(1), rtol=1e-13, atol=1e-13)


def test_bad_types_rejected():
    pos, box = wl.cluster(4, 3.0, seed=43)
    with pytest.raises(RuntimeError):
        oracle.snap_elements(pos, box, TJ, [0, 1, 2, 0], [2.0, 2.0], [1.0, 1.0], 1.0, _beta(2, 44))
