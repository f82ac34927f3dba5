"""Pins of the oracle's inner radius rmin0 > 0 (the 3-sphere map and the
switching function of eq. (u), with the conventions fixed for what Sec. II.A
leaves to its SNAP reference):

  theta0 = rfac0 pi (r - rmin0) / (rcut - rmin0),
  f_c    = (cos(pi (r - rmin0)/(rcut - rmin0)) + 1)/2 for rmin0 < r < rcut,
           1 for r <= rmin0.

Each check is a closed form or a finite difference, so that a wrong offset,
a wrong span or a missing plateau below rmin0 fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import workloads as wl

RC, RF = wl.RCUT, wl.RFAC0
RMIN = 2.9   # between the first (2.754 A) and second (3.180 A) BCC shells


def _z(r):
    return np.array([0.0, 0.0, r])


def test_theta0_closed_form_along_z():
    """Along +z, n = (0, 0, 1): a = exp(-i theta0) and b = 0, so arg(a) gives
    theta0 at every r, including theta0 = 0 at r = rmin0 (a = 1 exactly)."""
    g = oracle.geometry(_z(RMIN), RC, RF, RMIN)
    assert g["a"] == 1.0 and g["b"] == 0.0
    for r in (3.0, 3.5, 4.0, 4.6):
        g = oracle.geometry(_z(r), RC, RF, RMIN)
        th0 = RF * np.pi * (r - RMIN) / (RC - RMIN)
        assert abs(-np.angle(g["a"]) - th0) < 1e-14, r
        assert abs(g["b"]) == 0.0
    # below rmin0 the map continues linearly to negative angles
    g = oracle.geometry(_z(2.0), RC, RF, RMIN)
    assert abs(-np.angle(g["a"]) - RF * np.pi * (2.0 - RMIN) / (RC - RMIN)) < 1e-14


def test_switching_plateau_below_rmin0():
    """f_c is exactly 1 with a zero gradient on and below rmin0; half way
    between rmin0 and rcut it is 1/2; it vanishes at rcut."""
    for r in (0.5, 1.7, RMIN * (1 - 1e-12), RMIN):
        g = oracle.geometry(_z(r), RC, RF, RMIN)
        assert g["fc"] == 1.0 and np.all(g["dfc"] == 0.0), r
    g = oracle.geometry(_z(0.5 * (RMIN + RC)), RC, RF, RMIN)
    assert abs(g["fc"] - 0.5) < 1e-15
    g = oracle.geometry(_z(RC * (1 - 1e-12)), RC, RF, RMIN)
    assert abs(g["fc"]) < 1e-20
    # just above rmin0 the cosine starts at 1 with a zero slope (C1 join)
    g = oracle.geometry(_z(RMIN * (1 + 1e-9)), RC, RF, RMIN)
    assert abs(g["fc"] - 1.0) < 1e-15 and np.abs(g["dfc"]).max() < 1e-8


@pytest.mark.parametrize("r", [RMIN - 1e-3, RMIN + 1e-3, 2.2, 3.6, 4.5])
def test_geometry_derivatives_across_rmin0(r):
    """Gradients of a, b and f_c against central differences on both sides of
    rmin0 (random directions)."""
    rng = np.random.default_rng(int(r * 1000))
    h = 1e-7
    for _ in range(4):
        n = rng.normal(size=3)
        rv = r * n / np.linalg.norm(n)
        g = oracle.geometry(rv, RC, RF, RMIN)
        for al in range(3):
            e = np.zeros(3)
            e[al] = h
            gp, gm = oracle.geometry(rv + e, RC, RF, RMIN), oracle.geometry(rv - e, RC, RF, RMIN)
            assert abs((gp["a"] - gm["a"]) / (2 * h) - g["da"][al]) < 1e-7
            assert abs((gp["b"] - gm["b"]) / (2 * h) - g["db"][al]) < 1e-7
            assert abs((gp["fc"] - gm["fc"]) / (2 * h) - g["dfc"][al]) < 1e-7


@pytest.mark.parametrize("tj", [4, 8])
def test_single_neighbour_inside_rmin0(tj):
    """w_self = 0, one neighbour at r < rmin0: f_c = 1, so the Clebsch-Gordan
    series and unitarity give B = (J + 1) exactly, independent of r."""
    tri = oracle.components(tj)
    beta = np.random.default_rng(1).normal(0, 0.1, len(tri))
    for r in (1.1, 2.5):
        pos = np.array([[0.0, 0.0, 0.0], r * np.array([0.36, -0.48, 0.8])])
        o = oracle.snap(pos, np.zeros(3), tj, RC, RF, RMIN, wself=0.0, beta=beta)
        assert np.allclose(o["B"][0], tri[:, 2] + 1.0, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("tj", [4, 6])
def test_forces_with_neighbours_on_both_sides_of_rmin0(tj):
    """Central differences (h = 1e-5 A) of the local energy in a BCC crystal
    whose first shell (2.754 A) lies inside rmin0 and the others outside."""
    pos, box = wl.bcc(3, 0.08, 31)
    beta = np.random.default_rng(2).normal(0, 0.1, len(oracle.components(tj)))
    full = oracle.snap(pos, box, tj, RC, RF, RMIN, beta=beta)
    off, nbr = full["off"], full["nbr"]
    k = 4
    rv = pos[nbr[off[k]:off[k + 1]]] - pos[k]
    rv -= box * np.round(rv / box)
    r = np.linalg.norm(rv, axis=1)
    assert (r < RMIN).sum() >= 4 and (r > RMIN).sum() >= 10
    centres = np.unique(np.concatenate([[k], nbr[off[k]:off[k + 1]]]))
    h = 1e-5

    def local(p):
        o = oracle.snap(p, box, tj, RC, RF, RMIN, beta=beta, centers=centres, want_dE=False)
        return o["E"][centres].sum()
    for al in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[k, al] += h
        pm[k, al] -= h
        fd = -(local(pp) - local(pm)) / (2 * h)
        # O(h^2) truncation relative to the force (forces reach hundreds of
        # eV/A here: the short span rcut - rmin0 makes theta0 steep)
        assert abs(fd - full["F"][k, al]) < 1e-7 + 2e-9 * abs(fd), (al, fd, full["F"][k, al])
    # the inner radius changes the answer (it is not silently ignored)
    o0 = oracle.snap(pos, box, tj, RC, RF, 0.0, beta=beta, want_dE=False)
    assert np.abs(o0["E"] - full["E"]).max() > 1e-3
