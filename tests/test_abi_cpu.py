"""Host-side checks of the C ABI: the library loads, exports what the header
declares, validates its arguments and builds correct tables and neighbour
lists.  Nothing here launches a kernel."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2011_12875_amd import snapmi
from paper_2011_12875_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(snapmi.LIB_PATH):
        from paper_2011_12875_amd import build
        build.build()
    return snapmi.load()


def test_header_symbols_are_exported():
    hdr = open(os.path.join(ROOT, "include", "snapmi.h")).read()
    declared = set(re.findall(r"^(?:int|long long|const char \*)\s*(snap_\w+)\s*\(", hdr, re.M))
    assert declared == set(snapmi.EXPORTS)
    lib = _lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_setup_validates_parameters():
    lib = _lib()
    ctx = ctypes.c_void_p()
    bad = [(-1, 4.73, 0.99, 0.0, 1), (15, 4.73, 0.99, 0.0, 1), (4, 0.0, 0.99, 0.0, 1),
           (4, 4.73, 0.0, 0.0, 1), (4, 4.73, 1.5, 0.0, 1), (4, 4.73, 0.99, 5.0, 1),
           (4, 4.73, 0.99, -0.1, 1), (4, 4.73, 0.99, 0.0, 2)]
    for args in bad:
        assert lib.snap_setup(*args, ctypes.byref(ctx)) == -1, args
        assert lib.snap_last_error()
    assert lib.snap_setup(8, 4.73, 0.99363, 0.0, 1, ctypes.byref(ctx)) == 0
    assert lib.snap_ncoeff(ctx) == 55
    assert lib.snap_nhalf(ctx) == 155
    assert lib.snap_destroy(ctx) == 0
    assert lib.snap_destroy(None) == 0
    assert lib.snap_ncoeff(None) == -1


def test_set_elements_validates():
    lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.snap_setup(4, 4.73, 0.99363, 0.0, 1, ctypes.byref(ctx)) == 0
    dp = ctypes.POINTER(ctypes.c_double)

    def call(rad, wt, f):
        r = np.ascontiguousarray(rad, dtype=np.float64)
        w = np.ascontiguousarray(wt, dtype=np.float64)
        return lib.snap_set_elements(ctx, len(r), r.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                     float(f))
    assert call([2.0, 2.3], [1.0, 0.5], 1.0) == 0
    assert call([2.4], [1.0], 0.98) == 0                 # 4.704 <= 4.73
    assert call([2.4], [1.0], 1.0) == -1                 # 4.8 > rcut
    assert call([2.0, 0.0], [1.0, 1.0], 1.0) == -1       # radius must be > 0
    assert call([2.0], [float("nan")], 1.0) == -1
    assert call([2.0], [1.0], 0.0) == -1
    assert call(np.full(65, 1.0), np.ones(65), 1.0) == -1
    assert lib.snap_set_elements(ctx, 0, None, None, 0.0) == 0   # back to one element
    assert lib.snap_destroy(ctx) == 0


@pytest.mark.parametrize("tj,nb,nh", [(0, 1, 1), (2, 5, 9), (4, 14, 32), (8, 55, 155),
                                      (14, 204, 652)])
def test_table_sizes(tj, nb, nh):
    p = snapmi.SnapPotential(tj, wl.RCUT)
    assert p.ncoeff == nb and p.nhalf == nh
    comps = p.table(0)
    assert np.array_equal(comps, oracle.components(tj))  # same enumeration order
    helem = p.table(1)
    assert len(helem) == nh
    for J, pp, q in helem:
        assert 0 <= pp <= J and 0 <= 2 * q <= J


def test_device_clebsch_gordan_matches_sympy():
    from sympy import Rational
    from sympy.physics.quantum.cg import CG
    p = snapmi.SnapPotential(6, wl.RCUT)
    vals, keys = p.table(2), p.table(3)
    h = lambda x: Rational(int(x), 2)
    worst = 0.0
    for (J1, J2, J, M1, M2), v in zip(keys, vals):
        ref = float(CG(h(J1), h(M1), h(J2), h(M2), h(J), h(M1 + M2)).doit())
        worst = max(worst, abs(ref - v))
    assert worst < 1e-14


def test_device_clebsch_gordan_large_sample():
    from sympy import Rational
    from sympy.physics.quantum.cg import CG
    p = snapmi.SnapPotential(14, wl.RCUT)
    vals, keys = p.table(2), p.table(3)
    h = lambda x: Rational(int(x), 2)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(keys), 150, replace=False):
        J1, J2, J, M1, M2 = keys[k]
        ref = float(CG(h(J1), h(M1), h(J2), h(M2), h(J), h(M1 + M2)).doit())
        assert abs(ref - vals[k]) < 1e-13


@pytest.mark.parametrize("name", ["bcc128_2j4", "bcc2000_2j8"])
def test_neighbor_builder_matches_brute_force(name):
    pos, box, _, _ = wl.make(name)
    off, nbr, rev = snapmi.build_neighbors(pos, box, wl.RCUT)
    ooff, onbr = oracle.neighbors(pos, box, wl.RCUT)
    assert np.array_equal(off, ooff)
    for i in range(len(pos)):
        assert set(nbr[off[i]:off[i + 1]]) == set(onbr[ooff[i]:ooff[i + 1]])
    snapmi.check_neighbors(off, nbr, rev)
    # reverse index joins the same two atoms
    pair_atom = np.repeat(np.arange(len(pos)), np.diff(off))
    assert np.array_equal(pair_atom[rev], nbr)
    assert np.array_equal(nbr[rev], pair_atom)


def test_neighbor_builder_uneven_and_open():
    pos, box = wl.bcc_with_vacancies(6, 40, 0.15, 1, 2)
    off, nbr, rev = snapmi.build_neighbors(pos, box, wl.RCUT)
    counts = np.diff(off)
    assert counts.min() < counts.max()
    ooff, _ = oracle.neighbors(pos, box, wl.RCUT)
    assert np.array_equal(off, ooff)
    snapmi.check_neighbors(off, nbr, rev)
    cpos, cbox = wl.cluster(20, 4.0, 3)
    off, nbr, rev = snapmi.build_neighbors(cpos, cbox, wl.RCUT)
    ooff, _ = oracle.neighbors(cpos, cbox, wl.RCUT)
    assert np.array_equal(off, ooff)
    snapmi.check_neighbors(off, nbr, rev)
    # a single atom and an empty system
    off, nbr, rev = snapmi.build_neighbors(np.zeros((1, 3)), np.zeros(3), wl.RCUT)
    assert off.tolist() == [0, 0] and len(nbr) == 0
    off, nbr, rev = snapmi.build_neighbors(np.zeros((0, 3)), np.zeros(3), wl.RCUT)
    assert off.tolist() == [0]


def test_neighbor_errors():
    pos, box = wl.bcc(2, 0.0, 0)  # 6.36 A box < 2 rcut
    with pytest.raises(snapmi.SnapError) as e:
        snapmi.build_neighbors(pos, box, wl.RCUT)
    assert e.value.code == -2
    bad = np.array([[0.0, 0.0, np.nan]])
    with pytest.raises(snapmi.SnapError) as e:
        snapmi.build_neighbors(bad, np.zeros(3), wl.RCUT)
    assert e.value.code == -4
    pos, box = wl.bcc(3, 0.05, 1)
    off, nbr, rev = snapmi.build_neighbors(pos, box, wl.RCUT)
    for mutate in ("self", "range", "rev"):
        o, n_, r = off.copy(), nbr.copy(), rev.copy()
        if mutate == "self":
            n_[0] = 0
        elif mutate == "range":
            n_[3] = len(pos) + 5
        else:
            r[[0, 1]] = r[[1, 0]]
        with pytest.raises(snapmi.SnapError) as e:
            snapmi.check_neighbors(o, n_, r)
        assert e.value.code == -3


def _same_lists(pos, box, rcut):
    off, nbr, rev = snapmi.build_neighbors(pos, box, rcut)
    ooff, onbr = oracle.neighbors(pos, box, rcut)
    assert np.array_equal(off, ooff)
    for i in range(len(pos)):
        assert set(nbr[off[i]:off[i + 1]]) == set(onbr[ooff[i]:ooff[i + 1]]), i
    snapmi.check_neighbors(off, nbr, rev)
    return off


def test_neighbor_builder_open_axis_wider_than_two_cutoffs():
    """On an open axis whose extent exceeds 2 rcut the cells must still be at
    least rcut wide: a pair in cells two apart would otherwise be lost."""
    pos = np.array([[0.0, 0.0, 0.0], [0.8, 0.0, 0.0], [1.7, 0.0, 0.0], [2.5, 0.0, 0.0]])
    off = _same_lists(pos, np.zeros(3), 1.0)
    assert off[-1] == 6   # (0,1), (1,2), (2,3) in both directions
    for seed in (0, 1, 2):
        cpos, cbox = wl.cluster(300, 9.0, seed)
        _same_lists(cpos, cbox, wl.RCUT)


@pytest.mark.parametrize("open_axes", [(2,), (0, 1)])
def test_neighbor_builder_partly_open_box(open_axes):
    """Slab and wire geometries: some axes periodic, the others open and
    several cut-offs long."""
    pos, box = wl.bcc((5, 4, 6), 0.1, 21, open_axes=open_axes)
    assert all(box[d] == 0.0 for d in open_axes)
    off = _same_lists(pos, box, wl.RCUT)
    counts = np.diff(off)
    assert counts.min() < 26 and counts.max() >= 24


def test_neighbor_builder_orthorhombic_box():
    pos, box = wl.bcc((4, 5, 7), 0.1, 22)
    assert len(set(box.tolist())) == 3
    _same_lists(pos, box, wl.RCUT)


@pytest.mark.parametrize("tj,limit", [(14, 8947840), (8, 14913024)])
def test_sizes_beyond_the_row_addressing_limit_are_rejected(tj, limit):
    """compute_Y addresses a row of U_J with 32-bit byte counts, so
    16 (2J + 1) npad must stay below 2^31: larger n is refused on the host,
    before any device work (no pointer is dereferenced)."""
    lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.snap_setup(tj, wl.RCUT, wl.RFAC0, 0.0, 1, ctypes.byref(ctx)) == 0
    assert 16 * (tj + 1) * limit < 2 ** 31 <= 16 * (tj + 1) * (limit + 64)
    dummy = ctypes.c_void_p(256)
    box = (ctypes.c_double * 3)(1e4, 1e4, 1e4)
    for fn in ("snap_compute", "snap_forward", "snap_backward"):
        f = getattr(lib, fn)
        args = {"snap_compute": (ctx, limit + 1, 0, dummy, box, dummy, dummy, dummy, dummy, 0,
                                 dummy, dummy, None, None, None),
                "snap_forward": (ctx, limit + 1, 0, dummy, box, dummy, dummy, dummy, dummy, 0,
                                 dummy, dummy, None),
                "snap_backward": (ctx, limit + 1, 0, dummy, box, dummy, dummy, dummy, dummy, 0,
                                  dummy, dummy, None, None)}[fn]
        assert f(*args) == -1, fn
        assert b"too large" in lib.snap_last_error(), fn
    assert lib.snap_destroy(ctx) == 0


def test_backward_without_forward_is_rejected():
    """snap_backward reuses the U of a forward call on the same context; with
    none it refuses on the host."""
    lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.snap_setup(4, wl.RCUT, wl.RFAC0, 0.0, 1, ctypes.byref(ctx)) == 0
    dummy = ctypes.c_void_p(256)
    box = (ctypes.c_double * 3)(100.0, 100.0, 100.0)
    assert lib.snap_backward(ctx, 10, 20, dummy, box, dummy, dummy, dummy, dummy, 0, dummy, dummy,
                             None, None) == -1
    assert b"snap_forward" in lib.snap_last_error()
    assert lib.snap_copy_workspace(ctx, 0, 10, dummy, None) == -1
    assert lib.snap_destroy(ctx) == 0
