"""Plain FP64 CPU oracle for SNAP energies and forces -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and it imports nothing from the
product path.

The arithmetic lives in ``snap_oracle.c`` (plain C99 + OpenMP), which follows
Sec. II.A of the paper: eq. (u) for the density expansion, eq. (z) for the
bispectrum, eq. (snapatomenergy) for the energy and eq. (snapforce1) with
eq. (dbidrk) for forces, by the literal product rule (no adjoint).  This
module builds that file with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_snap.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c99", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_cg.restype = ctypes.c_double
        lib.oracle_cg.argtypes = [ctypes.c_int] * 6
        lib.oracle_components.restype = ctypes.c_int
        lib.oracle_components.argtypes = [ctypes.c_int, ip]
        lib.oracle_wigner.restype = None
        lib.oracle_wigner.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
        lib.oracle_geometry.restype = None
        lib.oracle_geometry.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, dp]
        lib.oracle_neighbors.restype = ctypes.c_int
        lib.oracle_neighbors.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ip, ip, ctypes.c_int]
        lib.oracle_snap.restype = ctypes.c_int
        lib.oracle_snap.argtypes = [
            ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
            ip, ip, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.oracle_snap_elements.restype = ctypes.c_int
        lib.oracle_snap_elements.argtypes = [
            ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_double, ctypes.c_int, ip, dp, dp, ctypes.c_double, dp, ctypes.c_int,
            ip, ip, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.oracle_snap_list.restype = ctypes.c_int
        lib.oracle_snap_list.argtypes = [
            ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
            ip, ip, dp, dp, dp, dp]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def cg(J1: int, M1: int, J2: int, M2: int, J: int, M: int) -> float:
    """<j1 m1 j2 m2 | j m> with every argument doubled (Condon-Shortley)."""
    return _load().oracle_cg(J1, M1, J2, M2, J, M)


def components(twojmax: int) -> np.ndarray:
    """Canonical (J1, J2, J) triples in the oracle's order, shape [N_B, 3]."""
    lib = _load()
    n = lib.oracle_components(twojmax, None)
    out = np.zeros((n, 3), dtype=np.int32)
    lib.oracle_components(twojmax, _ip(out))
    return out


def wigner(J: int, a: complex, b: complex) -> np.ndarray:
    """Explicit u^J(a, b), shape [J+1, J+1] complex, row p, column q."""
    out = np.zeros(2 * (J + 1) ** 2)
    _load().oracle_wigner(J, a.real, a.imag, b.real, b.imag, _dp(out))
    return (out[0::2] + 1j * out[1::2]).reshape(J + 1, J + 1)


def geometry(rv, rcut, rfac0, rmin0, switch_flag=1):
    """Cayley-Klein a, b, their gradients, f_c and grad f_c of one vector."""
    rv = np.ascontiguousarray(rv, dtype=np.float64)
    out = np.zeros(20)
    _load().oracle_geometry(_dp(rv), rcut, rfac0, rmin0, int(switch_flag), _dp(out))
    a = out[0] + 1j * out[1]
    b = out[2] + 1j * out[3]
    da = np.array([out[4 + 4 * k] + 1j * out[5 + 4 * k] for k in range(3)])
    db = np.array([out[6 + 4 * k] + 1j * out[7 + 4 * k] for k in range(3)])
    return dict(a=a, b=b, da=da, db=db, fc=out[16], dfc=out[17:20].copy())


def neighbors(pos, box, rcut):
    """Brute-force minimum-image full neighbour list: (off[n+1], nbr[P])."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    n = pos.shape[0]
    cap = max(64, n * 64)
    while True:
        off = np.zeros(n + 1, dtype=np.int32)
        nbr = np.zeros(cap, dtype=np.int32)
        np_ = _load().oracle_neighbors(n, _dp(pos), _dp(box), rcut, _ip(off), _ip(nbr), cap)
        if np_ >= 0:
            return off, nbr[:np_].copy()
        cap *= 2


def ufull_offsets(twojmax: int):
    """Offsets of each full (J+1)x(J+1) block inside the oracle's Utot rows."""
    offs, o = [], 0
    for J in range(twojmax + 1):
        offs.append(o)
        o += (J + 1) ** 2
    return offs, o


def snap(pos, box, twojmax, rcut, rfac0=0.99363, rmin0=0.0, switch_flag=1, wself=1.0,
         beta=None, centers=None, nthreads=0, want_utot=False, want_dE=True):
    """Evaluate SNAP with the oracle.

    Returns a dict with ``E`` [n], ``F`` [n,3] (accumulated from the evaluated
    centres only), ``B`` [n,N_B], ``off``/``nbr`` (CSR full neighbour list),
    optionally ``U`` ([n, sum (J+1)^2] complex, full matrices) and ``dE``
    [P,3] (dE_i/dr_ik per pair; rows of unevaluated centres are zero).
    ``beta`` is [N_B] or [n, N_B] (per-atom coefficients).
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    n = pos.shape[0]
    nb = lib.oracle_components(twojmax, None)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    per_atom = 1 if beta.ndim == 2 else 0
    if per_atom:
        assert beta.shape == (n, nb)
    else:
        assert beta.shape == (nb,)
    off_nb, nbr_nb = neighbors(pos, box, rcut)
    cap = max(1, len(nbr_nb))
    off = np.zeros(n + 1, dtype=np.int32)
    nbr = np.zeros(cap, dtype=np.int32)
    cen = None
    ncen = 0
    if centers is not None:
        cen = np.ascontiguousarray(centers, dtype=np.int32)
        ncen = len(cen)
    E = np.zeros(n)
    F = np.zeros((n, 3))
    B = np.zeros((n, max(nb, 1)))
    _, ufull = ufull_offsets(twojmax)
    U = np.zeros((n, ufull, 2)) if want_utot else None
    dE = np.zeros((cap, 3)) if want_dE else None
    st = lib.oracle_snap(n, _dp(pos), _dp(box), twojmax, rcut, rfac0, rmin0, int(switch_flag),
                         wself, _dp(beta), per_atom, ncen, _ip(cen), int(nthreads), _ip(off),
                         _ip(nbr), cap, _dp(E), _dp(F), _dp(B), _dp(U), _dp(dE))
    if st < 0:
        raise RuntimeError("oracle_snap failed with status %d" % st)
    out = dict(E=E, F=F, B=B[:, :nb], off=off, nbr=nbr[:st].copy())
    if want_utot:
        out["U"] = U[..., 0] + 1j * U[..., 1]
    if want_dE:
        out["dE"] = dE[:st].copy()
    return out


def snap_elements(pos, box, twojmax, types, radius, weight, rcutfac, beta, rfac0=0.99363,
                  rmin0=0.0, switch_flag=1, wself=1.0, nthreads=0, want_utot=False):
    """Several elements: atom i has element types[i]; element e has radius
    radius[e] and density weight weight[e]; the pair (i, k) has the cutoff
    rcutfac (radius[t_i] + radius[t_k]) and enters U_i with weight[t_k];
    ``beta`` is [n_elements, N_B], the coefficients of the centre's element.
    The neighbour list (``off``/``nbr``) is searched to rcutfac * 2 max(radius)
    and keeps the pairs beyond their own cutoff (their ``dE`` rows are zero).
    Returns the same dict as :func:`snap`."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    types = np.ascontiguousarray(types, dtype=np.int32)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    n = pos.shape[0]
    nb = lib.oracle_components(twojmax, None)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    assert beta.shape == (len(radius), nb) and weight.shape == radius.shape and types.shape == (n,)
    _, nbr_nb = neighbors(pos, box, 2.0 * rcutfac * float(radius.max()))
    cap = max(1, len(nbr_nb))
    off = np.zeros(n + 1, dtype=np.int32)
    nbr = np.zeros(cap, dtype=np.int32)
    E = np.zeros(n)
    F = np.zeros((n, 3))
    B = np.zeros((n, max(nb, 1)))
    _, ufull = ufull_offsets(twojmax)
    U = np.zeros((n, ufull, 2)) if want_utot else None
    dE = np.zeros((cap, 3))
    st = lib.oracle_snap_elements(n, _dp(pos), _dp(box), twojmax, rfac0, rmin0, int(switch_flag),
                                  wself, len(radius), _ip(types), _dp(radius), _dp(weight),
                                  float(rcutfac), _dp(beta), int(nthreads), _ip(off), _ip(nbr),
                                  cap, _dp(E), _dp(F), _dp(B), _dp(U), _dp(dE))
    if st < 0:
        raise RuntimeError("oracle_snap_elements failed with status %d" % st)
    out = dict(E=E, F=F, B=B[:, :nb], off=off, nbr=nbr[:st].copy(), dE=dE[:st].copy())
    if want_utot:
        out["U"] = U[..., 0] + 1j * U[..., 1]
    return out


def snap_on_list(pos, box, twojmax, rcut, off, nbr, beta, rfac0=0.99363, rmin0=0.0,
                 switch_flag=1, wself=1.0, centers=None, nthreads=0):
    """:func:`snap` on a neighbour list from :func:`neighbors` (same rcut),
    so that the evaluation is timed without the brute-force search.  Returns
    E, F, B (no dE)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr if len(nbr) else np.zeros(1), dtype=np.int32)
    n = pos.shape[0]
    nb = lib.oracle_components(twojmax, None)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    per_atom = 1 if beta.ndim == 2 else 0
    cen = None if centers is None else np.ascontiguousarray(centers, dtype=np.int32)
    E = np.zeros(n)
    F = np.zeros((n, 3))
    B = np.zeros((n, max(nb, 1)))
    st = lib.oracle_snap_list(n, _dp(pos), _dp(box), twojmax, rcut, rfac0, rmin0,
                              int(switch_flag), wself, _dp(beta), per_atom,
                              0 if cen is None else len(cen), _ip(cen), int(nthreads), _ip(off),
                              _ip(nbr), _dp(E), _dp(F), _dp(B), None)
    if st < 0:
        raise RuntimeError("oracle_snap_list failed with status %d" % st)
    return dict(E=E, F=F, B=B[:, :nb])


def snap_quadratic(pos, box, twojmax, rcut, beta, alpha, rfac0=0.99363, rmin0=0.0,
                   switch_flag=1, wself=1.0, nthreads=0):
    """Quadratic SNAP: E_i = beta . B_i + (1/2) B_i^T alpha B_i, the quadratic
    extension of eq. (snapatomenergy) in the bispectrum (Sec. II.A writes the
    energy as a function of B_i; this is its second-order form).

    By the chain rule dE_i/dr = g_i . dB_i/dr with g_i = dE_i/dB_i =
    beta + (1/2)(alpha + alpha^T) B_i, so the forces and pair derivatives are
    those of the oracle's literal dB/dr route with the per-atom coefficients
    g_i.  Returns the dict of :func:`snap` with E replaced by the quadratic
    energy and ``G`` = g_i [n, N_B]."""
    beta = np.asarray(beta, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    nb = len(beta)
    assert alpha.shape == (nb, nb)
    kw = dict(rfac0=rfac0, rmin0=rmin0, switch_flag=switch_flag, wself=wself, nthreads=nthreads)
    B = snap(pos, box, twojmax, rcut, beta=beta, want_dE=False, **kw)["B"]
    E = B @ beta + 0.5 * np.einsum("il,lm,im->i", B, alpha, B)
    G = beta[None, :] + B @ (0.5 * (alpha + alpha.T)).T
    out = snap(pos, box, twojmax, rcut, beta=np.ascontiguousarray(G), **kw)
    out["E"] = E
    out["G"] = G
    return out


def max_threads() -> int:
    return _load().oracle_max_threads()


def virial(pos, box, off, nbr, dE):
    """dE_total/d(strain) = sum over pairs p = (i -> k) of dE_p (x) r_ik, a
    3x3 matrix W[a][b] = sum_p dE_p[a] r_ik[b] (r_ik by minimum image), and
    the per-atom shares W_i (pairs of atom i).  Under r -> (I + eps) r the
    energy changes by sum_ab W[a][b] eps[a][b] to first order."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    W_atom = np.zeros((n, 3, 3))
    for i in range(n):
        for p in range(off[i], off[i + 1]):
            k = int(nbr[p])
            r = pos[k] - pos[i]
            for d in range(3):
                if box[d] > 0.0:
                    r[d] -= box[d] * np.round(r[d] / box[d])
            W_atom[i] += np.outer(dE[p], r)
    return W_atom.sum(0), W_atom
