"""Thin Python binding of libsnapmi.so (the C ABI declared in include/snapmi.h).

Argument marshalling only: every stage of the evaluation runs in the HIP
kernels of the library.  Device buffers are torch tensors on the current
HIP device and work is enqueued on torch's current stream.  The library must
have been built (``python -m paper_2011_12875_amd.build``); there is no
fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnapmi.so")

SNAP_OK = 0
ERRORS = {-1: "SNAP_EINVAL", -2: "SNAP_EBOX", -3: "SNAP_ENBR", -4: "SNAP_EGEOM",
          -5: "SNAP_ENOMEM", -6: "SNAP_EDEV"}

# every symbol include/snapmi.h declares
EXPORTS = ["snap_setup", "snap_setup_ex", "snap_destroy", "snap_ncoeff", "snap_nhalf",
           "snap_table", "snap_build_neighbors", "snap_check_neighbors", "snap_compute",
           "snap_compute_noalloc",
           "snap_forward", "snap_backward", "snap_copy_workspace", "snap_profile",
           "snap_stage_times", "snap_sync_status", "snap_last_error",
           "snap_mlp_nparams", "snap_mlp_workspace", "snap_mlp_forward", "snap_mlp_grad",
           "snap_adam_step", "snap_jacobian", "snap_jacobian_forces", "snap_jacobian_adjoint",
           "snap_fit_residuals", "snap_virial", "snap_set_elements", "snap_compute_elements",
           "snap_beta_grad", "snap_compute_quadratic"]


class SnapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class snap_params(ctypes.Structure):
    _fields_ = [("twojmax", ctypes.c_int), ("rcut", ctypes.c_double), ("rfac0", ctypes.c_double),
                ("rmin0", ctypes.c_double), ("switch_flag", ctypes.c_int),
                ("wself", ctypes.c_double), ("dedr_dirs", ctypes.c_int),
                ("y_kernel", ctypes.c_int), ("dedr_kernel", ctypes.c_int),
                ("dedr_waves", ctypes.c_int), ("u_kernel", ctypes.c_int)]


_lib = None


def load():
    """Load libsnapmi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsnapmi.so is not built: run python -m paper_2011_12875_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    i, d, f = ctypes.c_int, ctypes.c_double, ctypes.c_float
    sig = {
        "snap_setup": (i, [i, d, d, d, i, ctypes.POINTER(vp)]),
        "snap_setup_ex": (i, [ctypes.POINTER(snap_params), ctypes.POINTER(vp)]),
        "snap_destroy": (i, [vp]),
        "snap_ncoeff": (i, [vp]),
        "snap_nhalf": (i, [vp]),
        "snap_table": (i, [vp, i, vp, i]),
        "snap_build_neighbors": (i, [dp, i, dp, d, ip, ip, ip, i, ip]),
        "snap_check_neighbors": (i, [i, ip, ip, ip, i]),
        "snap_compute": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, i, vp, vp, vp, vp, vp]),
        "snap_compute_noalloc": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, i, vp, vp, vp, vp, vp]),
        "snap_set_elements": (i, [vp, i, dp, dp, d]),
        "snap_compute_elements": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "snap_forward": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, i, vp, vp, vp]),
        "snap_backward": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, i, vp, vp, vp, vp]),
        "snap_copy_workspace": (i, [vp, i, i, vp, vp]),
        "snap_beta_grad": (i, [vp, i, vp, vp, i, vp, vp]),
        "snap_compute_quadratic": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                       vp]),
        "snap_sync_status": (i, [vp, vp]),
        "snap_profile": (i, [vp, i]),
        "snap_stage_times": (i, [vp, dp, ip]),
        "snap_last_error": (ctypes.c_char_p, []),
        "snap_mlp_nparams": (i, [i]),
        "snap_mlp_workspace": (ctypes.c_longlong, [i, i]),
        "snap_mlp_forward": (i, [i, i, vp, vp, vp, f, vp, vp, vp, vp, vp, vp]),
        "snap_mlp_grad": (i, [i, i, vp, vp, vp, vp, vp, vp, vp, vp]),
        "snap_adam_step": (i, [i, vp, vp, vp, vp, f, f, f, f, i, vp]),
        "snap_jacobian": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, vp, vp]),
        "snap_jacobian_forces": (i, [i, i, i, vp, vp, vp, vp, vp, vp, vp]),
        "snap_jacobian_adjoint": (i, [i, i, i, vp, vp, vp, vp, vp, vp]),
        "snap_fit_residuals": (i, [i, vp, vp, vp, vp, d, d, vp, vp, vp, vp]),
        "snap_virial": (i, [vp, i, i, vp, dp, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != SNAP_OK:
        raise SnapError(code, load().snap_last_error().decode())
    return code


def _np_dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _np_ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def build_neighbors(pos, box, rcut):
    """Host cell-list full neighbour list: (off[n+1], nbr[P], rev[P]) int32."""
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    n = pos.shape[0]
    cap = max(16, 40 * n)
    while True:
        off = np.zeros(n + 1, dtype=np.int32)
        nbr = np.zeros(cap, dtype=np.int32)
        rev = np.zeros(cap, dtype=np.int32)
        npairs = ctypes.c_int(0)
        st = lib.snap_build_neighbors(_np_dp(pos), n, _np_dp(box), float(rcut), _np_ip(off),
                                      _np_ip(nbr), _np_ip(rev), cap, ctypes.byref(npairs))
        if st == -5 and npairs.value > cap:
            cap = npairs.value
            continue
        _check(st)
        P = npairs.value
        return off, nbr[:P].copy(), rev[:P].copy()


def check_neighbors(off, nbr, rev):
    off = np.ascontiguousarray(off, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    rev = np.ascontiguousarray(rev, dtype=np.int32)
    return _check(load().snap_check_neighbors(len(off) - 1, _np_ip(off), _np_ip(nbr), _np_ip(rev),
                                              len(nbr)))


class NeighborList:
    """CSR full neighbour list resident on the device (torch int32 tensors)."""

    def __init__(self, off, nbr, rev, device="cuda"):
        import torch
        self.n = len(off) - 1
        self.npairs = len(nbr)
        self.off = torch.as_tensor(np.asarray(off, dtype=np.int32), device=device)
        self.nbr = torch.as_tensor(np.asarray(nbr, dtype=np.int32), device=device)
        self.rev = torch.as_tensor(np.asarray(rev, dtype=np.int32), device=device)
        if self.npairs == 0:  # keep valid pointers
            self.nbr = torch.zeros(1, dtype=torch.int32, device=device)
            self.rev = torch.zeros(1, dtype=torch.int32, device=device)

    @classmethod
    def build(cls, pos, box, rcut, device="cuda"):
        off, nbr, rev = build_neighbors(pos, box, rcut)
        return cls(off, nbr, rev, device)


class SnapPotential:
    """One parameter set of the potential (a library context)."""

    def __init__(self, twojmax, rcut, rfac0=0.99363, rmin0=0.0, switch_flag=1, wself=1.0,
                 dedr_dirs=0, y_kernel=0, dedr_kernel=0, dedr_waves=0, u_kernel=0):
        lib = load()
        p = snap_params(int(twojmax), float(rcut), float(rfac0), float(rmin0), int(switch_flag),
                        float(wself), int(dedr_dirs), int(y_kernel), int(dedr_kernel),
                        int(dedr_waves), int(u_kernel))
        ctx = ctypes.c_void_p()
        _check(lib.snap_setup_ex(ctypes.byref(p), ctypes.byref(ctx)))
        self._ctx = ctx
        self.twojmax = int(twojmax)
        self.rcut = float(rcut)
        self.ncoeff = lib.snap_ncoeff(ctx)
        self.nhalf = lib.snap_nhalf(ctx)
        # counts snap_forward calls: backward() uses the U of the last one
        self._fwd_token = 0

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and _lib is not None:
            _lib.snap_destroy(ctx)
            self._ctx = None

    # -- tables ------------------------------------------------------------
    def table(self, which):
        lib = load()
        n = lib.snap_table(self._ctx, which, None, 0)
        _check(0 if n >= 0 else n)
        dtype = np.float64 if which == 2 else np.int32
        buf = np.zeros(max(n, 1), dtype=dtype)
        lib.snap_table(self._ctx, which, buf.ctypes.data_as(ctypes.c_void_p), n)
        buf = buf[:n]
        if which in (0, 1):
            return buf.reshape(-1, 3)
        if which == 3:
            return buf.reshape(-1, 5)
        return buf

    def program_size(self):
        """compute_Y work per atom: (Clebsch-Gordan products, partial sums,
        contributions, rows)."""
        return tuple(int(x) for x in self.table(4))

    STAGES = ("compute_U", "compute_Y", "compute_dE", "update_forces", "bispectrum")

    def profile(self, enable=True):
        _check(load().snap_profile(self._ctx, 1 if enable else 0))

    def stage_times(self):
        """{stage: (summed ms, launches)} since the last call (waits for them)."""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int * 5)()
        _check(load().snap_stage_times(self._ctx, ms, cnt))
        return {self.STAGES[k]: (ms[k], cnt[k]) for k in range(5)}

    # -- evaluation ----------------------------------------------------------
    @staticmethod
    def _stream():
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    def _args(self, pos, box, nl, beta):
        import torch
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        assert beta.dtype == torch.float64 and beta.is_cuda and beta.is_contiguous()
        n = pos.shape[0]
        assert nl.n == n
        per_atom = 1 if beta.dim() == 2 else 0
        if per_atom:
            assert beta.shape == (n, self.ncoeff)
        else:
            assert beta.shape == (self.ncoeff,)
        boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
        return n, boxa, per_atom

    def compute(self, pos, box, nl, beta, bispectrum=False, pair_derivs=False, out=None):
        """E_i and F_i (and optionally B_i and dE per pair), as torch tensors."""
        import torch
        n, boxa, per_atom = self._args(pos, box, nl, beta)
        dev = pos.device
        if out is None:
            out = {}
            out["energy"] = torch.empty(n, dtype=torch.float64, device=dev)
            out["force"] = torch.empty((n, 3), dtype=torch.float64, device=dev)
            if bispectrum:
                out["bispectrum"] = torch.empty((n, self.ncoeff), dtype=torch.float64, device=dev)
            if pair_derivs:
                out["dE"] = torch.empty((max(nl.npairs, 1), 3), dtype=torch.float64, device=dev)
        _check(load().snap_compute(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(beta), per_atom, self._ptr(out["energy"]),
            self._ptr(out["force"]), self._ptr(out.get("bispectrum")), self._ptr(out.get("dE")),
            self._stream()))
        self._fwd_token += 1  # U of this call replaces that of the last forward
        return out

    def compute_noalloc(self, pos, box, nl, beta, out, bispectrum=False, pair_derivs=False):
        """As compute(), through snap_compute_noalloc: the library allocates no
        device memory (its workspace is a static array).  The caller passes
        the output tensors (out["energy"], out["force"], and out["bispectrum"]
        / out["dE"] when asked for)."""
        n, boxa, per_atom = self._args(pos, box, nl, beta)
        _check(load().snap_compute_noalloc(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(beta), per_atom, self._ptr(out["energy"]),
            self._ptr(out["force"]), self._ptr(out["bispectrum"] if bispectrum else None),
            self._ptr(out["dE"] if pair_derivs else None), self._stream()))
        return out

    def compute_quadratic(self, pos, box, nl, beta, alpha, bispectrum=False, pair_derivs=False,
                          out=None):
        """Quadratic SNAP, E_i = beta . B_i + B_i^T alpha B_i / 2: E_i and F_i
        (optionally B_i and dE per pair).  beta [N_B], alpha [N_B, N_B]."""
        import torch
        n, boxa, per_atom = self._args(pos, box, nl, beta)
        assert not per_atom
        assert alpha.dtype == torch.float64 and alpha.is_cuda and alpha.is_contiguous()
        assert tuple(alpha.shape) == (self.ncoeff, self.ncoeff)
        dev = pos.device
        if out is None:
            out = {"energy": torch.empty(n, dtype=torch.float64, device=dev),
                   "force": torch.empty((n, 3), dtype=torch.float64, device=dev)}
            if bispectrum:
                out["bispectrum"] = torch.empty((n, self.ncoeff), dtype=torch.float64, device=dev)
            if pair_derivs:
                out["dE"] = torch.empty((max(nl.npairs, 1), 3), dtype=torch.float64, device=dev)
        _check(load().snap_compute_quadratic(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(beta), self._ptr(alpha), self._ptr(out["energy"]),
            self._ptr(out["force"]), self._ptr(out.get("bispectrum")), self._ptr(out.get("dE")),
            self._stream()))
        self._fwd_token += 1
        return out

    def set_elements(self, radius, weight, rcutfac):
        """Several elements: radius and density weight per element and the
        pair cutoff factor (pair cutoff rcutfac (R_t_i + R_t_k) <= rcut)."""
        radius = np.ascontiguousarray(radius, dtype=np.float64)
        weight = np.ascontiguousarray(weight, dtype=np.float64)
        assert radius.ndim == 1 and weight.shape == radius.shape
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().snap_set_elements(self._ctx, len(radius), radius.ctypes.data_as(dp),
                                        weight.ctypes.data_as(dp), float(rcutfac)))
        self.nelem = len(radius)

    def compute_elements(self, pos, box, nl, types, beta, bispectrum=False, pair_derivs=False,
                         out=None):
        """compute() for several elements: types [n] int32 on the device,
        beta [nelem, N_B] float64 on the device (coefficients per element)."""
        import torch
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        n = pos.shape[0]
        assert nl.n == n
        assert types.dtype == torch.int32 and types.is_cuda and types.shape == (n,)
        assert types.is_contiguous()
        assert beta.dtype == torch.float64 and beta.is_cuda and beta.is_contiguous()
        assert beta.shape == (getattr(self, "nelem", 0), self.ncoeff)
        boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
        dev = pos.device
        if out is None:
            out = {"energy": torch.empty(n, dtype=torch.float64, device=dev),
                   "force": torch.empty((n, 3), dtype=torch.float64, device=dev)}
            if bispectrum:
                out["bispectrum"] = torch.empty((n, self.ncoeff), dtype=torch.float64, device=dev)
            if pair_derivs:
                out["dE"] = torch.empty((max(nl.npairs, 1), 3), dtype=torch.float64, device=dev)
        _check(load().snap_compute_elements(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(types), self._ptr(beta), self._ptr(out["energy"]),
            self._ptr(out["force"]), self._ptr(out.get("bispectrum")), self._ptr(out.get("dE")),
            self._stream()))
        self._fwd_token += 1
        return out

    def forward(self, pos, box, nl, beta, bispectrum=None):
        """compute_U + bispectrum: (E_i, B_i); keeps U for backward().  With
        beta None only B_i is computed (E is None)."""
        import torch
        if beta is None:
            assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
            n = pos.shape[0]
            assert nl.n == n
            boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
            per_atom, E = 0, None
        else:
            n, boxa, per_atom = self._args(pos, box, nl, beta)
            E = torch.empty(n, dtype=torch.float64, device=pos.device)
        B = bispectrum if bispectrum is not None else torch.empty(
            (n, self.ncoeff), dtype=torch.float64, device=pos.device)
        _check(load().snap_forward(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(beta), per_atom, self._ptr(E), self._ptr(B),
            self._stream()))
        self._fwd_token += 1
        return E, B

    def backward(self, pos, box, nl, beta, grad_energy, force=None):
        """-d(sum_i g_i E_i)/dr (the forces of the weighted energy)."""
        import torch
        n, boxa, per_atom = self._args(pos, box, nl, beta)
        g = grad_energy.contiguous()
        assert g.dtype == torch.float64 and g.shape == (n,)
        F = force if force is not None else torch.empty((n, 3), dtype=torch.float64,
                                                        device=pos.device)
        _check(load().snap_backward(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(beta), per_atom, self._ptr(g), self._ptr(F), None,
            self._stream()))
        return F

    def jacobian(self, pos, box, nl, bispectrum=None, jac=None):
        """B_i [n, N_B] (float64) and J_p = dB_i/dr_ik [P, N_B, 3] (float32)."""
        import torch
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        n = pos.shape[0]
        assert nl.n == n
        boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
        if bispectrum is None:
            bispectrum = torch.empty((n, self.ncoeff), dtype=torch.float64, device=pos.device)
        if jac is None:
            jac = torch.empty((max(nl.npairs, 1), self.ncoeff, 3), dtype=torch.float32,
                              device=pos.device)
        _check(load().snap_jacobian(
            self._ctx, n, nl.npairs, self._ptr(pos), boxa, self._ptr(nl.off), self._ptr(nl.nbr),
            self._ptr(nl.rev), self._ptr(bispectrum), self._ptr(jac), self._stream()))
        self._fwd_token += 1
        return bispectrum, jac

    def virial(self, pos, box, nl, dE, per_atom=False):
        """W[a][b] = sum_p dE_p[a] r_ik[b] (3x3) from the pair derivatives of
        compute(..., pair_derivs=True); with per_atom also W_i [n, 3, 3]."""
        import torch
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        n = pos.shape[0]
        assert nl.n == n and dE.dtype == torch.float64 and dE.is_contiguous()
        boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
        W = torch.empty(9, dtype=torch.float64, device=pos.device)
        Wa = torch.empty((n, 9), dtype=torch.float64, device=pos.device) if per_atom else None
        _check(load().snap_virial(self._ctx, n, nl.npairs, self._ptr(pos), boxa,
                                  self._ptr(nl.off), self._ptr(nl.nbr), self._ptr(dE),
                                  self._ptr(Wa), self._ptr(W), self._stream()))
        W = W.reshape(3, 3)
        return (W, Wa.reshape(n, 3, 3)) if per_atom else W

    def workspace(self, which, n):
        """True U_j (which=0) or Y_j (which=1) of the last call: [nhalf, n]
        complex; n must be that call's atom count (the library checks)."""
        import torch
        dst = torch.empty((self.nhalf, max(int(n), 1), 2), dtype=torch.float64, device="cuda")
        _check(load().snap_copy_workspace(self._ctx, which, int(n), self._ptr(dst),
                                          self._stream()))
        return torch.view_as_complex(dst[:, :n])

    def beta_grad(self, grad_energy, bispectrum, per_atom=False):
        """d(sum_i g_i E_i)/dbeta: sum_i g_i B_i [N_B], or g_i B_i [n, N_B]."""
        import torch
        g = grad_energy.contiguous()
        n = g.shape[0]
        assert g.dtype == torch.float64 and g.is_cuda and g.dim() == 1
        assert bispectrum.dtype == torch.float64 and bispectrum.is_contiguous()
        assert tuple(bispectrum.shape) == (n, self.ncoeff)
        shape = (n, self.ncoeff) if per_atom else (self.ncoeff,)
        out = torch.empty(shape, dtype=torch.float64, device=g.device)
        _check(load().snap_beta_grad(self._ctx, n, self._ptr(g), self._ptr(bispectrum),
                                     1 if per_atom else 0, self._ptr(out), self._stream()))
        return out

    def sync_status(self):
        return _check(load().snap_sync_status(self._ctx, self._stream()))


# ---------------------------------------------------------------------------
# learned surrogate: network, optimiser and descriptor-Jacobian kernels
# ---------------------------------------------------------------------------
def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape=None):
    import torch
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.dtype, t.device)
    if shape is not None:
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
    return t


def mlp_nparams(nin):
    n = load().snap_mlp_nparams(int(nin))
    _check(0 if n >= 0 else n)
    return n


def mlp_workspace(nin, n):
    k = load().snap_mlp_workspace(int(nin), int(n))
    _check(0 if k >= 0 else int(k))
    return int(k)


def mlp_forward(params, norm, bispec, bounds=None, margin=0.0, flag=None, energy=None,
                grad_b=None, clear_flag=None):
    """(E_i, g_i = dE_i/dB_i) of the network; sets flag[0] = 1 on inputs
    outside the bounds widened by margin, and clear_flag[0] = 0."""
    import torch
    n, nin = bispec.shape
    _dev(params, torch.float32, (mlp_nparams(nin),))
    _dev(norm, torch.float32, (2, nin))
    _dev(bispec, torch.float64)
    if bounds is not None:
        _dev(bounds, torch.float32, (2, nin))
    if flag is not None:
        _dev(flag, torch.int32)
    if clear_flag is not None:
        _dev(clear_flag, torch.int32)
    E = energy if energy is not None else torch.empty(n, dtype=torch.float64, device=bispec.device)
    g = grad_b if grad_b is not None else torch.empty((n, nin), dtype=torch.float64,
                                                      device=bispec.device)
    _check(load().snap_mlp_forward(nin, n, _p(params), _p(norm), _p(bounds), float(margin),
                                   _p(bispec), _p(E), _p(g), _p(flag), _p(clear_flag),
                                   _stream()))
    return E, g


def mlp_grad(params, norm, bispec, dl_de, dl_dg=None, work=None, grad=None):
    """d/dtheta of sum_i dl_de_i E_i + dl_dg_i . g_i (float32 [nparams])."""
    import torch
    n, nin = bispec.shape
    np_ = mlp_nparams(nin)
    _dev(params, torch.float32, (np_,))
    _dev(norm, torch.float32, (2, nin))
    _dev(bispec, torch.float64)
    _dev(dl_de, torch.float64, (n,))
    if dl_dg is not None:
        _dev(dl_dg, torch.float64, (n, nin))
    need = mlp_workspace(nin, n)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.float32, device=bispec.device)
    assert work.numel() >= need
    if grad is None:
        grad = torch.empty(np_, dtype=torch.float32, device=bispec.device)
    _check(load().snap_mlp_grad(nin, n, _p(params), _p(norm), _p(bispec), _p(dl_de), _p(dl_dg),
                                _p(work), _p(grad), _stream()))
    return grad


def adam_step(params, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    import torch
    np_ = params.numel()
    for t in (params, m, v, grad):
        _dev(t, torch.float32, (np_,))
    _check(load().snap_adam_step(np_, _p(params), _p(m), _p(v), _p(grad), float(lr), float(beta1),
                                 float(beta2), float(eps), int(step), _stream()))


def jacobian_forces(nl, jac, grad_b, dE=None, force=None):
    """Forces of per-atom energies with input gradients grad_b, from J_p."""
    import torch
    n, nin = grad_b.shape
    assert nl.n == n
    _dev(grad_b, torch.float64)
    _dev(jac, torch.float32)
    assert jac.shape[0] >= nl.npairs and jac.shape[1:] == (nin, 3)
    if dE is None:
        dE = torch.empty((max(nl.npairs, 1), 3), dtype=torch.float64, device=grad_b.device)
    if force is None:
        force = torch.empty((n, 3), dtype=torch.float64, device=grad_b.device)
    _check(load().snap_jacobian_forces(nin, n, nl.npairs, _p(nl.off), _p(nl.rev), _p(jac),
                                       _p(grad_b), _p(dE), _p(force), _stream()))
    return force


def jacobian_adjoint(nl, jac, dl_dforce, nin, out=None):
    """dl_dg_i = sum_{p = (i -> k)} J_p (dl_dforce_i - dl_dforce_k)."""
    import torch
    n = nl.n
    _dev(dl_dforce, torch.float64, (n, 3))
    _dev(jac, torch.float32)
    assert jac.shape[0] >= nl.npairs and jac.shape[1:] == (nin, 3)
    if out is None:
        out = torch.empty((n, nin), dtype=torch.float64, device=dl_dforce.device)
    _check(load().snap_jacobian_adjoint(nin, n, nl.npairs, _p(nl.off), _p(nl.nbr), _p(jac),
                                        _p(dl_dforce), _p(out), _stream()))
    return out


def fit_residuals(energy, energy_ref, force, force_ref, w_energy, w_force, dl_de=None,
                  dl_dforce=None, sums=None):
    """(dl_de, dl_dforce, sums[nblk, 2]) of the weighted squared-error loss."""
    import torch
    n = energy.shape[0]
    for t, shp in ((energy, (n,)), (energy_ref, (n,)), (force, (n, 3)), (force_ref, (n, 3))):
        _dev(t, torch.float64, shp)
    dev = energy.device
    if dl_de is None:
        dl_de = torch.empty(n, dtype=torch.float64, device=dev)
    if dl_dforce is None:
        dl_dforce = torch.empty((n, 3), dtype=torch.float64, device=dev)
    if sums is None:
        sums = torch.empty((max((n + 255) // 256, 1), 2), dtype=torch.float64, device=dev)
    _check(load().snap_fit_residuals(n, _p(energy), _p(energy_ref), _p(force), _p(force_ref),
                                     float(w_energy), float(w_force), _p(dl_de), _p(dl_dforce),
                                     _p(sums), _stream()))
    return dl_de, dl_dforce, sums
