"""Thin Python binding of libdgmg.so (include/dgmg.h): argument marshalling
only.  Vectors are torch tensors on the GPU (float64, or float32 for the
*_f32 entry points), contiguous, shaped (ndofs,) or (nrhs, ndofs) in the
cell-wise lexicographic layout; every call is enqueued on torch's current
stream.  There is no fallback: if the library is missing or the device is not
a GPU the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmg.so")

FP64, FP32 = 64, 32
SMOOTH_EXACT, SMOOTH_LOCAL, SMOOTH_FULL, SMOOTH_CLAMPED = 0, 1, 2, 3

STATUS = {
    0: "DGMG_OK", -1: "DGMG_ERR_ARG", -2: "DGMG_ERR_ALLOC", -3: "DGMG_ERR_HIP",
    -4: "DGMG_ERR_NOT_CONVERGED", -5: "DGMG_ERR_BREAKDOWN", -6: "DGMG_ERR_STATE",
}

# name -> (restype, argtypes); mirrors include/dgmg.h
_c = ctypes
_P, _I, _D, _LL = _c.c_void_p, _c.c_int, _c.c_double, _c.c_longlong
SIGNATURES = {
    "dgmg_setup_mesh": (_I, [_I, _I, _I, _D, _D, _c.POINTER(_P)]),
    "dgmg_setup_levels": (_I, [_P, _I, _I, _I, _P]),
    "dgmg_set_stream": (_I, [_P, _P]),
    "dgmg_set_kappa": (_I, [_P, _D]),
    "dgmg_use_graphs": (_I, [_P, _I]),
    "dgmg_use_dense_bottom": (_I, [_P, _I]),
    "dgmg_dense_bottom_level": (_I, [_P]),
    "dgmg_level_ndofs": (_LL, [_P, _I]),
    "dgmg_level_cells": (_I, [_P, _I]),
    "dgmg_finest_level": (_I, [_P]),
    "dgmg_node_coords": (_I, [_P, _I, _P]),
    "dgmg_apply_sipg": (_I, [_P, _I, _P, _P, _I]),
    "dgmg_apply_sipg_f32": (_I, [_P, _I, _P, _P, _I]),
    "dgmg_apply_mass": (_I, [_P, _I, _P, _P, _I]),
    "dgmg_smooth_patch": (_I, [_P, _I, _P, _P, _I, _I]),
    "dgmg_smooth_patch_f32": (_I, [_P, _I, _P, _P, _I, _I]),
    "dgmg_restrict_residual": (_I, [_P, _I, _P, _P, _P, _I]),
    "dgmg_restrict_residual_f32": (_I, [_P, _I, _P, _P, _P, _I]),
    "dgmg_prolongate_add": (_I, [_P, _I, _P, _P, _I]),
    "dgmg_prolongate_add_f32": (_I, [_P, _I, _P, _P, _I]),
    "dgmg_coarse_solve": (_I, [_P, _P, _P, _I]),
    "dgmg_coarse_solve_f32": (_I, [_P, _P, _P, _I]),
    "dgmg_vcycle": (_I, [_P, _P, _P, _I]),
    "dgmg_vcycle_f32": (_I, [_P, _P, _P, _I]),
    "dgmg_vcycle_noalloc": (_I, [_P, _P, _P, _I]),
    "dgmg_pcg_solve": (_I, [_P, _P, _P, _I, _D, _I, _I, _P, _P]),
    "dgmg_gmres_solve": (_I, [_P, _P, _P, _D, _I, _P, _P]),
    "dgmg_dot": (_I, [_P, _I, _P, _P, _I, _P]),
    "dgmg_adjoint_dkappa": (_I, [_P, _P, _P, _I, _P, _P]),
    "dgmg_autotune": (_I, [_P, _I, _c.c_char_p, _P, _I]),
    "dgmg_patch_eigen": (_I, [_I, _D, _I, _I, _P, _P]),
    "dgmg_last_error": (_c.c_char_p, [_P]),
    "dgmg_destroy": (_I, [_P]),
}

_lib = None


def lib():
    """Load libdgmg.so (built in-tree by `paper_2405_18982_amd.build`)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_18982_amd.build`")
        # torch bundles its own HIP runtime (same soname as ROCm's).  Loading
        # torch first makes libdgmg bind to that copy, so the process holds a
        # single runtime that both torch tensors and libdgmg kernels use.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DGMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def patch_eigen(k, sigma, ptype, variant=SMOOTH_EXACT):
    """Host-only reference 1-D fast-diagonalisation data (S, lam) of a patch
    type for the local space of a smoother variant."""
    E = 2 * (k + 1)
    S = np.zeros(E * E)
    lam = np.zeros(E)
    st = lib().dgmg_patch_eigen(k, sigma, variant, ptype, S.ctypes.data, lam.ctypes.data)
    if st != 0:
        raise DGMGError(st, "dgmg_patch_eigen failed")
    return S.reshape(E, E), lam


def _torch():
    import torch
    return torch


class Problem:
    """One SIPG multigrid context: -kappa Laplace u = f on [0,1]^dim, Q_k,
    levels 0..L with 2^(l+1) cells per direction."""

    def __init__(self, dim, k, L, sigma=None, kappa=1.0, precision=FP64, variant=SMOOTH_EXACT,
                 nrhs_max=1):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libdgmg needs a GPU: torch.cuda.is_available() is False")
        # libdgmg runs on the HIP runtime torch has loaded: let torch create the
        # device context first so both share one initialised runtime.
        torch.cuda.init()
        torch.empty(1, device="cuda")
        torch.cuda.synchronize()
        self.dim, self.k, self.L = dim, k, L
        self.sigma = 2.0 * (k + 1) ** 2 if sigma is None else float(sigma)
        self.kappa = float(kappa)
        self.precision, self.variant, self.nrhs_max = precision, variant, nrhs_max
        self._ctx = ctypes.c_void_p()
        st = lib().dgmg_setup_mesh(dim, k, L, self.sigma, self.kappa, ctypes.byref(self._ctx))
        if st != 0:
            raise DGMGError(st, "dgmg_setup_mesh rejected the arguments")
        self._check(lib().dgmg_setup_levels(self._ctx, precision, variant, nrhs_max,
                                            self._stream()))

    # ---------------------------------------------------------- plumbing
    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)

    def _check(self, st):
        if st != 0:
            msg = lib().dgmg_last_error(self._ctx)
            raise DGMGError(st, msg.decode() if msg else "")

    def _sync_stream(self):
        self._check(lib().dgmg_set_stream(self._ctx, self._stream()))

    def _vec(self, t, level, dtype):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a CUDA (HIP) torch tensor")
        if t.dtype != dtype:
            raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        n = self.ndofs(level)
        if t.numel() % n != 0 or t.numel() == 0:
            raise ValueError(f"tensor size {t.numel()} is not a multiple of ndofs({level}) = {n}")
        return ctypes.c_void_p(t.data_ptr()), t.numel() // n

    def _vec_like(self, t, level, dtype, nrhs, what):
        """_vec for a secondary tensor, which must hold the same number of
        right-hand sides as the primary one (checked before any launch)."""
        ptr, nr = self._vec(t, level, dtype)
        if nr != nrhs:
            raise ValueError(f"{what} holds {nr} right-hand side(s), expected {nrhs}")
        return ptr

    def _lvl(self, level):
        return self.L if level is None else level

    # ------------------------------------------------------------- sizes
    def ndofs(self, level=None):
        return int(lib().dgmg_level_ndofs(self._ctx, self._lvl(level)))

    def cells(self, level=None):
        return int(lib().dgmg_level_cells(self._ctx, self._lvl(level)))

    def node_coords(self, level=None):
        level = self._lvl(level)
        out = np.zeros(self.ndofs(level) * self.dim)
        self._check(lib().dgmg_node_coords(self._ctx, level, out.ctypes.data))
        return out.reshape(-1, self.dim)

    def autotune(self, nrhs=1, cache=None):
        """Pick the fastest workgroup shapes of apply/smooth (finest level);
        returns the decisions as text.  cache: JSON file path or None."""
        buf = ctypes.create_string_buffer(4096)
        self._sync_stream()
        path = cache.encode() if cache else None
        self._check(lib().dgmg_autotune(self._ctx, int(nrhs), path, buf, len(buf)))
        return buf.value.decode()

    def use_graphs(self, enable=True):
        self._check(lib().dgmg_use_graphs(self._ctx, int(bool(enable))))

    def use_dense_bottom(self, enable=True):
        """V-cycle bottom levels as the dense operator built at set-up (True)
        or as the fused bottom launch (False)."""
        self._check(lib().dgmg_use_dense_bottom(self._ctx, int(bool(enable))))

    def dense_bottom_level(self):
        """Level whose correction the dense bottom operator gives, or -1."""
        return int(lib().dgmg_dense_bottom_level(self._ctx))

    def set_kappa(self, kappa):
        self.kappa = float(kappa)
        self._check(lib().dgmg_set_kappa(self._ctx, self.kappa))

    def empty(self, level=None, nrhs=1, dtype=None):
        torch = _torch()
        dtype = torch.float64 if dtype is None else dtype
        shape = (self.ndofs(level),) if nrhs == 1 else (nrhs, self.ndofs(level))
        return torch.empty(shape, dtype=dtype, device="cuda")

    # -------------------------------------------------------- operations
    def apply(self, x, level=None, out=None):
        torch = _torch()
        level = self._lvl(level)
        f32 = x.dtype == torch.float32
        px, nr = self._vec(x, level, x.dtype)
        out = torch.empty_like(x) if out is None else out
        py = self._vec_like(out, level, x.dtype, nr, "out")
        self._sync_stream()
        fn = lib().dgmg_apply_sipg_f32 if f32 else lib().dgmg_apply_sipg
        self._check(fn(self._ctx, level, px, py, nr))
        return out

    def mass(self, x, level=None, out=None):
        torch = _torch()
        level = self._lvl(level)
        px, nr = self._vec(x, level, torch.float64)
        out = torch.empty_like(x) if out is None else out
        py = self._vec_like(out, level, torch.float64, nr, "out")
        self._sync_stream()
        self._check(lib().dgmg_apply_mass(self._ctx, level, px, py, nr))
        return out

    def smooth(self, x, b, level=None, reverse=False):
        """One smoothing step in place on x; returns x."""
        torch = _torch()
        level = self._lvl(level)
        f32 = x.dtype == torch.float32
        px, nr = self._vec(x, level, x.dtype)
        pb = self._vec_like(b, level, x.dtype, nr, "b")
        self._sync_stream()
        fn = lib().dgmg_smooth_patch_f32 if f32 else lib().dgmg_smooth_patch
        self._check(fn(self._ctx, level, px, pb, int(bool(reverse)), nr))
        return x

    def restrict_residual(self, x, b, level=None, out=None):
        torch = _torch()
        level = self._lvl(level)
        f32 = x.dtype == torch.float32
        px, nr = self._vec(x, level, x.dtype)
        pb = self._vec_like(b, level, x.dtype, nr, "b")
        if out is None:
            shape = (self.ndofs(level - 1),) if x.dim() == 1 else (nr, self.ndofs(level - 1))
            out = torch.empty(shape, dtype=x.dtype, device=x.device)
        pc = self._vec_like(out, level - 1, x.dtype, nr, "out")
        self._sync_stream()
        fn = lib().dgmg_restrict_residual_f32 if f32 else lib().dgmg_restrict_residual
        self._check(fn(self._ctx, level, px, pb, pc, nr))
        return out

    def prolongate_add(self, xc, x, level=None):
        torch = _torch()
        level = self._lvl(level)
        f32 = x.dtype == torch.float32
        px, nr = self._vec(x, level, x.dtype)
        pc = self._vec_like(xc, level - 1, x.dtype, nr, "xc")
        self._sync_stream()
        fn = lib().dgmg_prolongate_add_f32 if f32 else lib().dgmg_prolongate_add
        self._check(fn(self._ctx, level, pc, px, nr))
        return x

    def coarse_solve(self, b, out=None):
        torch = _torch()
        f32 = b.dtype == torch.float32
        pb, nr = self._vec(b, 0, b.dtype)
        out = torch.empty_like(b) if out is None else out
        px = self._vec_like(out, 0, b.dtype, nr, "out")
        self._sync_stream()
        fn = lib().dgmg_coarse_solve_f32 if f32 else lib().dgmg_coarse_solve
        self._check(fn(self._ctx, pb, px, nr))
        return out

    def dot(self, a, b, level=None):
        """Per-right-hand-side inner products a_j . b_j (numpy array)."""
        torch = _torch()
        level = self._lvl(level)
        pa, nr = self._vec(a, level, torch.float64)
        pb = self._vec_like(b, level, torch.float64, nr, "b")
        out = np.zeros(nr)
        self._sync_stream()
        self._check(lib().dgmg_dot(self._ctx, level, pa, pb, nr, out.ctypes.data))
        return out

    def adjoint_dkappa(self, lam, u):
        """Coefficient gradient -lambda_j^T A_1 u_j per right-hand side (numpy
        array) and its sum over the right-hand sides (float), computed by the
        library."""
        torch = _torch()
        pl, nr = self._vec(lam, self.L, torch.float64)
        pu = self._vec_like(u, self.L, torch.float64, nr, "u")
        per = np.zeros(nr)
        tot = ctypes.c_double(0.0)
        self._sync_stream()
        self._check(lib().dgmg_adjoint_dkappa(self._ctx, pl, pu, nr, per.ctypes.data, ctypes.byref(tot)))
        return per, tot.value

    def vcycle(self, b, out=None):
        torch = _torch()
        f32 = b.dtype == torch.float32
        pb, nr = self._vec(b, self.L, b.dtype)
        out = torch.empty_like(b) if out is None else out
        px = self._vec_like(out, self.L, b.dtype, nr, "out")
        self._sync_stream()
        fn = lib().dgmg_vcycle_f32 if f32 else lib().dgmg_vcycle
        self._check(fn(self._ctx, pb, px, nr))
        return out

    def vcycle_noalloc(self, b, out):
        """dgmg_vcycle_noalloc: the V-cycle with its level vectors in the
        library's scratch array; b and out are FP64 and caller-allocated."""
        torch = _torch()
        pb, nr = self._vec(b, self.L, torch.float64)
        px = self._vec_like(out, self.L, torch.float64, nr, "out")
        self._sync_stream()
        self._check(lib().dgmg_vcycle_noalloc(self._ctx, pb, px, nr))
        return out

    def solve(self, b, rtol=1e-10, maxit=100, x0=None, out=None, raise_on_nonconvergence=True):
        """PCG solve; returns (x, iters[nrhs], relres[nrhs])."""
        torch = _torch()
        pb, nr = self._vec(b, self.L, torch.float64)
        out = torch.empty_like(b) if out is None else out
        px = self._vec_like(out, self.L, torch.float64, nr, "out")
        if x0 is not None:
            self._vec_like(x0, self.L, torch.float64, nr, "x0")
            if x0.data_ptr() != out.data_ptr():
                out.copy_(x0)  # the initial guess is not overwritten
        iters = np.zeros(nr, dtype=np.int32)
        relres = np.zeros(nr)
        self._sync_stream()
        st = lib().dgmg_pcg_solve(self._ctx, pb, px, int(x0 is not None), float(rtol), int(maxit), nr,
                                  iters.ctypes.data, relres.ctypes.data)
        if st == -4 and not raise_on_nonconvergence:
            return out, iters, relres
        self._check(st)
        return out, iters, relres

    def gmres(self, b, rtol=1e-8, maxit=50, out=None, raise_on_nonconvergence=True):
        """Right-preconditioned GMRES from x0 = 0 (one right-hand side);
        returns (x, iterations, residual history |r_i|/|b|, i = 0..iterations)."""
        torch = _torch()
        pb, nr = self._vec(b, self.L, torch.float64)
        if nr != 1:
            raise ValueError("gmres takes one right-hand side")
        out = torch.empty_like(b) if out is None else out
        px = self._vec_like(out, self.L, torch.float64, 1, "out")
        it = ctypes.c_int(0)
        hist = np.zeros(int(maxit) + 1)
        self._sync_stream()
        st = lib().dgmg_gmres_solve(self._ctx, pb, px, float(rtol), int(maxit), ctypes.byref(it),
                                    hist.ctypes.data)
        if not (st == -4 and not raise_on_nonconvergence):
            self._check(st)
        return out, it.value, hist[: it.value + 1].copy()

    def close(self):
        if self._ctx:
            lib().dgmg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solve_function():
    torch = _torch()

    class SolveFn(torch.autograd.Function):
        """u = A(kappa)^{-1} b with A(kappa) = kappa A_1, b of shape (ndofs,)
        or (nrhs, ndofs) sharing one kappa.  Backward: adjoint solve with the
        same symmetric operator, lambda = A^{-1} g; dL/db = lambda,
        dL/dkappa = -sum_j lambda_j^T A_1 u_j (library call)."""

        @staticmethod
        def forward(ctx, b, kappa, prob, rtol, maxit):
            prob.set_kappa(float(kappa))
            u, _, _ = prob.solve(b.contiguous(), rtol=rtol, maxit=maxit)
            ctx.prob, ctx.rtol, ctx.maxit = prob, rtol, maxit
            ctx.kappa = float(kappa)
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, g):
            (u,) = ctx.saved_tensors
            prob = ctx.prob
            prob.set_kappa(ctx.kappa)
            lam, _, _ = prob.solve(g.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
            # -sum_j lambda_j^T A_1 u_j over every right-hand side, in the library
            _, dkappa = prob.adjoint_dkappa(lam, u)
            return lam, torch.tensor(dkappa, dtype=torch.float64, device=g.device), None, None, None

    return SolveFn


_SOLVE_FN = None


def solve(b, kappa, prob, rtol=1e-12, maxit=200):
    """Differentiable solve u = A(kappa)^{-1} b (gradients for b and kappa)."""
    global _SOLVE_FN
    torch = _torch()
    if _SOLVE_FN is None:
        _SOLVE_FN = _solve_function()
    if not isinstance(kappa, torch.Tensor):
        kappa = torch.tensor(float(kappa), dtype=torch.float64, device=b.device)
    return _SOLVE_FN.apply(b, kappa, prob, rtol, maxit)
