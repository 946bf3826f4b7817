"""Oracle (test infrastructure only): the multilevel preconditioner of Sec. 3
and the outer Krylov solvers.

Mesh hierarchy: T_0 is one cell refined once (N_0 = 2 cells per direction);
level l has N_l = 2^(l+1) cells per direction.  Level operators are the SIPG
matrices rediscretised on each level (gamma = sigma/h_l).

V-cycle P_l^{-1} b (Sec. 3, with x_l = 0 on entry):
    l = 0:  x = A_0^{-1} b
    l >= 1: x = S_l(0, b)                 pre-smoothing, colours ascending
            x += P V_{l-1}(P^T (b - A_l x))  coarse-grid correction
            x = S_l(x, b)                 post-smoothing, colours descending
The reversed colour order in post-smoothing and the transpose restriction
make the preconditioner symmetric, which CG requires.

Outer solvers: preconditioned CG (optionally with the flexible
Polak-Ribiere beta used when the V-cycle runs in reduced precision) and
right-preconditioned GMRES without restart.  Fractional iteration count of
Sec. 3.3: nu = -8 / log10(rbar), rbar = (|r_n|/|r_0|)^(1/n).
"""
import numpy as np
import scipy.linalg as sla

from .sipg import KronApply, kron_operator
from .smoother import FDSmoother, colour_orders, smooth_dense
from .patches import PatchSet
from .transfer import prolongation


class Hierarchy:
    def __init__(self, d, k, L, sigma, kappa=1.0, mode="exact", dense=False, dtype=np.float64):
        self.d, self.k, self.L, self.sigma, self.kappa = d, k, L, sigma, kappa
        self.mode, self.dense, self.dtype = mode, dense, dtype
        self.N = [2 ** (l + 1) for l in range(L + 1)]
        self.P = [None] + [prolongation(d, k, self.N[l - 1]) for l in range(1, L + 1)]
        self.asc, self.desc = colour_orders(d)
        self.A, self.apply, self.smoothers, self.ps = [], [], [], []
        for l in range(L + 1):
            N = self.N[l]
            if dense:
                A = kron_operator(d, k, N, sigma, kappa)
                self.A.append(A)
                self.apply.append(lambda x, A=A: A @ x)
                self.ps.append(PatchSet(d, k, N) if l > 0 else None)
                self.smoothers.append(None)
            else:
                ap = KronApply(d, k, N, sigma, kappa)
                self.A.append(None)
                self.apply.append(ap)
                self.smoothers.append(FDSmoother(d, k, N, sigma, kappa, mode, ap) if l > 0 else None)
        A0 = kron_operator(d, k, self.N[0], sigma, kappa).toarray()
        self.coarse = sla.cho_factor(A0)

    def ndofs(self, l):
        return self.N[l] ** self.d * (self.k + 1) ** self.d

    def smooth(self, l, x, b, order):
        if self.dense:
            return smooth_dense(self.A[l], x, b, self.ps[l], order, self.mode, self.kappa)
        return self.smoothers[l].step(x, b, order)

    def _round(self, v):
        return v.astype(self.dtype).astype(np.float64) if self.dtype != np.float64 else v

    def vcycle(self, b, l=None):
        l = self.L if l is None else l
        if l == 0:
            return self._round(sla.cho_solve(self.coarse, b))
        x = np.zeros_like(b)
        x = self._round(self.smooth(l, x, b, self.asc))
        r = self._round(b - self.apply[l](x))
        bc = self._round(self.P[l].T @ r)
        xc = self.vcycle(bc, l - 1)
        x = self._round(x + self.P[l] @ xc)
        return self._round(self.smooth(l, x, b, self.desc))


def pcg(apply, precond, b, rtol=1e-10, maxit=200, x0=None, flexible=False):
    """Preconditioned CG with x0 = 0 (or x0).  Stops when |r|_2 / |b|_2 <= rtol
    on the recursively updated residual.  Returns x, iterations, history of
    relative residuals and the true final relative residual."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x) if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    if hist[0] <= rtol:
        return x, 0, hist, hist[0]
    z = precond(r)
    p = z.copy()
    rho = r @ z
    it = 0
    for it in range(1, maxit + 1):
        q = apply(p)
        pq = p @ q
        if not pq > 0:
            raise FloatingPointError("CG breakdown: p^T A p <= 0")
        alpha = rho / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z = precond(r)
        rho_new = z @ (r - r_old) if flexible else r @ z
        beta = rho_new / rho
        rho = r @ z if flexible else rho_new
        p = z + beta * p
    true_rel = np.linalg.norm(b - apply(x)) / nb
    return x, it, hist, true_rel


def gmres(apply, precond, b, rtol=1e-8, maxit=200):
    """Right-preconditioned GMRES(inf) with x0 = 0 (Arnoldi with modified
    Gram-Schmidt, Givens rotations).  Returns x, iterations and the history of
    |r_n| / |r_0|."""
    nb = np.linalg.norm(b)
    V = [b / nb]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = nb
    hist = [1.0]
    m = 0
    for j in range(maxit):
        z = precond(V[j])
        Z.append(z)
        w = apply(z)
        for i in range(j + 1):
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        m = j + 1
        hist.append(abs(g[j + 1]) / nb)
        if hist[-1] <= rtol:
            break
    y = sla.solve_triangular(H[:m, :m], g[:m])
    x = sum(y[i] * Z[i] for i in range(m))
    return x, m, hist


def fractional_iterations(hist):
    """nu = -8 / log10(rbar), rbar = (|r_n|/|r_0|)^(1/n) (Sec. 3.3)."""
    n = len(hist) - 1
    rbar = (hist[-1] / hist[0]) ** (1.0 / n)
    return -8.0 / np.log10(rbar)
