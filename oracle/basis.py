"""Oracle (test infrastructure only): one-dimensional Q_k building blocks.

Follows Appendix A of the paper: the 1-D shape functions are the Lagrange
polynomials on the k+1 Gauss-Lobatto points of the reference interval [0,1],
phi_nu(xi_mu) = delta_{mu nu}; the d-D shape functions are their tensor
products.  Integrals are exact Gauss-Legendre sums.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k):
    """k+1 Gauss-Lobatto points on [0,1]: the endpoints and the roots of P_k'
    (Appendix A), found by numpy's root finder and polished by Newton steps."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    dc = npleg.legder(c)
    d2c = npleg.legder(dc)
    r = np.sort(np.real(npleg.legroots(dc)))
    for _ in range(6):
        r = r - npleg.legval(r, dc) / npleg.legval(r, d2c)
    x = np.concatenate([[-1.0], r, [1.0]])
    return 0.5 * (x + 1.0)


def gll_weights(k):
    """Gauss-Lobatto weights on [0,1]: w_j = 1/(k(k+1) P_k(x_j)^2) (textbook closed form)."""
    x = 2.0 * gll_nodes(k) - 1.0
    c = np.zeros(k + 1)
    c[k] = 1.0
    pk = npleg.legval(x, c)
    return 1.0 / (k * (k + 1) * pk * pk)


def gauss(m):
    """m-point Gauss-Legendre rule on [0,1] (library primitive)."""
    x, w = npleg.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_eval(nodes, x):
    """V[i, j] = phi_j(x_i) and D[i, j] = phi_j'(x_i) for the Lagrange basis on
    `nodes`, written out as products (no barycentric shortcut)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.zeros((len(x), n))
    D = np.zeros((len(x), n))
    for j in range(n):
        others = [m for m in range(n) if m != j]
        denom = 1.0
        for m in others:
            denom *= nodes[j] - nodes[m]
        num = np.ones_like(x)
        for m in others:
            num = num * (x - nodes[m])
        V[:, j] = num / denom
        for l in others:
            prod = np.ones_like(x)
            for m in others:
                if m != l:
                    prod = prod * (x - nodes[m])
            D[:, j] += prod / denom
    return V, D


class Basis1D:
    """Reference 1-D data of Q_k on [0,1]:

    M  [mu,nu] = int phi_mu phi_nu          (mass)
    K  [mu,nu] = int phi_mu' phi_nu'        (stiffness)
    e0, e1     = phi(0), phi(1)             (traces)
    d0, d1     = phi'(0), phi'(1)           (end derivatives)
    P[o][mu,nu] = phi_nu((xi_mu + o)/2)     (embedding of a coarse cell into child o)
    """

    def __init__(self, k):
        self.k = k
        self.n = k + 1
        self.nodes = gll_nodes(k)
        xq, wq = gauss(k + 1)  # exact for degree 2k+1
        Vq, Dq = lagrange_eval(self.nodes, xq)
        self.M = Vq.T @ (wq[:, None] * Vq)
        self.K = Dq.T @ (wq[:, None] * Dq)
        V0, D0 = lagrange_eval(self.nodes, [0.0])
        V1, D1 = lagrange_eval(self.nodes, [1.0])
        self.e0, self.e1 = V0[0], V1[0]
        self.d0, self.d1 = D0[0], D1[0]
        self.P = []
        for o in (0, 1):
            Vc, _ = lagrange_eval(self.nodes, 0.5 * (self.nodes + o))
            self.P.append(Vc)

    def eval(self, x):
        return lagrange_eval(self.nodes, x)
