"""Oracle (test infrastructure only): load vectors, nodal interpolants and L2
errors on the cell-wise layout.

b_i = int f phi_i (eq. weak_form) by tensor Gauss quadrature with q points per
direction and cell (default k+2); the interpolated load b = M I_h f; nodal
interpolation at the Gauss-Lobatto nodes (Appendix A); the L2 error of a
discrete function against a closed-form one by Gauss quadrature.
"""
import numpy as np

from .basis import Basis1D, gauss


def _cell_origins(d, N):
    cells = np.arange(N ** d)
    return np.stack([((cells // N ** i) % N) / N for i in range(d)], axis=1)  # (ncell, d)


def _tensor_points(d, pts1):
    """(m^d, d) reference points, x fastest."""
    m = len(pts1)
    idx = np.arange(m ** d)
    return np.stack([pts1[(idx // m ** i) % m] for i in range(d)], axis=1)


def node_coords(d, k, N):
    """Physical coordinates of every DoF, shape (N^d (k+1)^d, d)."""
    b = Basis1D(k)
    h = 1.0 / N
    org = _cell_origins(d, N)
    ref = _tensor_points(d, b.nodes)
    X = org[:, None, :] + h * ref[None, :, :]
    return X.reshape(-1, d)


def interpolate(d, k, N, u):
    return u(node_coords(d, k, N))


def _contract_cells(d, C, A1):
    """For C of shape (ncell, m,...,m) (axis order z,y,x) return C contracted
    with A1 (m x n) along every axis: out[c, b...] = sum_q A1[q,b] ... C[c,q...]."""
    T = C
    for ax in range(1, d + 1):
        T = np.moveaxis(np.tensordot(T, A1, axes=([ax], [0])), -1, ax)
    return T


def load_vector(d, k, N, f, q=None):
    b = Basis1D(k)
    n = k + 1
    h = 1.0 / N
    q = k + 2 if q is None else q
    xq, wq = gauss(q)
    Vq, _ = b.eval(xq)  # (q, n)
    org = _cell_origins(d, N)
    ref = _tensor_points(d, xq)
    W = np.ones(len(ref))
    idx = np.arange(q ** d)
    for i in range(d):
        W = W * wq[(idx // q ** i) % q]
    X = org[:, None, :] + h * ref[None, :, :]
    F = f(X.reshape(-1, d)).reshape(N ** d, q ** d) * W[None, :] * h ** d
    F = F.reshape((N ** d,) + (q,) * d)
    B = _contract_cells(d, F, Vq)
    return B.reshape(N ** d * n ** d)


def l2_error(d, k, N, uh, u, q=None):
    b = Basis1D(k)
    h = 1.0 / N
    q = k + 3 if q is None else q
    xq, wq = gauss(q)
    Vq, _ = b.eval(xq)  # (q, n)
    n = k + 1
    org = _cell_origins(d, N)
    ref = _tensor_points(d, xq)
    W = np.ones(len(ref))
    idx = np.arange(q ** d)
    for i in range(d):
        W = W * wq[(idx // q ** i) % q]
    U = uh.reshape((N ** d,) + (n,) * d)
    T = U
    for ax in range(1, d + 1):
        T = np.moveaxis(np.tensordot(T, Vq.T, axes=([ax], [0])), -1, ax)
    uq = T.reshape(N ** d, q ** d)
    X = org[:, None, :] + h * ref[None, :, :]
    ex = u(X.reshape(-1, d)).reshape(N ** d, q ** d)
    return float(np.sqrt(np.sum((uq - ex) ** 2 * W[None, :]) * h ** d))


def sine_solution(X):
    return np.prod(np.sin(np.pi * X), axis=1)


def sine_load(X):
    d = X.shape[1]
    return d * np.pi ** 2 * np.prod(np.sin(np.pi * X), axis=1)


def bubble_solution(X):
    """u = prod x_i (1 - x_i): degree 2 per direction, zero on the boundary."""
    return np.prod(X * (1.0 - X), axis=1)


def bubble_load(X):
    d = X.shape[1]
    out = np.zeros(X.shape[0])
    for i in range(d):
        term = 2.0 * np.ones(X.shape[0])
        for j in range(d):
            if j != i:
                term = term * X[:, j] * (1.0 - X[:, j])
        out += term
    return out
