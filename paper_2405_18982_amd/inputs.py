"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds none of the method's arithmetic: it draws random
vectors, defines the closed-form load functions of the manufactured Poisson
problems, and lists the workloads.  Node coordinates, load vectors and
everything else that needs the discretisation are computed by each side on
its own.
"""
import numpy as np

# Workloads: unit square / cube, level l has 2^(l+1) cells per direction, the
# penalty per unit face length is sigma = 2 (k+1)^2 and gamma_F = sigma / h.
WORKLOADS = {
    "poisson2d_q2_8x8": dict(dim=2, k=2, L=2, kappa=1.0, nrhs=1, precision=64,
                             rhs="sine", seed=None),
    "poisson3d_q3_32c": dict(dim=3, k=3, L=4, kappa=1.0, nrhs=1, precision=64,
                             rhs="sine", seed=7),
    "poisson3d_q7_64c_mixed": dict(dim=3, k=7, L=5, kappa=1.0, nrhs=1, precision=32,
                                   rhs="uniform", seed=3),
    "poisson3d_q4_32c_16rhs": dict(dim=3, k=4, L=4, kappa=1.0, nrhs=16, precision=32,
                                   rhs="normal", seed=4),
    "poisson2d_q5_256c_adjoint": dict(dim=2, k=5, L=7, kappa=1.0, nrhs=1, precision=64,
                                      rhs="fourier", seed=5, target_seed=6),
}


def sigma_of(k):
    return 2.0 * (k + 1) ** 2


def ndofs(dim, k, L):
    return (2 ** (L + 1)) ** dim * (k + 1) ** dim


def uniform(seed, shape, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def normal(seed, shape):
    return np.random.default_rng(seed).standard_normal(size=shape)


def sine_solution(X):
    """u = prod_i sin(pi x_i)."""
    return np.prod(np.sin(np.pi * X), axis=1)


def sine_load(X):
    """f = -Laplace u = d pi^2 prod_i sin(pi x_i) for u = sine_solution."""
    return X.shape[1] * np.pi ** 2 * np.prod(np.sin(np.pi * X), axis=1)


def fourier_modes(seed, count=32, mmax=16):
    """Mode table of a random smooth 2-D field: integer wave numbers m_j in
    {1..mmax}^2 and amplitudes a_j = z_j / (1 + |m_j|^2), z_j ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, mmax + 1, size=(count, 2))
    z = rng.standard_normal(count)
    a = z / (1.0 + np.sum(m.astype(np.float64) ** 2, axis=1))
    return m, a


def fourier_field(modes, X):
    """f(x, y) = sum_j a_j sin(pi m_j1 x) sin(pi m_j2 y)."""
    m, a = modes
    out = np.zeros(X.shape[0])
    for (m1, m2), aj in zip(m, a):
        out += aj * np.sin(np.pi * m1 * X[:, 0]) * np.sin(np.pi * m2 * X[:, 1])
    return out
