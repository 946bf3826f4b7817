"""Oracle (test infrastructure only): gradients of the differentiable solve.

Forward: u = A(kappa)^{-1} b with A(kappa) = kappa A_1 (the whole SIPG form,
penalty included, scaled by kappa).  Loss L = 1/2 |u - u_t|_2^2 (Euclidean
norm over the DoF vector).  Because A is symmetric the adjoint solve uses the
same operator:
    lambda = A^{-1} (u - u_t),  dL/db = lambda,  dL/dkappa = -lambda^T A_1 u.
Since u(kappa) = u_1 / kappa the last one also has the closed form
    dL/dkappa = -(u - u_t)^T u / kappa.
"""
import numpy as np
import scipy.sparse.linalg as spla


def dense_adjoint(A1, kappa, b, u_target):
    A = (kappa * A1).tocsc()
    lu = spla.splu(A)
    u = lu.solve(b)
    lam = lu.solve(u - u_target)
    loss = 0.5 * float((u - u_target) @ (u - u_target))
    return u, loss, lam, float(-(lam @ (A1 @ u)))


def closed_form_dkappa(u, u_target, kappa):
    return float(-((u - u_target) @ u) / kappa)
