"""Oracle (test infrastructure only): exact discrete solve A u = b on the
whole brick by fast diagonalisation (Lynch-Rice-Thomas, cited in Sec. 3.2).

On the Cartesian brick A = sum_i (x)(M, .., L at i, .., M) with the 1-D global
mass M and SIPG matrix L; with L S = M S Lambda, S^T M S = I (one dense
generalised symmetric eigenproblem of size N(k+1)),
    A^{-1} = ((x) S) (sum_i Lambda_i)^{-1} ((x) S^T).
The eigenvalues sum_i lambda_i are exactly the spectrum of the generalised
problem A u = lambda ... with mass I, so min(sum lambda) > 0 certifies SPD.
"""
import numpy as np
import scipy.linalg as sla

from .sipg import lex_of_cellwise, sipg_1d


class GlobalFD:
    def __init__(self, d, k, N, sigma, kappa=1.0):
        M, L = sipg_1d(k, N, sigma)
        self.d, self.k, self.N = d, k, N
        self.lam, self.S = sla.eigh(kappa * L, M)
        self.perm = lex_of_cellwise(d, k, N)
        self.Nn = N * (k + 1)

    def _along(self, A1, X, axis):
        Xm = np.moveaxis(X, axis, 0)
        sh = Xm.shape
        Y = (A1 @ Xm.reshape(sh[0], -1)).reshape(sh)
        return np.moveaxis(Y, 0, axis)

    def eigenvalues_1d(self):
        return self.lam

    def solve(self, b):
        d, Nn = self.d, self.Nn
        bl = np.empty_like(b)
        bl[self.perm] = b
        X = bl.reshape((Nn,) * d)
        for ax in range(d):
            X = self._along(self.S.T, X, ax)
        lam = np.zeros((Nn,) * d)
        for ax in range(d):
            shape = [1] * d
            shape[ax] = Nn
            lam = lam + self.lam.reshape(shape)
        X = X / lam
        for ax in range(d):
            X = self._along(self.S, X, ax)
        return X.reshape(-1)[self.perm]
