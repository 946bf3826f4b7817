"""Oracle (test infrastructure only): grid transfer between level l-1 (N/2
cells per direction) and level l (N cells), Sec. 3.

Prolongation is the canonical embedding V_{l-1} in V_l: a coarse cell C has
the 2^d children F with f_i = 2 c_i + o_i, and on child o the coarse function
is re-interpolated at the child's nodes, i.e. the block (x)_i P[o_i] with
P[o][mu,nu] = phi_nu((xi_mu + o)/2).

The restriction applied to residual (dual) vectors is the transpose P^T; on
primal functions it corresponds to the L2 projection named in Sec. 3 (the
pairing <P^T r, v_c> = <r, P v_c>), and it keeps the V-cycle symmetric.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .basis import Basis1D


def prolongation(d, k, Nc):
    """Sparse P (fine cell-wise layout x coarse cell-wise layout), Nf = 2 Nc."""
    b = Basis1D(k)
    n = k + 1
    nl = n ** d
    Nf = 2 * Nc
    blocks = {}
    for o in itertools.product((0, 1), repeat=d):  # o[i] = child offset in direction i
        B = np.array([[1.0]])
        for i in range(d):
            B = np.kron(b.P[o[i]], B)  # direction i slower than i-1
        blocks[o] = B
    rows, cols, data = [], [], []
    for cc in itertools.product(range(Nc), repeat=d):
        c = cc[::-1]  # c[i] = coarse coordinate in direction i
        cidx = sum(c[i] * Nc ** i for i in range(d))
        for o, B in blocks.items():
            f = [2 * c[i] + o[i] for i in range(d)]
            fidx = sum(f[i] * Nf ** i for i in range(d))
            rr, ccol = np.meshgrid(fidx * nl + np.arange(nl), cidx * nl + np.arange(nl), indexing="ij")
            rows.append(rr.ravel())
            cols.append(ccol.ravel())
            data.append(B.ravel())
    return sp.csr_matrix(
        (np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
        shape=(Nf ** d * nl, Nc ** d * nl),
    )
