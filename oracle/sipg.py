"""Oracle (test infrastructure only): the SIPG Laplacian on the uniform
Cartesian mesh of [0,1]^d with N cells per direction.

Two independent constructions of the system matrix A of eq. (mat_form):

* `assemble_quadrature` integrates the bilinear form of eq. (bilinear_form)
  cell by cell and face by face with tensor Gauss quadrature in d dimensions,
  using the jump/mean definitions of eqs. (jump_mean, jump_boundary) read as
  [[u]] = u+ n+ + u- n- on interior faces and [[u]] = u n on boundary faces.
* `kron_operator` uses the Kronecker structure of Sec. 2.2 (A_j = L (x) M + M (x) L,
  extended by the face terms, which on a Cartesian mesh factor into a 1-D
  point term times the (d-1)-D face mass).

Penalty: gamma_F = sigma / h on every face (for the paper's choice
gamma_e = k(k+1)(1/h+ + 1/h-) on a uniform mesh sigma = 2k(k+1)); a scalar
coefficient kappa multiplies the whole form.

DoF layout ("cell-wise lexicographic", Sec. 4.1, Fig. dof_layout right):
index = cell * n^d + local, cell = sum_i c_i N^i, local = sum_i l_i n^i,
x (i=0) fastest.  The "global lexicographic" brick layout (Fig. dof_layout
left) is used internally for the Kronecker form: index = sum_i g_i (N n)^i with
g_i = c_i n + l_i.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .basis import Basis1D, gauss


def lex_of_cellwise(d, k, N):
    """perm[I_cellwise] = I_lex."""
    n = k + 1
    ncell = N ** d
    cells = np.arange(ncell)
    loc = np.arange(n ** d)
    c = [(cells // N ** i) % N for i in range(d)]
    l = [(loc // n ** i) % n for i in range(d)]
    lex = np.zeros((ncell, n ** d), dtype=np.int64)
    for i in range(d):
        g = c[i][:, None] * n + l[i][None, :]
        lex += g * (N * n) ** i
    return lex.reshape(-1)


def sipg_1d(k, N, sigma):
    """1-D global mass M and SIPG matrix L on N cells of [0,1] (dense, size N n).

    L = sum_K int u'v' + sum_F (gamma [u][v] - {u'}[v] - [u]{v'}) in one
    dimension, gamma = sigma/h; Nitsche terms on the two boundary points."""
    b = Basis1D(k)
    n = k + 1
    h = 1.0 / N
    g = sigma / h
    M = np.zeros((N * n, N * n))
    L = np.zeros((N * n, N * n))
    o = np.outer
    e0, e1, d0, d1 = b.e0, b.e1, b.d0, b.d1
    for c in range(N):
        s = slice(c * n, (c + 1) * n)
        M[s, s] = h * b.M
        L[s, s] += b.K / h
    for f in range(1, N):
        a = slice((f - 1) * n, f * n)
        c = slice(f * n, (f + 1) * n)
        L[a, a] += g * o(e1, e1) - (o(e1, d1) + o(d1, e1)) / (2 * h)
        L[c, c] += g * o(e0, e0) + (o(e0, d0) + o(d0, e0)) / (2 * h)
        Lac = -g * o(e1, e0) - o(e1, d0) / (2 * h) + o(d1, e0) / (2 * h)
        L[a, c] += Lac
        L[c, a] += Lac.T
    s0 = slice(0, n)
    s1 = slice((N - 1) * n, N * n)
    L[s0, s0] += g * o(e0, e0) + (o(e0, d0) + o(d0, e0)) / h
    L[s1, s1] += g * o(e1, e1) - (o(e1, d1) + o(d1, e1)) / h
    return M, L


def kron_terms(d, k, N, sigma):
    """The d Kronecker terms of A in global lexicographic order (x fastest),
    each a list of 1-D factors ordered (slowest ... fastest)."""
    M, L = sipg_1d(k, N, sigma)
    terms = []
    for dirn in range(d):
        fac = [L if i == dirn else M for i in range(d)]
        terms.append(fac[::-1])
    return M, L, terms


def kron_operator(d, k, N, sigma, kappa=1.0):
    """Sparse A (cell-wise layout) from the Kronecker sum of 1-D factors."""
    _, _, terms = kron_terms(d, k, N, sigma)
    A = None
    for fac in terms:
        T = sp.csr_matrix(fac[0])
        for F in fac[1:]:
            T = sp.kron(T, sp.csr_matrix(F), format="csr")
        A = T if A is None else A + T
    perm = lex_of_cellwise(d, k, N)
    A = A[perm][:, perm]
    A = (kappa * A).tocsr()
    A.eliminate_zeros()
    return A


def _cell_tabulation(d, k, N):
    """Values and physical gradients of the n^d cell basis functions at the
    m^d tensor Gauss points (m = k+1), plus the weights times |K|."""
    b = Basis1D(k)
    n = k + 1
    h = 1.0 / N
    xq, wq = gauss(k + 1)
    V, D = b.eval(xq)  # (m, n)
    m = len(xq)
    loc = list(itertools.product(range(n), repeat=d))  # tuples (l_{d-1},...,l_0)
    qts = list(itertools.product(range(m), repeat=d))
    nl, nq = len(loc), len(qts)
    val = np.ones((nl, nq))
    grad = np.ones((d, nl, nq))
    wts = np.ones(nq)
    for a, lt in enumerate(loc):
        li = lt[::-1]  # li[i] = local index in direction i
        for q, qt in enumerate(qts):
            qi = qt[::-1]
            val[a, q] = np.prod([V[qi[i], li[i]] for i in range(d)])
            for g in range(d):
                grad[g, a, q] = np.prod(
                    [(D[qi[i], li[i]] / h) if i == g else V[qi[i], li[i]] for i in range(d)]
                )
    for q, qt in enumerate(qts):
        qi = qt[::-1]
        wts[q] = np.prod([wq[qi[i]] for i in range(d)]) * h ** d
    # local lexicographic order: x fastest == reversed tuple order of itertools
    lex = [sum(lt[::-1][i] * n ** i for i in range(d)) for lt in loc]
    order = np.argsort(lex)
    return val[order], grad[:, order], wts


def _face_tabulation(d, k, N, normal_dir, side):
    """Values and physical gradients of the n^d basis functions of one cell on
    its face x_normal = side (0 or 1, reference), at the m^(d-1) tangential
    Gauss points, plus face weights times |F|."""
    b = Basis1D(k)
    n = k + 1
    h = 1.0 / N
    xq, wq = gauss(k + 1)
    V, D = b.eval(xq)
    Vs, Ds = b.eval([float(side)])
    m = len(xq)
    tdirs = [i for i in range(d) if i != normal_dir]
    qts = list(itertools.product(range(m), repeat=d - 1))
    nq = len(qts)
    nl = n ** d
    val = np.zeros((nl, nq))
    grad = np.zeros((d, nl, nq))
    wts = np.zeros(nq)
    for a in range(nl):
        li = [(a // n ** i) % n for i in range(d)]
        for q, qt in enumerate(qts):
            qi = dict(zip(tdirs, qt[::-1]))
            def v1(i, deriv):
                if i == normal_dir:
                    return (Ds[0, li[i]] / h) if deriv else Vs[0, li[i]]
                return (D[qi[i], li[i]] / h) if deriv else V[qi[i], li[i]]
            val[a, q] = np.prod([v1(i, False) for i in range(d)])
            for g in range(d):
                grad[g, a, q] = np.prod([v1(i, i == g) for i in range(d)])
    for q, qt in enumerate(qts):
        qi = dict(zip(tdirs, qt[::-1]))
        wts[q] = np.prod([wq[qi[i]] for i in tdirs]) * h ** (d - 1)
    return val, grad, wts


def assemble_quadrature(d, k, N, sigma, kappa=1.0):
    """Sparse A (cell-wise layout) by direct quadrature of eq. (bilinear_form).

    Cells:  int_K grad u . grad v.
    Faces:  int_F gamma [[u]].[[v]] - {grad u}.[[v]] - [[u]].{grad v}, with
            [[w]] = w_L n_L + w_R n_R (vector, n_L = +e_i from the left cell)
            on interior faces and [[w]] = w n, {grad w} = grad w on boundary faces.
    """
    n = k + 1
    nl = n ** d
    h = 1.0 / N
    gamma = sigma / h
    val, grad, wts = _cell_tabulation(d, k, N)
    Kloc = np.einsum("gaq,gbq,q->ab", grad, grad, wts)
    rows, cols, data = [], [], []

    def add(ri, ci, blk):
        rr, cc = np.meshgrid(ri, ci, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        data.append(blk.ravel())

    ncell = N ** d
    for c in range(ncell):
        dofs = c * nl + np.arange(nl)
        add(dofs, dofs, Kloc)
    for i in range(d):
        e = np.zeros(d)
        e[i] = 1.0
        vR, gR, wf = _face_tabulation(d, k, N, i, 1)  # left cell, its face x_i = 1
        vL, gL, _ = _face_tabulation(d, k, N, i, 0)   # right cell, its face x_i = 0
        for cidx in itertools.product(range(N), repeat=d):
            ci = list(cidx[::-1])  # ci[i] = cell coordinate in direction i
            cell = sum(ci[j] * N ** j for j in range(d))
            dofs = cell * nl + np.arange(nl)
            # boundary faces of this cell in direction i
            for side, (vv, gg, nrm) in ((0, (vL, gL, -e)), (1, (vR, gR, e))):
                if (side == 0 and ci[i] == 0) or (side == 1 and ci[i] == N - 1):
                    jump = vv[None, :, :] * nrm[:, None, None]  # (d, nl, nq)
                    avg = gg
                    blk = (gamma * np.einsum("gaq,gbq,q->ab", jump, jump, wf)
                           - np.einsum("gbq,gaq,q->ab", avg, jump, wf)
                           - np.einsum("gbq,gaq,q->ab", jump, avg, wf))
                    add(dofs, dofs, blk)
            # interior face to the right neighbour
            if ci[i] < N - 1:
                cj = list(ci)
                cj[i] += 1
                nb = sum(cj[j] * N ** j for j in range(d))
                nbd = nb * nl + np.arange(nl)
                # both cells' functions on the shared face: left uses vR (x=1), right vL (x=0)
                jumpL = vR[None] * e[:, None, None]          # left cell normal +e
                jumpRt = vL[None] * (-e)[:, None, None]      # right cell normal -e
                avgL, avgR = 0.5 * gR, 0.5 * gL
                both_d = np.concatenate([dofs, nbd])
                J = np.concatenate([jumpL, jumpRt], axis=1)   # (d, 2nl, nq)
                G = np.concatenate([avgL, avgR], axis=1)
                # row index = test function b, column = trial a
                blk = (gamma * np.einsum("gaq,gbq,q->ba", J, J, wf)
                       - np.einsum("gaq,gbq,q->ba", G, J, wf)
                       - np.einsum("gaq,gbq,q->ba", J, G, wf))
                add(both_d, both_d, blk)
    ndof = ncell * nl
    A = sp.csr_matrix(
        (np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))), shape=(ndof, ndof)
    )
    A.sum_duplicates()
    return (kappa * A).tocsr()


def mass_operator(d, k, N):
    """Sparse global mass matrix (cell-wise layout): blkdiag of (x) h M_hat."""
    b = Basis1D(k)
    h = 1.0 / N
    Mloc = np.array([[1.0]])
    for _ in range(d):
        Mloc = np.kron(h * b.M, Mloc)
    return sp.block_diag([Mloc] * (N ** d), format="csr")


class KronApply:
    """Matrix-free y = A x by the Kronecker form, sparse 1-D factors applied
    along each axis of the brick (global lexicographic layout internally)."""

    def __init__(self, d, k, N, sigma, kappa=1.0):
        self.d, self.k, self.N = d, k, N
        M, L = sipg_1d(k, N, sigma)
        self.M = sp.csr_matrix(M)
        self.L = sp.csr_matrix(kappa * L)
        self.perm = lex_of_cellwise(d, k, N)
        self.Nn = N * (k + 1)

    def _along(self, A1, X, axis):
        Xm = np.moveaxis(X, axis, 0)
        sh = Xm.shape
        Y = (A1 @ Xm.reshape(sh[0], -1)).reshape(sh)
        return np.moveaxis(Y, 0, axis)

    def to_lex(self, x):
        xl = np.empty_like(x)
        xl[self.perm] = x
        return xl

    def to_cellwise(self, xl):
        return xl[self.perm]

    def __call__(self, x):
        d, Nn = self.d, self.Nn
        X = self.to_lex(np.asarray(x, dtype=np.float64)).reshape((Nn,) * d)
        # axis (d-1-i) of the brick array is direction i
        Y = np.zeros_like(X)
        for dirn in range(d):
            T = X
            for i in range(d):
                T = self._along(self.L if i == dirn else self.M, T, d - 1 - i)
            Y += T
        return self.to_cellwise(Y.reshape(-1))


def apply_cells(d, k, N, sigma, x, cells, kappa=1.0):
    """(A x) restricted to the given cells (cell-wise indices), for meshes too
    large for a full oracle apply.  Each cell's rows of the Kronecker form only
    involve the cells within one step in every direction, so the product is
    taken on that 3^d-cell brick with the matching row/column blocks of the
    1-D matrices.  Returns an array (len(cells), (k+1)^d) in local
    lexicographic order."""
    M, L = sipg_1d(k, N, sigma)
    L = kappa * L
    n = k + 1
    nl = n ** d
    out = np.zeros((len(cells), nl))
    for j, c in enumerate(cells):
        ci = [(int(c) // N ** i) % N for i in range(d)]
        lo = [max(ci[i] - 1, 0) for i in range(d)]
        hi = [min(ci[i] + 1, N - 1) for i in range(d)]
        rows = [np.arange(ci[i] * n, (ci[i] + 1) * n) for i in range(d)]
        cols = [np.arange(lo[i] * n, (hi[i] + 1) * n) for i in range(d)]
        # gather the brick, axes ordered (slowest ... fastest) = (d-1 ... 0)
        shape = tuple((hi[i] - lo[i] + 1) * n for i in reversed(range(d)))
        X = np.zeros(shape)
        for cc in itertools.product(*[range(lo[i], hi[i] + 1) for i in reversed(range(d))]):
            cv = cc[::-1]  # cv[i] = cell coordinate in direction i
            cell = sum(cv[i] * N ** i for i in range(d))
            blk = x[cell * nl:(cell + 1) * nl].reshape((n,) * d)
            sl = tuple(slice((cv[i] - lo[i]) * n, (cv[i] - lo[i] + 1) * n) for i in reversed(range(d)))
            X[sl] = blk
        y = np.zeros((n,) * d)
        for dirn in range(d):
            T = X
            for i in range(d):
                F = (L if i == dirn else M)[np.ix_(rows[i], cols[i])]
                ax = d - 1 - i
                T = np.moveaxis(np.tensordot(F, T, axes=([1], [ax])), 0, ax)
            y += T
        out[j] = y.reshape(-1)
    return out
