"""Oracle (test infrastructure only): one step of the colourised
multiplicative vertex-patch Schwarz smoother S(x, b) of Alg. 1 (Sec. 3.1),
with local solves by fast diagonalisation (Sec. 3.2, eqs. inverse2d,
inverse3d, fast_inverse).

For every colour in the given order, and every patch j of that colour:
    r_j = local residual on V_j
    x|V_j += A[V_j, V_j]^{-1} r_j
Local spaces and residuals:
  'exact'  Dirichlet kernel: V_j drops the patch-boundary nodes on interior
           faces; r_j = (b - A x)|V_j, the residual of eq. (residual)
           restricted to V_j;
  'local'  the paper-literal Dirichlet kernel: r_j = b|V_j - A[V_j, Vbar_j]
           x|Vbar_j with Vbar_j the patch cells only (inconsistent by design);
  'full'   the Full kernel (Sec. 3.1): V_j = every node of the patch cells;
           its domain of dependence reaches into the face-neighbour cells,
           which belong to other patches of the same colour, so the residual
           is updated globally: r = b - A x once per colour, and every patch
           of the colour corrects from that r (additive inside a colour,
           multiplicative across colours).
  'clamped' the clamped kernel (Sec. 3.1): V_j = patch functions with zero
           value and normal derivative on the patch boundary (a subspace of
           the patch space, basis C = tensor product of the 1-D bases of
           `clamped_basis_1d`); r_j = C^T (b - A x)|patch and the correction
           C (C^T A_patch C)^{-1} r_j.  The face terms that couple the patch
           to outside cells act on rows that C^T annihilates, so r_j only
           depends on the patch cells and same-colour patches are independent.
All use the global matrix entries restricted to the index sets.

`smooth_dense` is the definition itself: patches visited one after another,
residual rows taken from the assembled sparse matrix, dense local solves.
`smooth_fd` processes one colour at a time (same-colour patches share no
cell and no patch reads another same-colour write set, so this equals the
sequential order) and inverts A[V_j,V_j] = sum_i (x) (M~ .. L~_i .. M~) by
fast diagonalisation: L~ S = M~ S Lambda, S^T M~ S = I,
A_j^{-1} = ((x) S) (sum_i Lambda_i)^{-1} ((x) S^T).
"""
import itertools

import numpy as np
import scipy.linalg as sla

from .basis import Basis1D
from .patches import PatchSet, _tiles_vectorised, clamped_basis_1d, kept_1d, patch_type_1d
from .sipg import KronApply, sipg_1d


def smooth_dense(A, x, b, ps, order, mode="exact", kappa=1.0):
    """Sequential by-definition smoothing step (in place on a copy of x); kappa
    is the coefficient A was built with (the 'local' residual needs it)."""
    x = np.array(x, dtype=np.float64, copy=True)
    A = A.tocsr()
    for c in order:
        if mode == "full":
            r = b - A @ x
            for j in ps.of_colour(c):
                V = ps.vbar(j)
                x[V] += np.linalg.solve(A[V][:, V].toarray(), r[V])
            continue
        if mode == "clamped":
            for j in ps.of_colour(c):
                V = ps.vbar(j)  # tile order: [p_{d-1}, ..., p_0], p_0 fastest
                C = np.ones((1, 1))
                for i in reversed(range(ps.d)):
                    C = np.kron(C, clamped_basis_1d(ps.k, patch_type_1d(ps.N, ps.verts[j][i])))
                r = C.T @ (b[V] - A[V] @ x)
                x[V] += C @ np.linalg.solve(C.T @ A[V][:, V].toarray() @ C, r)
            continue
        for j in ps.of_colour(c):
            V = ps.vj(j)
            if mode == "exact":
                r = b[V] - A[V] @ x
            elif mode == "local":
                Vb = ps.vbar(j)
                T = outer_face_consistency(ps.d, ps.k, ps.N, ps.verts[j], kappa)[ps.masks[j].reshape(-1)]
                r = b[V] - A[V][:, Vb] @ x[Vb] - T @ x[Vb]
            else:
                raise ValueError(mode)
            Ajj = A[V][:, V].toarray()
            x[V] += np.linalg.solve(Ajj, r)
    return x


def outer_face_consistency(d, k, N, v, kappa=1.0):
    """T[test, trial] = kappa/2 int_F u_P (n_P . grad v_P) summed over the faces
    F of patch v that lie inside the domain on the patch boundary, for u, v in
    the patch cell P next to F (n_P its outward normal): the inside half of
    the SIPG term -[[u]].{grad v}, which the global matrix carries with the
    opposite sign.  Dense over the patch tile in tile order, integrated by
    the face quadrature of the operator assembly."""
    from .sipg import _face_tabulation
    n = k + 1
    nl = n ** d
    E = 2 * n
    tile = _tiles_vectorised(d, k, N, np.array([v]))[0].reshape(-1)
    pos = {int(g): p for p, g in enumerate(tile)}
    T = np.zeros((E ** d, E ** d))
    for i in range(d):
        for side in (0, 1):
            c_i = v[i] - 1 if side == 0 else v[i]  # patch layer next to that face
            if (side == 0 and c_i == 0) or (side == 1 and c_i == N - 1):
                continue  # domain boundary: Nitsche terms stay
            val, grad, wf = _face_tabulation(d, k, N, i, side)
            nrm = np.zeros(d)
            nrm[i] = -1.0 if side == 0 else 1.0
            blk = 0.5 * kappa * np.einsum("g,gbq,aq,q->ba", nrm, grad, val, wf)
            for rest in itertools.product(*[(v[m] - 1, v[m]) for m in range(d) if m != i]):
                cc = list(rest)
                cc.insert(i, c_i)
                cell = sum(cc[m] * N ** m for m in range(d))
                idx = np.array([pos[cell * nl + a] for a in range(nl)])
                T[np.ix_(idx, idx)] += blk
    return T


class PatchFD:
    """1-D patch matrices and their generalised eigenpairs for every patch
    type along one direction (interior, touching x=0, touching x=1, both):
    S, lam on the Dirichlet local space, Sf, lamf on the whole patch (Full
    kernel), Sc = C S_C, lamc on the clamped space with basis C; Llit the
    patch matrix of the paper's Dirichlet residual (interior-end consistency
    halves removed)."""

    def __init__(self, k, N, sigma, kappa=1.0):
        M, L = sipg_1d(k, N, sigma)
        L = kappa * L
        n = k + 1
        self.k, self.N = k, N
        self.S, self.lam, self.Mt, self.Lt, self.keep = {}, {}, {}, {}, {}
        self.Mpatch, self.Lpatch, self.Sf, self.lamf = {}, {}, {}, {}
        self.Sc, self.lamc, self.Llit = {}, {}, {}
        bs = Basis1D(k)
        h = 1.0 / N
        for vi in range(1, N):
            t = patch_type_1d(N, vi)
            if t in self.S:
                continue
            s = slice((vi - 1) * n, (vi + 1) * n)
            Mp, Lp = M[s, s], L[s, s]
            keep = kept_1d(k, N, vi)
            Mt, Lt = Mp[np.ix_(keep, keep)], Lp[np.ix_(keep, keep)]
            lam, S = sla.eigh(Lt, Mt)
            self.S[t], self.lam[t] = S, lam
            self.Mt[t], self.Lt[t], self.keep[t] = Mt, Lt, keep
            self.Mpatch[t], self.Lpatch[t] = Mp, Lp
            Ll = Lp.copy()
            if not t & 1:  # left end inside the domain: drop +1/2 v'(x+) u(x+)
                Ll[:n, 0] -= kappa * 0.5 * bs.d0 / h
            if not t & 2:  # right end: drop -1/2 v'(x-) u(x-)
                Ll[n:, 2 * n - 1] += kappa * 0.5 * bs.d1 / h
            self.Llit[t] = Ll
            self.lamf[t], self.Sf[t] = sla.eigh(Lp, Mp)
            C = clamped_basis_1d(k, t)
            if C.shape[1] > 0:
                lc, Sc = sla.eigh(C.T @ Lp @ C, C.T @ Mp @ C)
                self.lamc[t], self.Sc[t] = lc, C @ Sc


def _along(A1, T, axis):
    """Contract the 1-D matrix A1 (rows out, cols in) along tile axis `axis` of a
    batch of tiles T (axis 0 is the patch batch)."""
    Tm = np.moveaxis(T, axis, -1)
    Y = Tm @ A1.T
    return np.moveaxis(Y, -1, axis)


def fd_inverse(fd, types, R, space="dirichlet"):
    """Apply A_j^{-1} by fast diagonalisation to a batch of tiles R (shape
    (np, n_{d-1}, ..., n_0)) of patches sharing the type tuple `types`
    (types[i] = type along direction i).  space 'dirichlet': R holds the kept
    set; 'full': the whole tile; 'clamped': the whole tile, and S = C S_C maps
    between tile values and the eigenbasis of the clamped space."""
    S, lm = {"dirichlet": (fd.S, fd.lam), "full": (fd.Sf, fd.lamf),
             "clamped": (fd.Sc, fd.lamc)}[space]
    d = len(types)
    T = R
    for i in range(d):
        T = _along(S[types[i]].T, T, d - i)
    lam = np.zeros(T.shape[1:])
    for i in range(d):
        shape = [1] * d
        shape[d - 1 - i] = -1
        lam = lam + lm[types[i]].reshape(shape)
    T = T / lam[None]
    for i in range(d):
        T = _along(S[types[i]], T, d - i)
    return T


class FDSmoother:
    """Vectorised smoothing step for one level (cell-wise layout)."""

    def __init__(self, d, k, N, sigma, kappa=1.0, mode="exact", apply=None):
        if mode == "clamped" and k < 3:
            # per direction a cell lies in two patches whose clamped spaces
            # together span 2(k - 1) of the k + 1 cell polynomials
            raise ValueError("the clamped spaces cover Q_k only for k >= 3")
        self.d, self.k, self.N, self.mode = d, k, N, mode
        self.ps = PatchSet(d, k, N)
        self.fd = PatchFD(k, N, sigma, kappa)
        self.apply = apply if apply is not None else KronApply(d, k, N, sigma, kappa)
        # group patches by (colour, type tuple)
        self.groups = {}
        for j, v in enumerate(self.ps.verts):
            types = tuple(patch_type_1d(N, v[i]) for i in range(d))
            self.groups.setdefault((int(self.ps.colours[j]), types), []).append(j)
        self.groups = {key: np.array(val) for key, val in self.groups.items()}

    def _kept_slices(self, types):
        if self.mode in ("full", "clamped"):
            return tuple(np.arange(2 * (self.k + 1)) for _ in range(self.d))
        return tuple(np.array(self.fd.keep[types[i]]) for i in reversed(range(self.d)))

    def step(self, x, b, order):
        d = self.d
        x = np.array(x, dtype=np.float64, copy=True)
        for c in order:
            r = b - self.apply(x) if self.mode in ("exact", "full", "clamped") else None
            updates = []
            for (cc, types), js in self.groups.items():
                if cc != c:
                    continue
                tiles = self.ps.tiles[js]  # (np, E,...,E)
                ks = self._kept_slices(types)
                sub = tiles[(slice(None),) + np.ix_(*ks)]
                if self.mode in ("exact", "full", "clamped"):
                    R = r[sub]
                else:
                    X = x[tiles]
                    AX = np.zeros_like(X)
                    for dirn in range(d):
                        T = X
                        for i in range(d):
                            mat = self.fd.Llit[types[i]] if i == dirn else self.fd.Mpatch[types[i]]
                            T = _along(mat, T, d - i)
                        AX += T
                    R = b[sub] - AX[(slice(None),) + np.ix_(*ks)]
                space = self.mode if self.mode in ("full", "clamped") else "dirichlet"
                updates.append((sub, fd_inverse(self.fd, types, R, space)))
            for sub, dx in updates:
                x[sub] += dx
        return x


def colour_orders(d):
    asc = list(range(2 ** d))
    return asc, asc[::-1]


def colour_disjointness(ps):
    """Race-freedom of one colour: write sets pairwise disjoint, and no patch
    reads (tile plus the face-neighbour nodes the exact residual needs) another
    same-colour patch's write set.  Returns True when every colour passes."""
    d, k, N = ps.d, ps.k, ps.N
    n = k + 1
    nl = n ** d
    for c in range(2 ** d):
        js = ps.of_colour(c)
        owner = {}
        for j in js:
            for g in ps.vj(j):
                if g in owner:
                    return False
                owner[int(g)] = j
        for j in js:
            reads = set(int(g) for g in ps.vbar(j))
            v = ps.verts[j]
            # trace nodes of face-neighbour cells across the patch boundary
            for i in range(d):
                for side in (-1, 1):
                    ci = v[i] - 2 if side < 0 else v[i] + 1
                    if ci < 0 or ci >= N:
                        continue
                    for rest in itertools.product(*[(v[m] - 1, v[m]) for m in range(d) if m != i]):
                        cc = list(rest)
                        cc.insert(i, ci)
                        cell = sum(cc[m] * N ** m for m in range(d))
                        for loc in range(nl):
                            li = (loc // n ** i) % n
                            if li == (n - 1 if side < 0 else 0):
                                reads.add(cell * nl + loc)
            for g in reads:
                if g in owner and owner[g] != j:
                    return False
    return True
