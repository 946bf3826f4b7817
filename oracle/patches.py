"""Oracle (test infrastructure only): vertex patches, local spaces and colours
(Sec. 3.1, Fig. smoother, Fig. hermite_type, Fig. patch_coloring).

A patch is the set of the 2^d cells sharing an interior vertex v in
{1..N-1}^d; its cells have coordinates {v_i - 1, v_i} in direction i.  Along
direction i the patch carries 2n = 2k+2 nodes, patch-local index
p = a (left cell, node a) or p = n + a (right cell, node a).

Dirichlet local space V_j: the patch nodes minus those on the patch boundary
that lie on an interior mesh face.  Per direction the kept set is
{1..2k}, plus p = 0 when the patch touches the boundary x_i = 0 (v_i = 1) and
plus p = 2k+1 when it touches x_i = 1 (v_i = N-1); boundary-of-domain nodes
are kept so that they are smoothed at all.  V_j is the tensor product of the
per-direction kept sets; the domain of dependence of the paper-literal kernel
is all DoFs of the patch cells.

Clamped local space (Sec. 3.1, Fig. hermite_type): the patch functions with
v = 0 and dv/dn = 0 on the patch boundary.  Along one direction these are
the vectors of the two-cell patch whose value and derivative vanish at each
end that lies on an interior mesh face (2k - 2 of them for an interior
patch); at an end on the domain boundary nothing is clamped, for the same
reason the Dirichlet space keeps those nodes.  The d-D space is the tensor
product of the 1-D ones.

Colours: colour(v) = sum_i ((v_i - 1) mod 2) 2^i, i.e. 2^d colours; patches of
one colour share no cell, and colour 0 (all v_i odd) tiles the mesh by the
children of the coarse cells.
"""
import itertools

import numpy as np


def vertices(d, N):
    """Interior vertices, as arrays v[i] (direction i), x fastest ordering."""
    out = []
    for vv in itertools.product(range(1, N), repeat=d):
        out.append(vv[::-1])
    return np.array(out, dtype=np.int64).reshape(-1, d)


def colour(v):
    return int(sum(((v[i] - 1) % 2) << i for i in range(len(v))))


def kept_1d(k, N, vi):
    """Kept patch-local 1-D indices of the Dirichlet space along one direction."""
    keep = list(range(1, 2 * k + 1))
    if vi == 1:
        keep = [0] + keep
    if vi == N - 1:
        keep = keep + [2 * k + 1]
    return keep


def clamped_basis_1d(k, ptype):
    """Orthonormal basis (columns, shape (2k+2, m)) of the 1-D clamped space
    of a patch type: the null space of the end constraints v(end) = 0 and
    v'(end) = 0 at every end not on the domain boundary (type bit 0: the left
    end lies on x = 0, bit 1: the right end on x = 1).  Node values at the
    ends are the traces (Gauss-Lobatto end points); the derivative at the
    left end is phi'(0) . v on the left cell, at the right end phi'(1) . v on
    the right cell (reference cell; h only scales the constraint)."""
    import scipy.linalg as sla

    from .basis import Basis1D
    n = k + 1
    E = 2 * n
    bs = Basis1D(k)
    rows = []
    if not ptype & 1:
        r = np.zeros(E)
        r[0] = 1.0
        rows.append(r)
        r = np.zeros(E)
        r[:n] = bs.d0
        rows.append(r)
    if not ptype & 2:
        r = np.zeros(E)
        r[E - 1] = 1.0
        rows.append(r)
        r = np.zeros(E)
        r[n:] = bs.d1
        rows.append(r)
    if not rows:
        return np.eye(E)
    return sla.null_space(np.array(rows))


def patch_type_1d(N, vi):
    """0 interior, 1 touches x=0, 2 touches x=1, 3 both (only N = 2)."""
    return int(vi == 1) + 2 * int(vi == N - 1)


def patch_dofs(d, k, N, v):
    """Global (cell-wise) DoF index of every patch-tile node, as an array of
    shape (2n,)*d indexed [p_{d-1}, ..., p_0]."""
    n = k + 1
    nl = n ** d
    E = 2 * n
    idx = np.zeros((E,) * d, dtype=np.int64)
    for pt in itertools.product(range(E), repeat=d):
        p = pt[::-1]
        c = [v[i] - 1 + p[i] // n for i in range(d)]
        l = [p[i] % n for i in range(d)]
        cell = sum(c[i] * N ** i for i in range(d))
        loc = sum(l[i] * n ** i for i in range(d))
        idx[pt] = cell * nl + loc
    return idx


def kept_mask(d, k, N, v):
    """Boolean mask over the patch tile (indexed [p_{d-1},...,p_0]) of V_j."""
    E = 2 * (k + 1)
    m = np.ones((E,) * d, dtype=bool)
    for i in range(d):
        keep = np.zeros(E, dtype=bool)
        keep[kept_1d(k, N, v[i])] = True
        shape = [1] * d
        shape[d - 1 - i] = E
        m &= keep.reshape(shape)
    return m


def _tiles_vectorised(d, k, N, verts):
    """Global DoF indices of every patch tile, shape (P, 2n, ..., 2n) indexed
    [patch, p_{d-1}, ..., p_0] (the same index rule as `patch_dofs`)."""
    n = k + 1
    E = 2 * n
    P = len(verts)
    p = np.arange(E)
    cell = np.zeros((P,) + (1,) * d, dtype=np.int64)
    loc = np.zeros((1,) + (1,) * d, dtype=np.int64)
    for i in range(d):
        shape = [1] * (d + 1)
        shape[d - i] = E
        ci = (verts[:, i][:, None] - 1 + (p // n)[None, :])
        cell = cell + ci.reshape([P] + shape[1:]) * N ** i
        loc = loc + (p % n).reshape(shape) * n ** i
    return cell * n ** d + loc


def _masks_vectorised(d, k, N, verts):
    E = 2 * (k + 1)
    P = len(verts)
    m = np.ones((P,) + (E,) * d, dtype=bool)
    p = np.arange(E)
    for i in range(d):
        vi = verts[:, i][:, None]
        keep = ((p[None, :] >= 1) | (vi == 1)) & ((p[None, :] <= 2 * k) | (vi == N - 1))
        shape = [P] + [1] * d
        shape[d - i] = E
        m &= keep.reshape(shape)
    return m


class PatchSet:
    """All interior-vertex patches of a level with their tiles and colours."""

    def __init__(self, d, k, N):
        self.d, self.k, self.N = d, k, N
        self.verts = vertices(d, N)
        self.colours = np.zeros(len(self.verts), dtype=np.int64)
        for i in range(d):
            self.colours += ((self.verts[:, i] - 1) % 2) << i
        self.tiles = _tiles_vectorised(d, k, N, self.verts)
        self.masks = _masks_vectorised(d, k, N, self.verts)

    def of_colour(self, c):
        return np.nonzero(self.colours == c)[0]

    def vj(self, j):
        """Global DoF indices of V_j (in tile order)."""
        return self.tiles[j][self.masks[j]]

    def vbar(self, j):
        return self.tiles[j].reshape(-1)
