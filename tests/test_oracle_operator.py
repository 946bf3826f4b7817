"""Pins of the oracle's SIPG operator, transfers and patch index sets
(Sec. 2.1-2.2, Sec. 3, Sec. 3.1) against independent constructions,
closed-form solutions and invariants."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import sipg as osipg
from oracle.fdsolve import GlobalFD
from oracle.patches import PatchSet
from oracle.rhs import (bubble_load, bubble_solution, interpolate, l2_error, load_vector,
                        sine_load, sine_solution)
from oracle.sipg import KronApply, assemble_quadrature, kron_operator, mass_operator
from oracle.smoother import colour_disjointness
from oracle.transfer import prolongation

CASES = [(2, 1, 3), (2, 2, 3), (2, 3, 2), (2, 5, 2), (3, 1, 2), (3, 2, 2), (3, 3, 2)]


def sig(k):
    return 2.0 * (k + 1) ** 2


@pytest.mark.parametrize("d,k,N", CASES)
def test_quadrature_assembly_equals_kronecker(d, k, N):
    A1 = kron_operator(d, k, N, sig(k), kappa=1.3)
    A2 = assemble_quadrature(d, k, N, sig(k), kappa=1.3)
    assert abs(A1 - A2).max() <= 1e-14 * abs(A1).max()


@pytest.mark.parametrize("d,k,N", CASES)
def test_symmetric_positive_definite(d, k, N):
    A = kron_operator(d, k, N, sig(k))
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    if A.shape[0] <= 2000:
        assert np.linalg.eigvalsh(A.toarray())[0] > 0
    # spectrum of A (relative to the mass) is {sum_i lambda_i}: min > 0 certifies SPD
    fd = GlobalFD(d, k, N, sig(k))
    assert d * fd.eigenvalues_1d().min() > 0


def test_paper_penalty_also_spd():
    for k in (1, 2, 3, 5, 7):
        fd = GlobalFD(3, k, 8, 2.0 * k * (k + 1))
        assert fd.eigenvalues_1d().min() > 0


@pytest.mark.parametrize("d,k,N", [(2, 2, 4), (2, 3, 3), (2, 4, 2), (3, 2, 3), (3, 3, 2)])
def test_consistency_reproduces_bubble(d, k, N):
    # u = prod x(1-x) is in V_h for k >= 2 and vanishes on the boundary; SIPG is
    # consistent, so A u_I = b exactly (up to round-off).
    A = kron_operator(d, k, N, sig(k))
    b = load_vector(d, k, N, bubble_load)
    u = interpolate(d, k, N, bubble_solution)
    assert np.abs(A @ u - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_l2_convergence_rate(k):
    errs = []
    Ns = (8, 16, 32)
    for N in Ns:
        fd = GlobalFD(2, k, N, sig(k))
        errs.append(l2_error(2, k, N, fd.solve(load_vector(2, k, N, sine_load)), sine_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(rates[-1] - (k + 1)) < 0.15, rates


@pytest.mark.parametrize("d,k,N", [(2, 2, 4), (2, 5, 2), (3, 2, 2), (3, 3, 2)])
def test_global_fd_equals_sparse_direct(d, k, N):
    A = kron_operator(d, k, N, sig(k), kappa=0.7)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(A.shape[0])
    x1 = spla.spsolve(A.tocsc(), b)
    x2 = GlobalFD(d, k, N, sig(k), kappa=0.7).solve(b)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)


@pytest.mark.parametrize("d,k,N", [(2, 3, 8), (3, 3, 4), (3, 2, 6)])
def test_matrix_free_apply_equals_sparse(d, k, N):
    A = kron_operator(d, k, N, sig(k), kappa=2.0)
    x = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    y = KronApply(d, k, N, sig(k), kappa=2.0)(x)
    assert np.abs(y - A @ x).max() <= 1e-14 * np.abs(A @ x).max()


@pytest.mark.parametrize("d,k,Nc", [(2, 2, 2), (2, 3, 4), (3, 2, 2), (3, 3, 2)])
def test_prolongation_is_embedding(d, k, Nc):
    P = prolongation(d, k, Nc)
    Mf, Mc = mass_operator(d, k, 2 * Nc), mass_operator(d, k, Nc)
    # P^T M_f P = M_c because V_c is a subspace of V_f
    assert abs(P.T @ Mf @ P - Mc).max() <= 1e-15 * abs(Mc).max() * 10
    # interpolant of a Q_k polynomial maps to its fine interpolant
    def poly(X):
        return np.prod(X ** k + 0.3 * X, axis=1) + 1.0
    uc = interpolate(d, k, Nc, poly)
    uf = interpolate(d, k, 2 * Nc, poly)
    assert np.abs(P @ uc - uf).max() <= 1e-13


@pytest.mark.parametrize("d,k,N", [(2, 2, 4), (2, 1, 6), (3, 1, 4), (3, 2, 4)])
def test_colours_are_race_free(d, k, N):
    ps = PatchSet(d, k, N)
    assert len(set(ps.colours.tolist())) == 2 ** d
    assert colour_disjointness(ps)


def test_colour_check_catches_a_patch_with_the_wrong_colour():
    """Planted mistake: a patch next to a colour-0 patch relabelled colour 0.
    Their Dirichlet write sets share the interior nodes of the common cells,
    so the race-freedom check must fail."""
    for d, k, N in [(2, 2, 4), (3, 1, 4)]:
        ps = PatchSet(d, k, N)
        j0 = next(j for j, v in enumerate(ps.verts) if all(c == 1 for c in v))
        nb = next(j for j, v in enumerate(ps.verts)
                  if v[0] == 2 and all(c == 1 for c in v[1:]))
        assert ps.colours[j0] == 0 and ps.colours[nb] != 0
        ps.colours[nb] = 0
        assert not colour_disjointness(ps)


def test_colour_check_catches_a_kept_interior_end_node():
    """Planted mistake: one interior patch keeps a patch-boundary node on an
    interior mesh face in its write set.  That node is the face trace that the
    exact residual of the same-colour patch two cells over reads, so the
    check must fail; the same patch set without the change passes."""
    d, k, N = 2, 2, 6
    ps = PatchSet(d, k, N)
    assert colour_disjointness(ps)
    j = next(j for j, v in enumerate(ps.verts) if tuple(v) == (3, 3))
    E = 2 * (k + 1)
    m = ps.masks[j].reshape(E, E)  # (y, x) in tile order
    assert not m[3, E - 1]
    m[3, E - 1] = True             # the x = right end of a middle tile row
    ps.masks[j] = m.reshape(ps.masks[j].shape)
    assert not colour_disjointness(ps)


def test_colour0_tiles_mesh_and_dirichlet_sizes():
    # Q3, 3-D: V_j of an interior patch is 6^3, the patch tile 8^3 (Sec. 3.3)
    ps = PatchSet(3, 3, 4)
    j = next(j for j, v in enumerate(ps.verts) if tuple(v) == (2, 2, 2))
    assert ps.masks[j].sum() == 6 ** 3 and ps.tiles[j].size == 8 ** 3
    # colour 0 patches cover every cell exactly once
    cells = np.concatenate([np.unique(ps.tiles[j] // 64) for j in ps.of_colour(0)])
    assert sorted(cells.tolist()) == list(range(64))
    # every DoF is in some V_j (boundary-of-domain nodes included)
    allv = np.unique(np.concatenate([ps.vj(j) for j in range(len(ps.verts))]))
    assert len(allv) == 64 * 64


def test_planted_sign_error_is_caught(monkeypatch):
    """A sign slip in the 1-D consistency term must break bubble reproduction."""
    orig = osipg.sipg_1d

    def wrong(k, N, sigma):
        M, L = orig(k, N, sigma)
        from oracle.basis import Basis1D
        b = Basis1D(k)
        n = k + 1
        h = 1.0 / N
        s = slice(n, 2 * n)
        L[s, s] -= (np.outer(b.e0, b.d0) + np.outer(b.d0, b.e0)) / h  # flip one face term
        return M, L

    monkeypatch.setattr(osipg, "sipg_1d", wrong)
    d, k, N = 2, 2, 4
    A = osipg.kron_operator(d, k, N, sig(k))
    b = load_vector(d, k, N, bubble_load)
    u = interpolate(d, k, N, bubble_solution)
    assert np.abs(A @ u - b).max() > 1e-3 * np.abs(b).max()
    A2 = assemble_quadrature(d, k, N, sig(k))
    assert abs(A - A2).max() > 1e-3 * abs(A2).max()


@pytest.mark.parametrize("d,k,N", [(2, 2, 4), (3, 1, 4), (3, 2, 3)])
def test_vectorised_patch_indices_equal_loop_definition(d, k, N):
    from oracle.patches import colour, kept_mask, patch_dofs
    ps = PatchSet(d, k, N)
    for j, v in enumerate(ps.verts):
        assert np.array_equal(ps.tiles[j], patch_dofs(d, k, N, v))
        assert np.array_equal(ps.masks[j], kept_mask(d, k, N, v))
        assert ps.colours[j] == colour(v)


@pytest.mark.parametrize("d,k,N", [(2, 3, 6), (3, 2, 4), (3, 4, 3)])
def test_sampled_cell_apply_equals_full_apply(d, k, N):
    from oracle.sipg import apply_cells
    x = np.random.default_rng(8).uniform(-1, 1, N ** d * (k + 1) ** d)
    y = KronApply(d, k, N, sig(k), kappa=1.7)(x).reshape(N ** d, -1)
    cells = np.arange(N ** d)
    got = apply_cells(d, k, N, sig(k), x, cells, kappa=1.7)
    assert np.abs(got - y).max() <= 1e-13 * np.abs(y).max()
