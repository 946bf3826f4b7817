"""CPU checks of libdgmg.so that need no GPU: it loads, exports every entry
point of include/dgmg.h, validates arguments before any device work, and its
host-side FP64 tables (node coordinates, fast-diagonalisation eigenpairs)
agree with the oracle's independent construction."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.patches import clamped_basis_1d, kept_1d
from oracle.rhs import node_coords as oracle_coords
from oracle.smoother import PatchFD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgmg.h")

dgmg = pytest.importorskip("paper_2405_18982_amd.dgmg")
if not os.path.exists(dgmg.LIB_PATH):
    pytest.skip("libdgmg.so not built", allow_module_level=True)


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgmg_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = dgmg.lib()
    names = header_symbols()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    # the binding's table mirrors the header exactly
    assert sorted(dgmg.SIGNATURES) == names


def _ctx(dim, k, L, sigma=None, kappa=1.0):
    ctx = ctypes.c_void_p()
    sigma = 2.0 * (k + 1) ** 2 if sigma is None else sigma
    st = dgmg.lib().dgmg_setup_mesh(dim, k, L, sigma, kappa, ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("args", [(1, 2, 2), (4, 2, 2), (2, 0, 2), (2, 8, 2), (3, 3, 0),
                                  (3, 7, 10)])
def test_setup_mesh_rejects_bad_arguments(args):
    st, ctx = _ctx(*args)
    assert st == -1 and not ctx.value


def test_setup_mesh_rejects_bad_penalty_and_kappa():
    assert _ctx(2, 2, 2, sigma=-1.0)[0] == -1
    assert _ctx(2, 2, 2, kappa=0.0)[0] == -1
    assert _ctx(2, 2, 2, kappa=float("nan"))[0] == -1


def test_calls_before_setup_levels_are_state_errors():
    st, ctx = _ctx(2, 2, 2)
    assert st == 0
    lib = dgmg.lib()
    assert lib.dgmg_apply_sipg(ctx, 2, None, None, 1) == -6
    assert lib.dgmg_level_ndofs(ctx, 2) == 8 * 8 * 9
    assert lib.dgmg_level_ndofs(ctx, 3) == -1
    assert lib.dgmg_level_cells(ctx, 0) == 2
    assert lib.dgmg_destroy(ctx) == 0


@pytest.mark.parametrize("dim,k,l", [(2, 2, 2), (3, 3, 1), (2, 5, 1)])
def test_node_coords_match_oracle(dim, k, l):
    st, ctx = _ctx(dim, k, l)
    lib = dgmg.lib()
    n = lib.dgmg_level_ndofs(ctx, l)
    xyz = np.zeros(n * dim)
    assert lib.dgmg_node_coords(ctx, l, xyz.ctypes.data) == 0
    ref = oracle_coords(dim, k, 2 ** (l + 1))
    assert np.abs(xyz.reshape(-1, dim) - ref).max() < 1e-15
    lib.dgmg_destroy(ctx)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("sigma_rule", ["config", "paper"])
def test_patch_eigenpairs_match_oracle(k, sigma_rule):
    sigma = 2.0 * (k + 1) ** 2 if sigma_rule == "config" else 2.0 * k * (k + 1)
    for N, types in ((8, (0, 1, 2)), (2, (3,))):
        h = 1.0 / N
        fd = PatchFD(k, N, sigma)
        for t in types:
            S, lam = dgmg.patch_eigen(k, sigma, t)
            keep = kept_1d(k, N, {0: 2, 1: 1, 2: N - 1, 3: 1}[t])
            m = len(keep)
            Sk = S[np.ix_(keep, list(range(m)))]
            # unused slots: zero rows/columns and infinite eigenvalues
            assert np.all(np.isinf(lam[m:]))
            assert np.all(S[np.setdiff1d(np.arange(S.shape[0]), keep)] == 0)
            # reference (h = 1) patch matrices from the oracle's global ones
            Lt = fd.Lt[t] * h
            Mt = fd.Mt[t] / h
            assert np.allclose(Sk.T @ Mt @ Sk, np.eye(m), atol=1e-11)
            Linv = Sk @ np.diag(1.0 / lam[:m]) @ Sk.T
            assert np.abs(Linv @ Lt - np.eye(m)).max() < 1e-10
            if t == 0:
                # interior patch: columns q < k even, k <= q < 2k odd under
                # the reflection of the patch, exactly (the kernels contract
                # half lines on that structure)
                E = 2 * (k + 1)
                R = S[::-1, :]
                assert np.array_equal(R[:, :k], S[:, :k])
                assert np.array_equal(R[:, k:2 * k], -S[:, k:2 * k])
            # Full kernel: the whole patch, every slot used
            Sf, lamf = dgmg.patch_eigen(k, sigma, t, dgmg.SMOOTH_FULL)
            E = 2 * (k + 1)
            assert np.all(np.isfinite(lamf)) and np.all(lamf > 0)
            Lp, Mp = fd.Lpatch[t] * h, fd.Mpatch[t] / h
            assert np.allclose(Sf.T @ Mp @ Sf, np.eye(E), atol=1e-11)
            Lfinv = Sf @ np.diag(1.0 / lamf) @ Sf.T
            assert np.abs(Lfinv @ Lp - np.eye(E)).max() < 1e-10
            if k >= 3:
                # clamped space: C (C^T L C)^{-1} C^T does not depend on the
                # basis C; the oracle's is orthonormal, the library's is not
                Sc, lamc = dgmg.patch_eigen(k, sigma, t, dgmg.SMOOTH_CLAMPED)
                Co = clamped_basis_1d(k, t)
                mc = Co.shape[1]
                assert np.all(np.isinf(lamc[mc:])) and np.all(Sc[:, mc:] == 0)
                Scm = Sc[:, :mc]
                assert np.allclose(Scm.T @ Mp @ Scm, np.eye(mc), atol=1e-10)
                ref = Co @ np.linalg.solve(Co.T @ Lp @ Co, Co.T)
                got = Scm @ np.diag(1.0 / lamc[:mc]) @ Scm.T
                assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
