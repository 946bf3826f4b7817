"""GPU parity of every libdgmg entry point against the FP64 oracle, on the
same seeded inputs, through the C ABI.  Tolerances: FP64 kernels
|gpu - oracle|_2 <= 1e-12 |oracle|_2 and max-abs <= 1e-11 max|oracle|;
FP32 kernels 2e-5 relative (single-precision rounding of O(k^2) terms)."""
import sys

import numpy as np
import pytest

from oracle.multigrid import Hierarchy
from oracle.fdsolve import GlobalFD
from oracle.rhs import interpolate
from oracle.sipg import KronApply, kron_operator, mass_operator
from oracle.smoother import FDSmoother
from oracle.transfer import prolongation
from paper_2405_18982_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_18982_amd import dgmg  # noqa: E402

# (dim, k, L): small meshes spanning every patch type, ragged last workgroups
# (npatch not a multiple of the patches per block) and several levels
SMALL = [(2, 1, 3), (2, 2, 2), (2, 5, 2), (2, 7, 1), (3, 1, 2), (3, 2, 2), (3, 3, 2), (3, 4, 1),
         (3, 7, 1)]

_probs = {}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problem(dim, k, L, precision=64, variant=0, nrhs_max=2, kappa=1.0):
    key = (dim, k, L, precision, variant, nrhs_max, kappa)
    if key not in _probs:
        _probs[key] = dgmg.Problem(dim, k, L, kappa=kappa, precision=precision, variant=variant,
                                   nrhs_max=nrhs_max)
    return _probs[key]


def cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_load(dim, k, N):
    """Interpolated sine load b = M I_h f built by the oracle (an input to
    both sides; never taken from the library)."""
    return mass_operator(dim, k, N) @ interpolate(dim, k, N, inputs.sine_load)


def close(got, ref, rtol=1e-12, mtol=1e-11):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    nr = np.linalg.norm(ref)
    err = np.linalg.norm(got - ref)
    assert err <= rtol * max(nr, 1e-300), f"rel l2 err {err / nr:.3e}"
    assert np.abs(got - ref).max() <= mtol * max(np.abs(ref).max(), 1e-300)


@pytest.mark.parametrize("dim,k,L", SMALL)
def test_apply_fp64_all_levels(dim, k, L):
    note(f"apply fp64 d={dim} k={k} L={L}")
    sig = inputs.sigma_of(k)
    prob = problem(dim, k, L, kappa=1.0)
    for l in range(L + 1):
        N = 2 ** (l + 1)
        X = inputs.uniform(100 + l, (2, prob.ndofs(l)))
        Y = host(prob.apply(cuda(X), level=l))
        A = kron_operator(dim, k, N, sig)
        for j in range(2):
            close(Y[j], A @ X[j])


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2), (3, 7, 1)])
def test_apply_kappa_scaling(dim, k, L):
    note(f"apply kappa d={dim} k={k}")
    prob = problem(dim, k, L, kappa=0.37, nrhs_max=1)
    X = inputs.uniform(5, prob.ndofs())
    Y = host(prob.apply(cuda(X)))
    close(Y, KronApply(dim, k, 2 ** (L + 1), inputs.sigma_of(k), kappa=0.37)(X))


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2), (3, 7, 1), (3, 4, 1)])
def test_apply_fp32(dim, k, L):
    note(f"apply fp32 d={dim} k={k}")
    prob = problem(dim, k, L)
    X = inputs.uniform(7, prob.ndofs()).astype(np.float32).astype(np.float64)
    Y = host(prob.apply(cuda(X, torch.float32)))
    close(Y, kron_operator(dim, k, 2 ** (L + 1), inputs.sigma_of(k)) @ X, rtol=2e-5, mtol=2e-5)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2)])
def test_mass(dim, k, L):
    note(f"mass d={dim} k={k}")
    prob = problem(dim, k, L)
    X = inputs.uniform(8, prob.ndofs())
    close(host(prob.mass(cuda(X))), mass_operator(dim, k, 2 ** (L + 1)) @ X)


@pytest.mark.parametrize("dim,k,L", SMALL)
@pytest.mark.parametrize("variant", ["exact", "local"])
def test_smooth_fp64(dim, k, L, variant):
    note(f"smooth fp64 d={dim} k={k} L={L} {variant}")
    vid = 0 if variant == "exact" else 1
    prob = problem(dim, k, L, variant=vid)
    sig = inputs.sigma_of(k)
    for l in range(1, L + 1):
        N = 2 ** (l + 1)
        fs = FDSmoother(dim, k, N, sig, mode=variant)
        X = inputs.uniform(200 + l, (2, prob.ndofs(l)))
        B = inputs.uniform(300 + l, (2, prob.ndofs(l)))
        for reverse in (False, True):
            order = list(range(2 ** dim))[::-1] if reverse else list(range(2 ** dim))
            Xg = cuda(X)
            prob.smooth(Xg, cuda(B), level=l, reverse=reverse)
            G = host(Xg)
            for j in range(2):
                close(G[j], fs.step(X[j], B[j], order))


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2), (3, 7, 1)])
def test_smooth_fp32(dim, k, L):
    note(f"smooth fp32 d={dim} k={k}")
    prob = problem(dim, k, L)
    fs = FDSmoother(dim, k, 2 ** (L + 1), inputs.sigma_of(k))
    X = inputs.uniform(11, prob.ndofs()).astype(np.float32).astype(np.float64)
    B = inputs.uniform(12, prob.ndofs()).astype(np.float32).astype(np.float64)
    Xg = cuda(X, torch.float32)
    prob.smooth(Xg, cuda(B, torch.float32))
    ref = fs.step(X, B, list(range(2 ** dim)))
    close(host(Xg), ref, rtol=5e-5, mtol=5e-4)


@pytest.mark.parametrize("dim,k,L", SMALL)
def test_restrict_and_prolongate(dim, k, L):
    note(f"transfer d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    sig = inputs.sigma_of(k)
    for l in range(1, L + 1):
        N = 2 ** (l + 1)
        A = kron_operator(dim, k, N, sig)
        P = prolongation(dim, k, N // 2)
        X = inputs.uniform(400 + l, (2, prob.ndofs(l)))
        B = inputs.uniform(500 + l, (2, prob.ndofs(l)))
        Xc = inputs.uniform(600 + l, (2, prob.ndofs(l - 1)))
        Bc = host(prob.restrict_residual(cuda(X), cuda(B), level=l))
        Xg = cuda(X)
        prob.prolongate_add(cuda(Xc), Xg, level=l)
        Xp = host(Xg)
        for j in range(2):
            close(Bc[j], P.T @ (B[j] - A @ X[j]))
            close(Xp[j], X[j] + P @ Xc[j])


@pytest.mark.parametrize("dim,k,L", [(3, 2, 3), (3, 4, 2), (3, 5, 1), (3, 6, 1)])
def test_restrict_residual_register_face_degrees(dim, k, L):
    # 3-D degrees whose restriction runs on the register-face operator: every
    # level, three right-hand sides, interior and boundary patches
    note(f"restrict d={dim} k={k} L={L}")
    prob = problem(dim, k, L, nrhs_max=4)
    sig = inputs.sigma_of(k)
    for l in range(1, L + 1):
        N = 2 ** (l + 1)
        A = kron_operator(dim, k, N, sig)
        P = prolongation(dim, k, N // 2)
        X = inputs.uniform(700 + l, (3, prob.ndofs(l)))
        B = inputs.uniform(800 + l, (3, prob.ndofs(l)))
        Bc = host(prob.restrict_residual(cuda(X), cuda(B), level=l))
        for j in range(3):
            close(Bc[j], P.T @ (B[j] - A @ X[j]))


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 5), (3, 1), (3, 3), (3, 7)])
def test_coarse_solve(dim, k):
    note(f"coarse d={dim} k={k}")
    prob = problem(dim, k, 1)
    A0 = kron_operator(dim, k, 2, inputs.sigma_of(k)).toarray()
    B = inputs.uniform(13, (2, prob.ndofs(0)))
    X = host(prob.coarse_solve(cuda(B)))
    for j in range(2):
        close(X[j], np.linalg.solve(A0, B[j]), rtol=1e-11, mtol=1e-10)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (2, 5, 3), (3, 2, 2), (3, 3, 2), (3, 7, 1)])
def test_vcycle_fp64(dim, k, L):
    note(f"vcycle fp64 d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    H = Hierarchy(dim, k, L, inputs.sigma_of(k))
    B = inputs.uniform(14, (2, prob.ndofs()))
    X = host(prob.vcycle(cuda(B)))
    for j in range(2):
        close(X[j], H.vcycle(B[j]), rtol=1e-11, mtol=1e-10)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2)])
def test_vcycle_fp32(dim, k, L):
    note(f"vcycle fp32 d={dim} k={k}")
    prob = problem(dim, k, L, precision=32)
    H = Hierarchy(dim, k, L, inputs.sigma_of(k))
    B = inputs.uniform(15, prob.ndofs())
    close(host(prob.vcycle(cuda(B))), H.vcycle(B), rtol=1e-5, mtol=1e-4)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (2, 5, 3), (3, 3, 2), (3, 2, 3)])
def test_pcg_fp64(dim, k, L):
    note(f"pcg fp64 d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    B = oracle_load(dim, k, N)
    x, it, rel = prob.solve(cuda(B), rtol=1e-10)
    X = host(x)
    ap = KronApply(dim, k, N, sig)
    true_rel = np.linalg.norm(B - ap(X)) / np.linalg.norm(B)
    assert true_rel <= 2e-10, true_rel
    u = GlobalFD(dim, k, N, sig).solve(B)
    assert np.linalg.norm(X - u) <= 1e-8 * np.linalg.norm(u)
    # same iteration count as the oracle's PCG (+-1 for rounding)
    from oracle.multigrid import pcg
    H = Hierarchy(dim, k, L, sig)
    _, it_o, _, _ = pcg(H.apply[L], H.vcycle, B, rtol=1e-10)
    assert abs(int(it[0]) - it_o) <= 1, (it, it_o)


@pytest.mark.parametrize("dim,k,L", [(2, 3, 3), (3, 3, 2)])
def test_pcg_mixed_precision(dim, k, L):
    note(f"pcg mixed d={dim} k={k}")
    prob = problem(dim, k, L, precision=32)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    B = inputs.uniform(16, prob.ndofs())
    x, it, rel = prob.solve(cuda(B), rtol=1e-10)
    X = host(x)
    true_rel = np.linalg.norm(B - KronApply(dim, k, N, sig)(X)) / np.linalg.norm(B)
    assert true_rel <= 2e-10 and rel[0] <= 1e-10
    u = GlobalFD(dim, k, N, sig).solve(B)
    assert np.linalg.norm(X - u) <= 1e-8 * np.linalg.norm(u)


def test_pcg_batched_equals_single():
    note("pcg batched")
    dim, k, L = 3, 2, 2
    prob = problem(dim, k, L, nrhs_max=4)
    B = inputs.normal(17, (4, prob.ndofs()))
    B[2] *= 1e-3  # different scales converge at different iterations
    X, it, rel = prob.solve(cuda(B), rtol=1e-10)
    X = host(X)
    for j in range(4):
        xj, itj, _ = prob.solve(cuda(B[j]), rtol=1e-10)
        assert int(itj[0]) == int(it[j])
        close(X[j], host(xj), rtol=1e-13, mtol=1e-12)
        assert rel[j] <= 1e-10


@pytest.mark.parametrize("precision", [64, 32])
def test_pcg_batched_masks_match_single_solves(precision):
    """Right-hand sides that stop at different iterations in one batched
    solve (a zero one stops before the first, a smooth one early): the
    device-side convergence mask freezes each at its own iteration, with the
    single solve's iteration count, residual and solution."""
    note(f"pcg batched masks fp{precision}")
    dim, k, L = 3, 3, 2
    prob = problem(dim, k, L, precision=precision, nrhs_max=4)
    n = prob.ndofs()
    B = inputs.normal(23, (4, n))
    B[1] = 0.0
    B[3] = host(prob.mass(cuda(inputs.sine_load(prob.node_coords()))))
    X, it, rel = prob.solve(cuda(B), rtol=1e-10)
    X = host(X)
    assert int(it[1]) == 0 and np.all(X[1] == 0.0)
    assert len({int(v) for v in it}) > 1
    for j in (0, 2, 3):
        xj, itj, relj = prob.solve(cuda(B[j]), rtol=1e-10)
        assert int(itj[0]) == int(it[j])
        assert rel[j] <= 1e-10 and abs(float(relj[0]) - float(rel[j])) <= 1e-6 * float(rel[j])
        close(X[j], host(xj), rtol=1e-13, mtol=1e-12)


def test_repeatable_bitwise():
    note("determinism")
    prob = problem(3, 3, 2)
    B = cuda(inputs.uniform(18, prob.ndofs()))
    x1, _, _ = prob.solve(B, rtol=1e-10)
    x2, _, _ = prob.solve(B, rtol=1e-10)
    assert torch.equal(x1, x2)


def test_errors_are_reported():
    note("error paths")
    prob = problem(2, 2, 2)
    b = cuda(inputs.uniform(19, prob.ndofs()))
    b[3] = float("nan")
    with pytest.raises(dgmg.DGMGError) as e:
        prob.solve(b)
    assert e.value.status == -1
    b = cuda(inputs.uniform(19, prob.ndofs()))
    with pytest.raises(dgmg.DGMGError) as e:
        prob.solve(b, rtol=1e-14, maxit=2)
    assert e.value.status == -4
    x, it, rel = prob.solve(b, rtol=1e-14, maxit=2, raise_on_nonconvergence=False)
    assert int(it[0]) == 2 and rel[0] > 1e-14
    with pytest.raises(dgmg.DGMGError):
        prob.apply(b, level=5)
    with pytest.raises(ValueError):
        prob.apply(cuda(np.zeros(7)))
    z, it, rel = prob.solve(torch.zeros_like(b))
    assert int(it[0]) == 0 and float(torch.abs(z).max()) == 0.0


def test_full_size_poisson3d_q3_32c():
    """Workload of the benchmark (3-D Q3, 32^3 cells, 2.1M DoFs, FP64):
    full-vector parity of apply and one smoothing step; PCG to 1e-10 checked
    against the exact discrete solution by global fast diagonalisation."""
    note("full size 3-D Q3 32^3")
    w = inputs.WORKLOADS["poisson3d_q3_32c"]
    dim, k, L = w["dim"], w["k"], w["L"]
    prob = problem(dim, k, L, nrhs_max=1)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    X = inputs.uniform(w["seed"], prob.ndofs())
    close(host(prob.apply(cuda(X))), KronApply(dim, k, N, sig)(X))
    B = inputs.uniform(w["seed"] + 1, prob.ndofs())
    Xg = cuda(X)
    prob.smooth(Xg, cuda(B))
    close(host(Xg), FDSmoother(dim, k, N, sig).step(X, B, list(range(8))))
    Bh = oracle_load(dim, k, N)
    x, it, rel = prob.solve(cuda(Bh), rtol=1e-10)
    u = GlobalFD(dim, k, N, sig).solve(Bh)
    assert np.linalg.norm(host(x) - u) <= 1e-8 * np.linalg.norm(u)
    assert it[0] <= 12


@pytest.mark.parametrize("precision", [64, 32])
def test_graph_replays_equal_eager(precision):
    note(f"graph replay precision={precision}")
    prob = dgmg.Problem(3, 2, 2, precision=precision, nrhs_max=3)
    B = cuda(inputs.uniform(31, (3, prob.ndofs())))
    y = torch.empty_like(B[0])
    for kappa in (1.0, 2.5):
        prob.set_kappa(kappa)
        prob.use_graphs(False)
        x_e, it_e, _ = prob.solve(B, rtol=1e-10)
        x_e = x_e.clone()
        x1, it1, _ = prob.solve(B[1].contiguous(), rtol=1e-10)
        x1 = x1.clone()
        prob.use_graphs(True)
        for rep in range(3):
            x_g, it_g, _ = prob.solve(B, rtol=1e-10)
            assert torch.equal(x_g, x_e), (kappa, rep)
            assert list(it_g) == list(it_e)
            xs, _, _ = prob.solve(B[1].contiguous(), rtol=1e-10)  # second graph (nrhs = 1)
            assert torch.equal(xs, x1)
            prob.apply(B[rep].contiguous(), out=y)  # eager work between replays
            torch.cuda.synchronize()
    prob.close()


@pytest.mark.parametrize("dim,k,L,precision,variant", [
    (2, 2, 1, 64, 0), (2, 5, 3, 64, 0), (2, 3, 2, 64, 0), (2, 7, 3, 32, 1), (2, 4, 3, 64, 3),
    (3, 1, 2, 64, 0), (3, 2, 1, 64, 0), (3, 3, 3, 64, 0),
    (3, 3, 2, 32, 0), (3, 4, 2, 32, 0), (3, 3, 2, 64, 1), (3, 3, 2, 64, 3), (3, 4, 1, 64, 0)])
def test_fused_vcycle_bottom_equals_separate_kernels(monkeypatch, dim, k, L, precision, variant):
    """Levels 1 and 0 in one launch, with one or two waves per patch, give
    bitwise the V-cycle of the separate kernels (where the kernels allow the
    fusion; elsewhere the paths fall back to the separate kernels)."""
    note(f"fused bottom d={dim} k={k} L={L} fp{precision} variant={variant}")
    outs = {}
    for fuse in ("2", "1", "0"):
        monkeypatch.setenv("DGMG_FUSE_BOTTOM", fuse)
        prob = dgmg.Problem(dim, k, L, precision=precision, variant=variant, nrhs_max=2)
        prob.use_dense_bottom(False)
        B = inputs.uniform(33, (2, prob.ndofs()))
        dt = torch.float64 if precision == 64 else torch.float32
        res = [prob.vcycle(cuda(B, dt)).clone()]
        if variant != 1:  # the paper's residual makes the V-cycle unsymmetric (no CG)
            res.append(prob.solve(cuda(B), rtol=1e-10, maxit=200)[0].clone())
        outs[fuse] = res
        prob.close()
    torch.cuda.synchronize()
    for a, b, c in zip(outs["2"], outs["1"], outs["0"]):
        assert torch.equal(a, c) and torch.equal(b, c)


MODES = {0: "exact", 1: "local", 2: "full", 3: "clamped"}


@pytest.mark.parametrize("dim,k,L,precision,variant,level", [
    (3, 3, 2, 64, 0, 1), (3, 3, 2, 32, 1, 1), (3, 3, 2, 64, 3, 1), (3, 2, 3, 64, 0, 1),
    (3, 1, 3, 32, 0, 2), (2, 5, 3, 64, 0, 2), (2, 7, 3, 32, 3, 2), (2, 3, 4, 64, 1, 3),
    (3, 4, 2, 32, 0, 1), (3, 4, 2, 64, 0, 1), (2, 3, 2, 64, 0, 1), (2, 2, 1, 64, 0, -1),
    (3, 3, 2, 64, 2, 1), (2, 4, 3, 32, 2, 2)])
def test_dense_bottom_equals_bottom_launch(dim, k, L, precision, variant, level):
    """The V-cycle with its bottom levels (0..level: the finest level below
    L with at most 8192 DoFs) as the dense operator built at set-up equals
    the V-cycle with its kernels (fused bottom launches or separate ones, as
    for FP64 Q4) up to rounding order, and the oracle's V-cycle; also after
    a change of kappa (the operator is scaled, not rebuilt); for every
    smoother variant, the Full one included.  Where no operator is built
    (no level between 0 and L) both switches give the kernels bitwise."""
    note(f"dense bottom d={dim} k={k} L={L} fp{precision} variant={variant}")
    prob = dgmg.Problem(dim, k, L, precision=precision, variant=variant, nrhs_max=3)
    assert prob.dense_bottom_level() == level
    dt = torch.float64 if precision == 64 else torch.float32
    B = inputs.uniform(34, (3, prob.ndofs()))
    tol = 1e-13 if precision == 64 else 1e-5
    for kappa in (1.0, 0.37):
        prob.set_kappa(kappa)
        got = {}
        for dense in (True, False):
            prob.use_dense_bottom(dense)
            got[dense] = host(prob.vcycle(cuda(B, dt)))
        if level < 0:
            assert np.array_equal(got[True], got[False])
        else:
            close(got[True], got[False], rtol=tol, mtol=10 * tol)
        H = Hierarchy(dim, k, L, inputs.sigma_of(k), kappa=kappa, mode=MODES[variant])
        ref = H.vcycle(B[1])
        close(got[True][1], ref, rtol=1e-11 if precision == 64 else 1e-5,
              mtol=1e-10 if precision == 64 else 1e-4)
    prob.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_dense_bottom_many_rhs(precision):
    """Up to 16 right-hand sides take the dense bottom (11: two groups of 8,
    the second ragged), each equal to its single-RHS V-cycle up to rounding
    order; 17 take the bottom launch, bitwise as with the matrix switched
    off."""
    note(f"dense bottom many rhs fp{precision}")
    prob = dgmg.Problem(3, 3, 2, precision=precision, nrhs_max=17)
    assert prob.dense_bottom_level() == 1
    dt = torch.float64 if precision == 64 else torch.float32
    tol = 1e-13 if precision == 64 else 1e-5
    B = inputs.uniform(36, (17, prob.ndofs()))
    X11 = host(prob.vcycle(cuda(B[:11], dt)))
    for j in (0, 7, 8, 10):
        close(X11[j], host(prob.vcycle(cuda(B[j], dt))), rtol=tol, mtol=10 * tol)
    prob.use_dense_bottom(False)
    L11 = host(prob.vcycle(cuda(B[:11], dt)))
    close(X11, L11, rtol=tol, mtol=10 * tol)
    L17 = host(prob.vcycle(cuda(B, dt)))
    prob.use_dense_bottom(True)
    assert np.array_equal(host(prob.vcycle(cuda(B, dt))), L17)
    prob.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_dense_bottom_in_graph_and_noalloc(precision):
    """CG with the dense bottom in the captured V-cycle equals CG with eager
    launches bitwise, and the allocation-free V-cycle uses the same bottom."""
    note(f"dense bottom graph fp{precision}")
    prob = dgmg.Problem(3, 3, 2, precision=precision, nrhs_max=2)
    assert prob.dense_bottom_level() == 1
    B = inputs.uniform(35, (2, prob.ndofs()))
    res = {}
    for graphs in (True, False):
        prob.use_graphs(graphs)
        x, it, _ = prob.solve(cuda(B), rtol=1e-10, maxit=100)
        res[graphs] = (host(x), list(it))
    assert res[True][1] == res[False][1]
    assert np.array_equal(res[True][0], res[False][0])
    a = host(prob.vcycle(cuda(B)))
    out = torch.empty((2, prob.ndofs()), dtype=torch.float64, device="cuda")
    prob.vcycle_noalloc(cuda(B), out)
    assert np.array_equal(a, host(out))
    prob.close()
