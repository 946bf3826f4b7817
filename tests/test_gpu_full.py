"""GPU parity of the Full vertex-patch kernel (Sec. 3.1: V_j = the whole
patch, residual taken once per colour) against the FP64 oracle, through the
C ABI: one smoothing step on every level and patch type in both colour
orders, FP32, the V-cycle, PCG (FP64 and mixed) against the exact discrete
solution, graph replays, every tunable shape, and the benchmark workload at
full size.  Tolerances as in the other parity tests: FP64 1e-12 relative
(l2) / 1e-11 (max), FP32 5e-5 / 5e-4."""
import itertools
import sys

import numpy as np
import pytest

from oracle.fdsolve import GlobalFD
from oracle.multigrid import Hierarchy, pcg
from oracle.rhs import interpolate
from oracle.sipg import KronApply, mass_operator
from oracle.smoother import FDSmoother
from paper_2405_18982_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_18982_amd import dgmg  # noqa: E402

FULL = dgmg.SMOOTH_FULL
SMALL = [(2, 1, 3), (2, 2, 2), (2, 5, 2), (2, 7, 1), (3, 1, 2), (3, 2, 2), (3, 3, 2), (3, 4, 1),
         (3, 7, 1)]

_probs = {}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problem(dim, k, L, precision=64, nrhs_max=2):
    key = (dim, k, L, precision, nrhs_max)
    if key not in _probs:
        _probs[key] = dgmg.Problem(dim, k, L, precision=precision, variant=FULL, nrhs_max=nrhs_max)
    return _probs[key]


def cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def close(got, ref, rtol=1e-12, mtol=1e-11):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    nr = np.linalg.norm(ref)
    err = np.linalg.norm(got - ref)
    assert err <= rtol * max(nr, 1e-300), f"rel l2 err {err / nr:.3e}"
    assert np.abs(got - ref).max() <= mtol * max(np.abs(ref).max(), 1e-300)


def oracle_load(dim, k, N):
    return mass_operator(dim, k, N) @ interpolate(dim, k, N, inputs.sine_load)


@pytest.mark.parametrize("dim,k,L", SMALL)
def test_full_smooth_fp64(dim, k, L):
    note(f"full smooth fp64 d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    sig = inputs.sigma_of(k)
    for l in range(1, L + 1):
        N = 2 ** (l + 1)
        fs = FDSmoother(dim, k, N, sig, mode="full")
        X = inputs.uniform(700 + l, (2, prob.ndofs(l)))
        B = inputs.uniform(800 + l, (2, prob.ndofs(l)))
        for reverse in (False, True):
            order = list(range(2 ** dim))[::-1] if reverse else list(range(2 ** dim))
            Xg = cuda(X)
            Bg = cuda(B)
            prob.smooth(Xg, Bg, level=l, reverse=reverse)
            G = host(Xg)
            assert np.array_equal(host(Bg), B)  # b is read only
            for j in range(2):
                close(G[j], fs.step(X[j], B[j], order))


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2), (3, 7, 1)])
def test_full_smooth_fp32(dim, k, L):
    note(f"full smooth fp32 d={dim} k={k}")
    prob = problem(dim, k, L)
    fs = FDSmoother(dim, k, 2 ** (L + 1), inputs.sigma_of(k), mode="full")
    X = inputs.uniform(21, prob.ndofs()).astype(np.float32).astype(np.float64)
    B = inputs.uniform(22, prob.ndofs()).astype(np.float32).astype(np.float64)
    Xg = cuda(X, torch.float32)
    prob.smooth(Xg, cuda(B, torch.float32))
    close(host(Xg), fs.step(X, B, list(range(2 ** dim))), rtol=5e-5, mtol=5e-4)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (2, 5, 3), (3, 2, 2), (3, 3, 2), (3, 7, 1)])
def test_full_vcycle_fp64(dim, k, L):
    note(f"full vcycle fp64 d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    H = Hierarchy(dim, k, L, inputs.sigma_of(k), mode="full")
    B = inputs.uniform(23, (2, prob.ndofs()))
    X = host(prob.vcycle(cuda(B)))
    for j in range(2):
        close(X[j], H.vcycle(B[j]), rtol=1e-11, mtol=1e-10)


@pytest.mark.parametrize("dim,k,L", [(2, 2, 2), (3, 3, 2)])
def test_full_vcycle_fp32(dim, k, L):
    note(f"full vcycle fp32 d={dim} k={k}")
    prob = problem(dim, k, L, precision=32)
    H = Hierarchy(dim, k, L, inputs.sigma_of(k), mode="full")
    B = inputs.uniform(24, prob.ndofs())
    close(host(prob.vcycle(cuda(B))), H.vcycle(B), rtol=1e-5, mtol=1e-4)


@pytest.mark.parametrize("dim,k,L,precision", [(2, 3, 3, 64), (3, 2, 3, 64), (3, 3, 2, 64),
                                               (3, 3, 2, 32), (3, 5, 1, 64)])
def test_full_pcg_against_exact_solution(dim, k, L, precision):
    note(f"full pcg d={dim} k={k} L={L} fp{precision}")
    prob = problem(dim, k, L, precision=precision, nrhs_max=1)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    B = oracle_load(dim, k, N)
    x, it, rel = prob.solve(cuda(B), rtol=1e-10)
    X = host(x)
    true_rel = np.linalg.norm(B - KronApply(dim, k, N, sig)(X)) / np.linalg.norm(B)
    assert rel[0] <= 1e-10 and true_rel <= 2e-10, (rel, true_rel)
    u = GlobalFD(dim, k, N, sig).solve(B)
    assert np.linalg.norm(X - u) <= 1e-8 * np.linalg.norm(u)
    H = Hierarchy(dim, k, L, sig, mode="full")
    _, it_o, _, _ = pcg(H.apply[L], H.vcycle, B, rtol=1e-10, flexible=precision == 32)
    assert abs(int(it[0]) - it_o) <= 1, (it, it_o)


def test_full_graph_replays_equal_eager():
    note("full graph replay")
    prob = dgmg.Problem(3, 2, 2, variant=FULL, nrhs_max=2)
    B = cuda(inputs.uniform(32, (2, prob.ndofs())))
    prob.use_graphs(False)
    x_e, it_e, _ = prob.solve(B, rtol=1e-10)
    x_e = x_e.clone()
    prob.use_graphs(True)
    for rep in range(3):
        x_g, it_g, _ = prob.solve(B, rtol=1e-10)
        assert torch.equal(x_g, x_e), rep
        assert list(it_g) == list(it_e)
        prob.apply(B[rep % 2].contiguous())  # eager work between replays
        torch.cuda.synchronize()
    prob.close()


def _force_cache(path, dim, k, L, nrhs, shape, remap):
    lines = []
    keys = [("apply", shape % 2)] + [(f"smooth/l{l}", shape) for l in range(1, L + 1)]
    for kern, sh in keys:
        key = f"gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/{kern}"
        lines.append(f'  "{key}": {{"shape": {sh}, "remap": {remap}, "us": 1.000}}')
    path.write_text("{\n" + ",\n".join(lines) + "\n}\n")


@pytest.mark.parametrize("dim,k,L", [(2, 3, 2), (3, 1, 2), (3, 3, 2), (3, 4, 1)])
@pytest.mark.parametrize("shape,remap", list(itertools.product([0, 1, 2, 3], [0, 1])))
def test_full_every_tunable_shape(tmp_path, dim, k, L, shape, remap):
    note(f"full tuned shape={shape} remap={remap} d={dim} k={k} L={L}")
    nrhs = 2
    prob = dgmg.Problem(dim, k, L, variant=FULL, nrhs_max=nrhs)
    cache = tmp_path / "tune.json"
    _force_cache(cache, dim, k, L, nrhs, shape, remap)
    rep = prob.autotune(nrhs=nrhs, cache=str(cache))
    assert rep.count("(cached)") == 1 + L
    N = 2 ** (L + 1)
    X = inputs.uniform(51, (nrhs, prob.ndofs()))
    B = inputs.uniform(52, (nrhs, prob.ndofs()))
    Xg = cuda(X)
    prob.smooth(Xg, cuda(B))
    S = host(Xg)
    fs = FDSmoother(dim, k, N, inputs.sigma_of(k), mode="full")
    for j in range(nrhs):
        close(S[j], fs.step(X[j], B[j], list(range(2 ** dim))))
    prob.close()


def test_full_size_poisson3d_q3_32c():
    """The benchmark workload (3-D Q3, 32^3 cells, 2.1M DoFs) with the Full
    kernel: one smoothing step element by element, and PCG to 1e-10 against
    the exact discrete solution."""
    note("full kernel, full size 3-D Q3 32^3")
    w = inputs.WORKLOADS["poisson3d_q3_32c"]
    dim, k, L = w["dim"], w["k"], w["L"]
    prob = problem(dim, k, L, nrhs_max=1)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    X = inputs.uniform(w["seed"], prob.ndofs())
    B = inputs.uniform(w["seed"] + 1, prob.ndofs())
    Xg = cuda(X)
    prob.smooth(Xg, cuda(B))
    close(host(Xg), FDSmoother(dim, k, N, sig, mode="full").step(X, B, list(range(8))))
    Bh = oracle_load(dim, k, N)
    x, it, rel = prob.solve(cuda(Bh), rtol=1e-10)
    u = GlobalFD(dim, k, N, sig).solve(Bh)
    assert np.linalg.norm(host(x) - u) <= 1e-8 * np.linalg.norm(u)
    assert it[0] <= 10
