"""GPU parity of the clamped vertex-patch kernel (Sec. 3.1: zero value and
normal derivative on the patch faces inside the domain) against the FP64
oracle through the C ABI: smoothing steps on every level and patch type in
both colour orders, FP32, V-cycle, PCG against the exact discrete solution,
every tunable shape, and the rejection of degrees below 3.  Tolerances as in
the other parity tests."""
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

CLAMPED = dgmg.SMOOTH_CLAMPED
SMALL = [(2, 3, 2), (2, 5, 2), (2, 7, 1), (3, 3, 2), (3, 4, 1), (3, 7, 1)]

_probs = {}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problem(dim, k, L, precision=64, nrhs_max=2):
    key = (dim, k, L, precision, nrhs_max)
    if key not in _probs:
        _probs[key] = dgmg.Problem(dim, k, L, precision=precision, variant=CLAMPED,
                                   nrhs_max=nrhs_max)
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


@pytest.mark.parametrize("dim,k,L", SMALL)
def test_clamped_smooth_fp64(dim, k, L):
    note(f"clamped smooth fp64 d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    sig = inputs.sigma_of(k)
    for l in range(1, L + 1):
        N = 2 ** (l + 1)
        fs = FDSmoother(dim, k, N, sig, mode="clamped")
        X = inputs.uniform(900 + l, (2, prob.ndofs(l)))
        B = inputs.uniform(950 + l, (2, prob.ndofs(l)))
        for reverse in (False, True):
            order = list(range(2 ** dim))[::-1] if reverse else list(range(2 ** dim))
            Xg = cuda(X)
            prob.smooth(Xg, cuda(B), level=l, reverse=reverse)
            G = host(Xg)
            for j in range(2):
                close(G[j], fs.step(X[j], B[j], order))


@pytest.mark.parametrize("dim,k,L", [(2, 3, 2), (3, 3, 2)])
def test_clamped_smooth_fp32(dim, k, L):
    note(f"clamped smooth fp32 d={dim} k={k}")
    prob = problem(dim, k, L)
    fs = FDSmoother(dim, k, 2 ** (L + 1), inputs.sigma_of(k), mode="clamped")
    X = inputs.uniform(25, prob.ndofs()).astype(np.float32).astype(np.float64)
    B = inputs.uniform(26, prob.ndofs()).astype(np.float32).astype(np.float64)
    Xg = cuda(X, torch.float32)
    prob.smooth(Xg, cuda(B, torch.float32))
    close(host(Xg), fs.step(X, B, list(range(2 ** dim))), rtol=5e-5, mtol=5e-4)


@pytest.mark.parametrize("dim,k,L", [(2, 3, 3), (3, 3, 2), (3, 5, 1)])
def test_clamped_vcycle_fp64(dim, k, L):
    note(f"clamped vcycle d={dim} k={k} L={L}")
    prob = problem(dim, k, L)
    H = Hierarchy(dim, k, L, inputs.sigma_of(k), mode="clamped")
    B = inputs.uniform(27, (2, prob.ndofs()))
    X = host(prob.vcycle(cuda(B)))
    for j in range(2):
        close(X[j], H.vcycle(B[j]), rtol=1e-11, mtol=1e-10)


@pytest.mark.parametrize("dim,k,L,precision", [(2, 4, 3, 64), (3, 3, 2, 64), (3, 4, 2, 32)])
def test_clamped_pcg_against_exact_solution(dim, k, L, precision):
    note(f"clamped pcg d={dim} k={k} L={L} fp{precision}")
    prob = problem(dim, k, L, precision=precision, nrhs_max=1)
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    B = mass_operator(dim, k, N) @ interpolate(dim, k, N, inputs.sine_load)
    x, it, rel = prob.solve(cuda(B), rtol=1e-10, maxit=200)
    X = host(x)
    true_rel = np.linalg.norm(B - KronApply(dim, k, N, sig)(X)) / np.linalg.norm(B)
    assert rel[0] <= 1e-10 and true_rel <= 2e-10, (rel, true_rel)
    u = GlobalFD(dim, k, N, sig).solve(B)
    assert np.linalg.norm(X - u) <= 1e-8 * np.linalg.norm(u)
    H = Hierarchy(dim, k, L, sig, mode="clamped")
    _, it_o, _, _ = pcg(H.apply[L], H.vcycle, B, rtol=1e-10, maxit=200, flexible=precision == 32)
    assert abs(int(it[0]) - it_o) <= 1, (it, it_o)


@pytest.mark.parametrize("shape,remap", list(itertools.product(range(8), [0, 1])))
def test_clamped_every_tunable_shape(tmp_path, shape, remap):
    dim, k, L, nrhs = 3, 3, 2, 2
    note(f"clamped tuned shape={shape} remap={remap}")
    prob = dgmg.Problem(dim, k, L, variant=CLAMPED, nrhs_max=nrhs)
    lines = [f'  "gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/apply": {{"shape": {shape % 2}, '
             f'"remap": {remap}, "us": 1.000}}']
    for l in range(1, L + 1):
        lines.append(f'  "gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/smooth/l{l}": '
                     f'{{"shape": {shape}, "remap": {remap}, "us": 1.000}}')
    cache = tmp_path / "tune.json"
    cache.write_text("{\n" + ",\n".join(lines) + "\n}\n")
    assert prob.autotune(nrhs=nrhs, cache=str(cache)).count("(cached)") == 1 + L
    X = inputs.uniform(53, (nrhs, prob.ndofs()))
    B = inputs.uniform(54, (nrhs, prob.ndofs()))
    Xg = cuda(X)
    prob.smooth(Xg, cuda(B))
    S = host(Xg)
    fs = FDSmoother(dim, k, 2 ** (L + 1), inputs.sigma_of(k), mode="clamped")
    for j in range(nrhs):
        close(S[j], fs.step(X[j], B[j], list(range(2 ** dim))))
    prob.close()


def test_clamped_needs_degree_3():
    with pytest.raises(dgmg.DGMGError) as e:
        dgmg.Problem(3, 2, 1, variant=CLAMPED)
    assert e.value.status == -1
