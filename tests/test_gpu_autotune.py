"""The autotuner's choices are all correct: every workgroup shape (patches
per workgroup, b prefetch, one or two waves per patch) and patch
numbering it can pick is forced through its JSON cache and checked against
the oracle; tuning writes the cache and a second call reads it back."""
import itertools
import sys

import numpy as np
import pytest

from oracle.sipg import kron_operator
from oracle.smoother import FDSmoother
from paper_2405_18982_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_18982_amd import dgmg  # noqa: E402


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def force_cache(path, dim, k, L, nrhs, shape, remap):
    """Cache entries forcing the FP64 apply (shape mod 4) and the FP64
    smoother on every level (shape 0..11) to one choice."""
    lines = []
    keys = [("apply", shape % 4)] + [(f"smooth/l{l}", shape) for l in range(1, L + 1)]
    for kern, sh in keys:
        key = f"gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/{kern}"
        lines.append(f'  "{key}": {{"shape": {sh}, "remap": {remap}, "us": 1.000}}')
    path.write_text("{\n" + ",\n".join(lines) + "\n}\n")


@pytest.mark.parametrize("dim,k,L", [(2, 2, 3), (2, 5, 2), (3, 1, 2), (3, 2, 2), (3, 3, 2), (3, 4, 1)])
@pytest.mark.parametrize("shape,remap", list(itertools.product(range(12), [0, 1])))
def test_every_tunable_shape_matches_oracle(tmp_path, dim, k, L, shape, remap):
    note(f"tuned shape={shape} remap={remap} d={dim} k={k} L={L}")
    nrhs = 2
    prob = dgmg.Problem(dim, k, L, nrhs_max=nrhs)
    cache = tmp_path / "tune.json"
    force_cache(cache, dim, k, L, nrhs, shape, remap)
    rep = prob.autotune(nrhs=nrhs, cache=str(cache))
    assert rep.count("(cached)") == 1 + L and f"shape={shape} remap={remap}" in rep
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    X = inputs.uniform(41, (nrhs, prob.ndofs()))
    B = inputs.uniform(42, (nrhs, prob.ndofs()))
    Y = prob.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    A = kron_operator(dim, k, N, sig)
    Xg = torch.from_numpy(X).cuda()
    prob.smooth(Xg, torch.from_numpy(B).cuda())
    S = Xg.cpu().numpy()
    fs = FDSmoother(dim, k, N, sig)
    for j in range(nrhs):
        assert rel(Y[j], A @ X[j]) <= 1e-12
        assert rel(S[j], fs.step(X[j], B[j], list(range(2 ** dim)))) <= 1e-12
    prob.close()


def test_tuning_writes_and_reads_cache(tmp_path):
    note("autotune run + cache")
    prob = dgmg.Problem(3, 3, 3, precision=32, nrhs_max=4)
    cache = tmp_path / "tune.json"
    rep1 = prob.autotune(nrhs=4, cache=str(cache))
    # FP64 apply on the finest level + FP32 smoother on levels 1..3
    assert len(rep1.strip().splitlines()) == 4 and "(cached)" not in rep1
    txt = cache.read_text()
    assert txt.startswith("{") and txt.count('"shape"') == 4
    rep2 = prob.autotune(nrhs=4, cache=str(cache))
    assert rep2.count("(cached)") == 4
    strip = [ln.replace(" (cached)", "") for ln in rep2.strip().splitlines()]
    assert strip == rep1.strip().splitlines()
    # the tuned context still solves to tolerance
    B = torch.from_numpy(inputs.normal(43, (4, prob.ndofs()))).cuda()
    x, it, relres = prob.solve(B, rtol=1e-10)
    assert np.all(relres <= 1e-10) and np.all(it <= 15)
    prob.close()


@pytest.mark.parametrize("dim,k,L", [(3, 3, 2), (3, 7, 1)])
@pytest.mark.parametrize("variant", [0, 1, 3])
@pytest.mark.parametrize("precision", [64, 32])
def test_two_wave_shapes_are_bitwise_one_wave(tmp_path, dim, k, L, variant, precision):
    """The two-waves-per-patch smoother computes every output with the
    operations of the one-wave kernel: shapes 4..7 equal shapes 0..3 bit for
    bit, for a smoothing step and for a V-cycle (colour 0 from zero)."""
    note(f"two-wave bitwise d={dim} k={k} variant={variant} fp{precision}")
    nrhs = 2
    dt = torch.float64 if precision == 64 else torch.float32
    X = inputs.uniform(61, (nrhs, 2 ** ((L + 1) * dim) * (k + 1) ** dim))
    B = inputs.uniform(62, X.shape)
    outs = {}
    for shape in (0, 2, 4, 6):
        prob = dgmg.Problem(dim, k, L, precision=precision, variant=variant, nrhs_max=nrhs)
        cache = tmp_path / f"tune{shape}.json"
        lines = []
        for l in range(1, L + 1):
            key = f"gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp{precision}/smooth/l{l}"
            lines.append(f'  "{key}": {{"shape": {shape}, "remap": 1, "us": 1.000}}')
        cache.write_text("{\n" + ",\n".join(lines) + "\n}\n")
        prob.autotune(nrhs=nrhs, cache=str(cache))
        Xg = torch.from_numpy(X).to("cuda", dt)
        prob.smooth(Xg, torch.from_numpy(B).to("cuda", dt))
        V = prob.vcycle(torch.from_numpy(B).to("cuda", dt))
        torch.cuda.synchronize()
        outs[shape] = (Xg.cpu(), V.cpu())
        prob.close()
    for one, two in ((0, 4), (2, 6)):
        assert torch.equal(outs[one][0], outs[two][0])
        assert torch.equal(outs[one][1], outs[two][1])


@pytest.mark.parametrize("dim,k,L", [(3, 1, 3), (3, 3, 2), (3, 3, 1), (3, 2, 2), (3, 4, 1), (3, 5, 1),
                                     (3, 6, 1), (3, 7, 1), (2, 3, 3)])
def test_register_face_apply_is_bitwise_lds_apply(tmp_path, dim, k, L):
    """Apply shape 2 (neighbour face data contracted in registers, then across
    lanes (3-D Q1, Q3) or through a small LDS array (other degrees); in 2-D
    the same as shape 0) evaluates every output with the operations of shape
    0: equal bit for bit, on every right-hand side."""
    note(f"register-face apply bitwise d={dim} k={k} L={L}")
    nrhs = 3
    X = inputs.uniform(71, (nrhs, 2 ** ((L + 1) * dim) * (k + 1) ** dim))
    outs = {}
    for shape in (0, 2):
        prob = dgmg.Problem(dim, k, L, nrhs_max=nrhs)
        cache = tmp_path / f"tune{shape}.json"
        key = f"gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/apply"
        cache.write_text("{\n" + f'  "{key}": {{"shape": {shape}, "remap": 1, "us": 1.000}}' + "\n}\n")
        prob.autotune(nrhs=nrhs, cache=str(cache))
        outs[shape] = prob.apply(torch.from_numpy(X).to("cuda", torch.float64)).cpu()
        prob.close()
    assert torch.equal(outs[0], outs[2])
    A = kron_operator(dim, k, 2 ** (L + 1), inputs.sigma_of(k))
    for j in range(nrhs):
        assert rel(outs[2][j].numpy(), A @ X[j]) <= 1e-12


@pytest.mark.parametrize("dim,k,L", [(2, 2, 3), (2, 5, 2), (3, 1, 2), (3, 3, 2), (3, 4, 1), (3, 7, 1)])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", [64, 32])
def test_rhs_packed_shapes_are_bitwise_patch_packed(tmp_path, dim, k, L, variant, precision):
    """Shapes that hold one patch for several right-hand sides per workgroup
    (apply 3, smoother 8..11) compute every output with the operations of
    the patch-packed shapes (apply 0, smoother 0..3): equal bit for bit for a
    smoothing step, a V-cycle and the apply, with a right-hand-side count (5)
    that leaves the last workgroup partly empty."""
    if variant == 3 and k < 3:
        pytest.skip("the clamped kernel needs k >= 3")
    note(f"rhs-packed bitwise d={dim} k={k} L={L} variant={variant} fp{precision}")
    nrhs = 5
    dt = torch.float64 if precision == 64 else torch.float32
    X = inputs.uniform(81, (nrhs, 2 ** ((L + 1) * dim) * (k + 1) ** dim))
    B = inputs.uniform(82, X.shape)
    outs = {}
    for sm, ap in ((0, 0), (8, 3), (2, 0), (11, 3)):
        prob = dgmg.Problem(dim, k, L, precision=precision, variant=variant, nrhs_max=nrhs)
        cache = tmp_path / f"tune{sm}.json"
        lines = [f'  "gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp64/apply": {{"shape": {ap}, "remap": 1, "us": 1.000}}']
        for l in range(1, L + 1):
            key = f"gfx950/d{dim}/k{k}/L{L}/nrhs{nrhs}/fp{precision}/smooth/l{l}"
            lines.append(f'  "{key}": {{"shape": {sm}, "remap": 1, "us": 1.000}}')
        cache.write_text("{\n" + ",\n".join(lines) + "\n}\n")
        prob.autotune(nrhs=nrhs, cache=str(cache))
        Xg = torch.from_numpy(X).to("cuda", dt)
        prob.smooth(Xg, torch.from_numpy(B).to("cuda", dt))
        V = prob.vcycle(torch.from_numpy(B).to("cuda", dt))
        Y = prob.apply(torch.from_numpy(X).to("cuda", torch.float64))
        torch.cuda.synchronize()
        outs[sm] = (Xg.cpu(), V.cpu(), Y.cpu())
        prob.close()
    for a, b in ((0, 8), (2, 11)):
        for i in range(3):
            assert torch.equal(outs[a][i], outs[b][i]), f"shapes {a}/{b} output {i}"
    if precision == 64 and variant == 0:
        A = kron_operator(dim, k, 2 ** (L + 1), inputs.sigma_of(k))
        fs = FDSmoother(dim, k, 2 ** (L + 1), inputs.sigma_of(k))
        for j in range(nrhs):
            assert rel(outs[8][2][j].numpy(), A @ X[j]) <= 1e-12
            assert rel(outs[8][0][j].numpy(), fs.step(X[j], B[j], list(range(2 ** dim)))) <= 1e-12
