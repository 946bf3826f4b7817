"""The allocation-free V-cycle (dgmg_vcycle_noalloc) against the V-cycle with
the context's own level vectors (dgmg_vcycle), through the C ABI: the same
kernels on the same inputs, so the results must agree bit for bit.  Each case
makes two calls in a row on one GPU, the second with a smaller input, so the
second call runs on whatever the first left in the shared scratch array; one
small case is also checked against the oracle's V-cycle (FP64 bar 1e-12)."""
import sys

import numpy as np
import pytest

from oracle.multigrid import Hierarchy
from paper_2405_18982_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_18982_amd import dgmg  # noqa: E402


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(prob, b):
    """(dgmg_vcycle(b), dgmg_vcycle_noalloc(b)) with caller-allocated outputs."""
    ref = torch.empty_like(b)
    out = torch.full_like(b, float("nan"))
    prob.vcycle(b, out=ref)
    prob.vcycle_noalloc(b, out)
    torch.cuda.synchronize()
    return ref, out


def rhs(prob, nrhs, seed):
    return torch.from_numpy(inputs.uniform(seed, nrhs * prob.ndofs())).cuda().view(nrhs, -1)


# (dim, k, L, precision, variant, nrhs of the first call, nrhs of the second)
CASES = [
    (3, 3, 3, 64, dgmg.SMOOTH_EXACT, 3, 1),
    (2, 5, 4, 64, dgmg.SMOOTH_EXACT, 2, 1),
    (3, 4, 2, 32, dgmg.SMOOTH_EXACT, 2, 1),
    (3, 3, 2, 64, dgmg.SMOOTH_FULL, 2, 1),
    (3, 3, 2, 64, dgmg.SMOOTH_CLAMPED, 2, 1),
    (2, 2, 3, 64, dgmg.SMOOTH_LOCAL, 2, 1),
]


@pytest.mark.parametrize("dim,k,L,prec,variant,n1,n2", CASES)
def test_noalloc_vcycle_equals_vcycle_two_calls(dim, k, L, prec, variant, n1, n2):
    note(f"noalloc vcycle d={dim} k={k} L={L} prec={prec} variant={variant} nrhs {n1} then {n2}")
    prob = dgmg.Problem(dim, k, L, precision=prec, variant=variant, nrhs_max=max(n1, n2))
    for call, (nr, seed) in enumerate([(n1, 11), (n2, 12)]):
        b = rhs(prob, nr, seed)
        ref, out = both(prob, b)
        assert torch.isfinite(ref).all()
        assert torch.equal(ref, out), f"call {call}: max diff {float((ref - out).abs().max()):.3e}"
    prob.close()


def test_noalloc_smaller_context_after_larger():
    """A second context with a smaller mesh reuses the scratch array the
    first (larger) one filled; both agree with dgmg_vcycle, and the small one
    with the oracle's V-cycle."""
    big = dgmg.Problem(3, 3, 3, nrhs_max=2)
    b = rhs(big, 2, 21)
    ref, out = both(big, b)
    assert torch.equal(ref, out)
    big.close()
    dim, k, L = 2, 2, 2
    small = dgmg.Problem(dim, k, L)
    b = rhs(small, 1, 22)
    ref, out = both(small, b)
    assert torch.equal(ref, out)
    v = Hierarchy(dim, k, L, small.sigma).vcycle(b.cpu().numpy().ravel())
    got = out.cpu().numpy().ravel()
    assert np.linalg.norm(got - v) <= 1e-12 * np.linalg.norm(v)
    small.close()


def test_noalloc_rejects_inputs_beyond_the_scratch_size():
    """3-D Q3 32^3 in FP64: the coarse levels take 4,792,320 bytes per
    right-hand side (b and x), so 14 fit in 64 MiB and 15 do not."""
    prob = dgmg.Problem(3, 3, 4, nrhs_max=15)
    b = rhs(prob, 15, 31)
    out = torch.empty_like(b)
    with pytest.raises(dgmg.DGMGError, match="scratch"):
        prob.vcycle_noalloc(b, out)
    b14 = b[:14].contiguous()
    ref, out = both(prob, b14)
    assert torch.equal(ref, out)
    prob.close()
