"""GPU checks of the differentiable solve u = A(kappa)^{-1} b (torch.autograd
around dgmg_pcg_solve, adjoint backward): gradients against the oracle's
dense adjoint, the closed form dL/dkappa = -(u - u_t)^T u / kappa and central
differences; the full-size 2-D Q5 256^2 workload against the oracle's exact
fast-diagonalisation solves."""
import sys

import numpy as np
import pytest

from oracle.adjoint import closed_form_dkappa, dense_adjoint
from oracle.fdsolve import GlobalFD
from oracle.rhs import interpolate, load_vector
from oracle.sipg import kron_operator
from paper_2405_18982_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_18982_amd import dgmg  # noqa: E402


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def loss_and_grads(prob, b_np, ut_np, kappa, rtol):
    b = torch.from_numpy(b_np).cuda().requires_grad_(True)
    kap = torch.tensor(kappa, dtype=torch.float64, device="cuda", requires_grad=True)
    ut = torch.from_numpy(ut_np).cuda()
    u = dgmg.solve(b, kap, prob, rtol=rtol)
    loss = 0.5 * ((u - ut) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (float(loss), u.detach().cpu().numpy(), b.grad.cpu().numpy(), float(kap.grad))


def test_gradients_small_against_dense_adjoint_and_fd():
    note("autograd 2-D Q2 8x8")
    dim, k, L, kappa = 2, 2, 2, 1.3
    N = 2 ** (L + 1)
    prob = dgmg.Problem(dim, k, L, kappa=kappa)
    rng = np.random.default_rng(21)
    b = rng.standard_normal(prob.ndofs())
    ut = 0.01 * rng.standard_normal(prob.ndofs())
    loss, u, gb, gk = loss_and_grads(prob, b, ut, kappa, rtol=1e-13)
    A1 = kron_operator(dim, k, N, inputs.sigma_of(k))
    u_o, loss_o, lam_o, dk_o = dense_adjoint(A1, kappa, b, ut)
    assert np.linalg.norm(u - u_o) <= 1e-10 * np.linalg.norm(u_o)
    assert abs(loss - loss_o) <= 1e-10 * abs(loss_o)
    assert np.linalg.norm(gb - lam_o) <= 1e-9 * np.linalg.norm(lam_o)
    assert abs(gk - dk_o) <= 1e-9 * abs(dk_o)
    assert abs(gk - closed_form_dkappa(u_o, ut, kappa)) <= 1e-9 * abs(dk_o)
    # central differences through the GPU forward with step 1e-6
    eps = 1e-6
    lp = loss_and_grads(prob, b, ut, kappa + eps, 1e-13)[0]
    lm = loss_and_grads(prob, b, ut, kappa - eps, 1e-13)[0]
    assert abs((lp - lm) / (2 * eps) - gk) <= 1e-5 * abs(gk)
    j = 17
    e = np.zeros_like(b)
    e[j] = eps
    lp = loss_and_grads(prob, b + e, ut, kappa, 1e-13)[0]
    lm = loss_and_grads(prob, b - e, ut, kappa, 1e-13)[0]
    assert abs((lp - lm) / (2 * eps) - gb[j]) <= 1e-5 * np.abs(gb).max()
    prob.close()


def test_gradients_3d_against_dense_adjoint():
    note("autograd 3-D Q2 8^3")
    dim, k, L, kappa = 3, 2, 2, 0.8
    N = 2 ** (L + 1)
    prob = dgmg.Problem(dim, k, L, kappa=kappa)
    rng = np.random.default_rng(22)
    b = rng.uniform(-1, 1, prob.ndofs())
    ut = 0.1 * rng.uniform(-1, 1, prob.ndofs())
    loss, u, gb, gk = loss_and_grads(prob, b, ut, kappa, rtol=1e-12)
    A1 = kron_operator(dim, k, N, inputs.sigma_of(k))
    u_o, loss_o, lam_o, dk_o = dense_adjoint(A1, kappa, b, ut)
    assert np.linalg.norm(gb - lam_o) <= 1e-8 * np.linalg.norm(lam_o)
    assert abs(gk - dk_o) <= 1e-8 * abs(dk_o)
    prob.close()


def test_full_size_poisson2d_q5_256c_adjoint():
    """2-D Q5, 256^2 cells (2,359,296 DoFs), kappa = 1, Fourier load (32 seeded
    modes) and target (second seed): forward and adjoint solves against the
    oracle's exact global fast-diagonalisation solves; dL/dkappa against the
    closed form on the oracle's solution."""
    note("autograd full size 2-D Q5 256^2")
    w = inputs.WORKLOADS["poisson2d_q5_256c_adjoint"]
    dim, k, L, kappa = w["dim"], w["k"], w["L"], w["kappa"]
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    modes_f = inputs.fourier_modes(w["seed"])
    modes_t = inputs.fourier_modes(w["target_seed"])
    b = load_vector(dim, k, N, lambda X: inputs.fourier_field(modes_f, X))
    ut = interpolate(dim, k, N, lambda X: inputs.fourier_field(modes_t, X))
    prob = dgmg.Problem(dim, k, L, kappa=kappa)
    loss, u, gb, gk = loss_and_grads(prob, b, ut, kappa, rtol=1e-12)
    fd = GlobalFD(dim, k, N, sig, kappa)
    u_o = fd.solve(b)
    lam_o = fd.solve(u_o - ut)
    assert np.linalg.norm(u - u_o) <= 1e-9 * np.linalg.norm(u_o)
    assert np.linalg.norm(gb - lam_o) <= 1e-9 * np.linalg.norm(lam_o)
    dk_o = closed_form_dkappa(u_o, ut, kappa)
    assert abs(gk - dk_o) <= 1e-8 * abs(dk_o)
    prob.close()


def test_batched_right_hand_sides_share_one_kappa():
    """b of shape (3, ndofs) with one kappa: dL/db per right-hand side equals
    the dense adjoint, and dL/dkappa is the sum of the three single-RHS
    gradients (dense adjoint per right-hand side); the library's per-RHS
    values of -lambda_j^T A_1 u_j match the closed form on each."""
    note("autograd 2-D Q2 8x8, 3 right-hand sides")
    dim, k, L, kappa = 2, 2, 2, 0.7
    N = 2 ** (L + 1)
    prob = dgmg.Problem(dim, k, L, kappa=kappa, nrhs_max=3)
    rng = np.random.default_rng(23)
    n = prob.ndofs()
    b = rng.standard_normal((3, n))
    ut = 0.05 * rng.standard_normal((3, n))
    loss, u, gb, gk = loss_and_grads(prob, b, ut, kappa, rtol=1e-13)
    A1 = kron_operator(dim, k, N, inputs.sigma_of(k))
    dks = []
    for j in range(3):
        u_o, _, lam_o, dk_o = dense_adjoint(A1, kappa, b[j], ut[j])
        assert np.linalg.norm(u[j] - u_o) <= 1e-10 * np.linalg.norm(u_o)
        assert np.linalg.norm(gb[j] - lam_o) <= 1e-9 * np.linalg.norm(lam_o)
        dks.append(dk_o)
    assert abs(gk - sum(dks)) <= 1e-9 * sum(abs(d) for d in dks)
    # the library call itself, per right-hand side
    lam = torch.from_numpy(gb).cuda()
    per, tot = prob.adjoint_dkappa(lam, torch.from_numpy(u).cuda())
    for j in range(3):
        assert abs(per[j] - closed_form_dkappa(u[j], ut[j], kappa)) <= 1e-9 * abs(dks[j])
    assert tot == sum(per.tolist())  # summed in index order
    prob.close()


def test_mismatched_right_hand_side_counts_raise():
    """Every secondary tensor must hold as many right-hand sides as the first
    one; the binding raises before any launch."""
    note("binding nrhs checks")
    prob = dgmg.Problem(2, 2, 2, nrhs_max=2)
    n, nc = prob.ndofs(), prob.ndofs(1)
    two = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    one = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        prob.apply(two, out=one)
    with pytest.raises(ValueError):
        prob.smooth(two, one)
    with pytest.raises(ValueError):
        prob.restrict_residual(two, one)
    with pytest.raises(ValueError):
        prob.prolongate_add(torch.zeros(nc, dtype=torch.float64, device="cuda"), two)
    with pytest.raises(ValueError):
        prob.vcycle(two, out=one)
    with pytest.raises(ValueError):
        prob.dot(two, one)
    with pytest.raises(ValueError):
        prob.solve(two, out=one)
    with pytest.raises(ValueError):
        prob.solve(two, x0=one)
    with pytest.raises(ValueError):
        prob.adjoint_dkappa(two, one)
    # x0 is not overwritten by the solve
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x, _, _ = prob.solve(b, x0=x0)
    assert float(x0.abs().max()) == 0.0 and float(x.abs().max()) > 0.0
    prob.close()
