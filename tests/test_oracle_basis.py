"""Pins of the oracle's 1-D building blocks against textbook facts
(Appendix A: Lagrange basis on Gauss-Lobatto points of [0,1])."""
import numpy as np
import pytest

from oracle.basis import Basis1D, gll_nodes, gll_weights

KS = [1, 2, 3, 4, 5, 6, 7]


def test_gll_nodes_closed_forms():
    assert np.allclose(gll_nodes(1), [0, 1], atol=1e-15)
    assert np.allclose(gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s5 = 1 / np.sqrt(5)
    assert np.allclose(gll_nodes(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    s37 = np.sqrt(3 / 7)
    assert np.allclose(gll_nodes(4), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("k", KS)
def test_nodes_symmetric_sorted(k):
    x = gll_nodes(k)
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x + x[::-1], 1.0, atol=1e-15)


@pytest.mark.parametrize("k", KS)
def test_mass_rows_are_gll_weights(k):
    # sum_nu M[mu,nu] = int phi_mu = GLL weight (GLL is exact for degree 2k-1 >= k)
    b = Basis1D(k)
    assert np.allclose(b.M.sum(axis=1), gll_weights(k), atol=1e-15)
    assert abs(b.M.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("k", KS)
def test_stiffness_kernel_and_energy(k):
    b = Basis1D(k)
    assert np.allclose(b.K @ np.ones(k + 1), 0, atol=1e-13)
    # u = x: nodal values are the nodes, int (u')^2 = 1
    x = b.nodes
    assert abs(x @ b.K @ x - 1.0) < 1e-13
    # u = x^2: int (2x)^2 = 4/3 (exact for k >= 2)
    if k >= 2:
        assert abs((x ** 2) @ b.K @ (x ** 2) - 4.0 / 3.0) < 1e-12
    assert np.allclose(b.M, b.M.T, atol=1e-16)
    assert np.allclose(b.K, b.K.T, atol=1e-13)
    assert np.linalg.eigvalsh(b.M)[0] > 0


@pytest.mark.parametrize("k", KS)
def test_traces_and_end_derivatives(k):
    b = Basis1D(k)
    e0 = np.zeros(k + 1)
    e0[0] = 1
    assert np.allclose(b.e0, e0, atol=1e-14)
    assert np.allclose(b.e1, e0[::-1], atol=1e-14)
    x = b.nodes
    for j in range(k + 1):  # derivative of x^j at 0 and 1
        assert abs(b.d0 @ x ** j - (1.0 if j == 1 else 0.0)) < 1e-11
        assert abs(b.d1 @ x ** j - j) < 1e-10


@pytest.mark.parametrize("k", KS)
def test_prolongation_reproduces_polynomials(k):
    b = Basis1D(k)
    x = b.nodes
    for j in range(k + 1):
        for o in (0, 1):
            assert np.allclose(b.P[o] @ x ** j, ((x + o) / 2) ** j, atol=1e-13)
