"""Pins of the GLL module against textbook values and exactness properties."""
import numpy as np
import pytest

from oracle.gll import gll_nodes_weights, derivative_matrix, interpolation_matrix, legendre


def test_known_nodes_weights():
    x, w = gll_nodes_weights(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = gll_nodes_weights(3)
    assert np.allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = gll_nodes_weights(4)
    s = np.sqrt(3 / 7)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 13))
def test_quadrature_exactness(N):
    x, w = gll_nodes_weights(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(2 * N):  # exact to degree 2N-1
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, x ** p) - exact) < 1e-13
    # not exact at degree 2N: GLL sums L_N^2 to 2/N instead of the integral 2/(2N+1)
    assert abs(np.dot(w, legendre(N, x) ** 2) - 2.0 / N) < 1e-13


@pytest.mark.parametrize("N", range(1, 13))
def test_derivative_exact_on_polynomials(N):
    x, _ = gll_nodes_weights(N)
    D = derivative_matrix(N)
    for p in range(N + 1):
        dp = p * x ** (p - 1) if p > 0 else np.zeros_like(x)
        assert np.max(np.abs(D @ x ** p - dp)) < 1e-11 * max(1, N ** 2)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12  # derivative of a constant


@pytest.mark.parametrize("Nc,Nf", [(1, 3), (3, 7), (2, 5), (4, 9), (1, 2)])
def test_interpolation_reproduces_polynomials(Nc, Nf):
    xc, _ = gll_nodes_weights(Nc)
    xf, _ = gll_nodes_weights(Nf)
    J = interpolation_matrix(Nc, Nf)
    for p in range(Nc + 1):
        assert np.max(np.abs(J @ xc ** p - xf ** p)) < 1e-13
