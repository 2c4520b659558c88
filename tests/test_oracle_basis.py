"""Pins of the oracle's polynomial bases against textbook closed forms."""
import numpy as np
import pytest
from oracle import basis


def test_gll_closed_forms():
    # textbook GLL points on [-1,1]: p=2: 0; p=3: +-1/sqrt5; p=4: 0, +-sqrt(3/7)
    np.testing.assert_allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s = 1 / np.sqrt(5)
    np.testing.assert_allclose(basis.gll_nodes(3), 0.5 * (1 + np.array([-1, -s, s, 1])), atol=1e-15)
    s = np.sqrt(3 / 7)
    np.testing.assert_allclose(basis.gll_nodes(4), 0.5 * (1 + np.array([-1, -s, 0, s, 1])), atol=1e-15)
    # weights p=4 on [-1,1]: 1/10, 49/90, 32/45
    np.testing.assert_allclose(basis.gll_weights(4), 0.5 * np.array([1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]), atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 6, 8, 12])
def test_gll_quadrature_exactness(p):
    x, w = basis.gll_nodes(p), basis.gll_weights(p)
    for k in range(2 * p):  # exact to degree 2p-1
        assert abs(w @ x**k - 1.0 / (k + 1)) < 1e-14


@pytest.mark.parametrize("p", [1, 3, 8])
def test_lagrange_interpolation_and_derivative(p):
    nodes = basis.gll_nodes(p)
    np.testing.assert_allclose(basis.lagrange(nodes, nodes), np.eye(p + 1), atol=1e-14)
    xs = np.linspace(0, 1, 17)
    L = basis.lagrange(nodes, xs)
    np.testing.assert_allclose(L.sum(0), 1.0, atol=1e-13)
    # reproduces x^p and its derivative p x^(p-1)
    np.testing.assert_allclose(nodes**p @ L, xs**p, atol=1e-13)
    dL = basis.lagrange_deriv(nodes, xs)
    np.testing.assert_allclose(nodes**p @ dL, p * xs ** (p - 1), atol=1e-11)
    np.testing.assert_allclose(dL.sum(0), 0.0, atol=1e-11)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_bernstein(m):
    x = np.linspace(0, 1, 11)
    B = basis.bernstein(m, x)
    np.testing.assert_allclose(B.sum(0), 1.0, atol=1e-15)
    # linear precision: sum a/m B_a = x
    np.testing.assert_allclose((np.arange(m + 1) / m) @ B, x, atol=1e-15)
    h = 1e-6
    fd = (basis.bernstein(m, x + h) - basis.bernstein(m, x - h)) / (2 * h)
    np.testing.assert_allclose(basis.bernstein_deriv(m, x), fd, atol=1e-8)


def test_tensor_basis_gradient_fd():
    p = 4
    rng = np.random.default_rng(0)
    x1, x2 = rng.random(5), rng.random(5)
    B, dB = basis.tensor_basis(p, x1, x2)
    h = 1e-6
    fd1 = (basis.tensor_basis(p, x1 + h, x2)[0] - basis.tensor_basis(p, x1 - h, x2)[0]) / (2 * h)
    fd2 = (basis.tensor_basis(p, x1, x2 + h)[0] - basis.tensor_basis(p, x1, x2 - h)[0]) / (2 * h)
    np.testing.assert_allclose(dB[:, 0], fd1, atol=1e-7)
    np.testing.assert_allclose(dB[:, 1], fd2, atol=1e-7)
