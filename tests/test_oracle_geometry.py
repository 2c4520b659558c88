"""Pins of the map, material and pulled-back tensor."""
import numpy as np
from oracle import geometry as g
from oracle.adjoint import chat_dJ


def test_material_plane_strain():
    C = g.material_tensor(1.0, 0.3)
    lam, mu = 0.3 / (1.3 * 0.4), 1 / 2.6
    # Voigt entries: C1111 = lam + 2 mu, C1122 = lam, C1212 = mu
    assert abs(C[0, 0, 0, 0] - (lam + 2 * mu)) < 1e-15
    assert abs(C[0, 0, 1, 1] - lam) < 1e-15
    assert abs(C[0, 1, 0, 1] - mu) < 1e-15
    assert abs(C[0, 1, 1, 0] - mu) < 1e-15


def test_pullback_identity_and_scaling():
    C = g.material_tensor(2.0, 0.25)
    J = np.eye(2)[None]
    Ch, det = g.pulled_back_tensor(J, C)
    np.testing.assert_allclose(Ch[0], C, atol=1e-15)
    # uniform scaling x = s xi: Chat = s^2 * (1/s)(1/s) C = C in 2D
    Ch, _ = g.pulled_back_tensor(3.0 * np.eye(2)[None], C)
    np.testing.assert_allclose(Ch[0], C, atol=1e-14)
    # stretch x1 = a xi1: Chat_{i1 j1 i2 j2} = a C_{i1 m i2 n} A_{j1 m} A_{j2 n}, A = diag(1/a, 1)
    a = 2.5
    Ch, _ = g.pulled_back_tensor(np.diag([a, 1.0])[None], C)
    assert abs(Ch[0][0, 0, 0, 0] - a * C[0, 0, 0, 0] / a**2) < 1e-14
    assert abs(Ch[0][0, 1, 0, 1] - a * C[0, 1, 0, 1]) < 1e-14


def test_map_jacobian_fd():
    rng = np.random.default_rng(1)
    X = np.stack(np.meshgrid(np.arange(4) / 3, np.arange(4) / 3, indexing="xy"), -1) + 0.03 * rng.normal(size=(4, 4, 2))
    x1, x2 = rng.random(6), rng.random(6)
    F, J = g.map_eval(X, x1, x2)
    h = 1e-6
    fd0 = (g.map_eval(X, x1 + h, x2)[0] - g.map_eval(X, x1 - h, x2)[0]) / (2 * h)
    fd1 = (g.map_eval(X, x1, x2 + h)[0] - g.map_eval(X, x1, x2 - h)[0]) / (2 * h)
    np.testing.assert_allclose(J[:, :, 0], fd0, atol=1e-8)
    np.testing.assert_allclose(J[:, :, 1], fd1, atol=1e-8)
    # corner interpolation of a Bezier patch
    F0, _ = g.map_eval(X, np.array([0.0, 1.0]), np.array([0.0, 1.0]))
    np.testing.assert_allclose(F0, [X[0, 0], X[3, 3]], atol=1e-15)


def test_chat_derivative_fd():
    C = g.material_tensor(1.0, 0.3)
    rng = np.random.default_rng(2)
    J = np.eye(2) + 0.2 * rng.normal(size=(2, 2))
    D = chat_dJ(J[None], C)[0]
    h = 1e-6
    for p in range(2):
        for q in range(2):
            E = np.zeros((2, 2))
            E[p, q] = h
            fd = (g.pulled_back_tensor((J + E)[None], C)[0][0] - g.pulled_back_tensor((J - E)[None], C)[0][0]) / (2 * h)
            np.testing.assert_allclose(D[..., p, q], fd, atol=1e-8)
