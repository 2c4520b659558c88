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


def _bilinear_net(m, a, b):
    """Bezier net of order m of the bilinear map with corners (0,0), (1,0),
    (0,1), (a,b).  The map is linear in each coordinate separately, so its
    order-m Bernstein coefficients are its values at the points (i/m, j/m)."""
    t = np.arange(m + 1) / m
    x1, x2 = np.meshgrid(t, t, indexing="xy")       # [b, a]
    P00, P10, P01, P11 = map(np.array, ([0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [a, b]))
    w = lambda u, v: ((1 - u) * (1 - v))[..., None] * P00 + (u * (1 - v))[..., None] * P10 \
        + ((1 - u) * v)[..., None] * P01 + (u * v)[..., None] * P11
    return w(x1, x2)


def test_min_det_jacobian_closed_form():
    """For the bilinear map with corners (0,0), (1,0), (0,1), (a,b),
    det J = 1 + (b - 1) xi1 + (a - 1) xi2 exactly (the xi1 xi2 terms cancel),
    so its minimum over the unit square is min(1, b, a, a + b - 1), taken at a
    corner.  Checked for the same map written as nets of order 1, 2 and 3."""
    for m in (1, 2, 3):
        # a fold confined to the corner (1, 1): every interior Gauss point of
        # the (2m+2)^2 sample has det J > 0, only the corner itself is negative
        a = b = 0.495
        X = _bilinear_net(m, a, b)
        assert abs(g.min_det_jacobian(X) - (a + b - 1.0)) < 1e-14
        assert g.min_det_jacobian(X) < 0
        gp, _ = np.polynomial.legendre.leggauss(2 * m + 2)
        gp = 0.5 * (gp + 1.0)
        assert 1 + (b - 1) * gp.max() + (a - 1) * gp.max() > 0
        # a regular map: the minimum (not the maximum 1.4) is the corner (0, 0)
        X = _bilinear_net(m, 1.2, 1.2)
        assert abs(g.min_det_jacobian(X) - 1.0) < 1e-14
        # a regular map whose minimum is the corner (1, 0): det = b
        X = _bilinear_net(m, 1.3, 0.6)
        assert abs(g.min_det_jacobian(X) - 0.6) < 1e-14
        # the mirrored net x -> -x flips the sign of det J everywhere:
        # min over the square of -(1 + 0.2 xi1 + 0.2 xi2) is -1.4 at (1, 1)
        X = _bilinear_net(m, 1.2, 1.2) * np.array([-1.0, 1.0])
        assert abs(g.min_det_jacobian(X) - (-1.4)) < 1e-14


def test_min_det_jacobian_affine():
    """An affine map x = A xi + c written as an order-m net has det J = det A."""
    rng = np.random.default_rng(5)
    for m in (1, 2, 3, 4):
        A = np.eye(2) + 0.3 * rng.normal(size=(2, 2))
        t = np.arange(m + 1) / m
        x1, x2 = np.meshgrid(t, t, indexing="xy")
        X = np.stack([x1, x2], -1) @ A.T + np.array([2.0, -1.0])
        assert abs(g.min_det_jacobian(X) - np.linalg.det(A)) < 1e-13


def test_cell_control_points_by_hand():
    """A 3 x 2 lattice with an order-2 net of 5 x 7 points, point (jx, jy)
    at (jx, 100 + jy): each cell's corner control points, written out."""
    m, nx, ny = 2, 3, 2
    jx, jy = np.meshgrid(np.arange(m * nx + 1), np.arange(m * ny + 1), indexing="xy")
    ctrl = np.stack([jx, 100 + jy], -1).astype(float)
    assert ctrl.shape == (5, 7, 2)
    # cell (ix, iy) -> X[0,0], X[0,m] (xi1 = 1), X[m,0] (xi2 = 1), X[m,m]
    expect = {
        (0, 0): [(0, 100), (2, 100), (0, 102), (2, 102)],
        (1, 0): [(2, 100), (4, 100), (2, 102), (4, 102)],
        (2, 0): [(4, 100), (6, 100), (4, 102), (6, 102)],
        (0, 1): [(0, 102), (2, 102), (0, 104), (2, 104)],
        (1, 1): [(2, 102), (4, 102), (2, 104), (4, 104)],
        (2, 1): [(4, 102), (6, 102), (4, 104), (6, 104)],
    }
    for (ix, iy), corners in expect.items():
        X = g.cell_control_points(ctrl, m, ix, iy)
        assert X.shape == (3, 3, 2)
        got = [tuple(X[0, 0]), tuple(X[0, m]), tuple(X[m, 0]), tuple(X[m, m])]
        assert got == [tuple(map(float, c)) for c in corners], (ix, iy, got)
        # the middle control point and the map's image of the cell centre
        assert tuple(X[1, 1]) == (2 * ix + 1.0, 100 + 2 * iy + 1.0)
        F, _ = g.map_eval(X, np.array([1.0, 0.5]), np.array([0.0, 0.5]))
        np.testing.assert_allclose(F, [[2 * ix + 2, 100 + 2 * iy], [2 * ix + 1, 101 + 2 * iy]], atol=1e-13)


def test_cell_control_points_on_the_annulus():
    """cell_control_points against the closed form of the benchmark's quarter
    annulus (no jitter): the map of cell (ix, iy) takes its parametric corners
    to the annulus points at s = ix/nx or (ix+1)/nx and u = iy/ny or
    (iy+1)/ny, x = -r sin(pi s / 2), y = -r cos(pi s / 2), r = 0.6 + 0.4 u.
    A lattice of 5 x 3 cells (nx != ny), so a transposed (ix, iy) or a
    swapped corner fails."""
    from workloads import make_problem
    prob = make_problem(7, nx=5, ny=3, p=4)
    nx, ny, m = prob["nx"], prob["ny"], prob["m"]

    def annulus(s, u):
        r = 0.6 + 0.4 * u
        return np.array([-r * np.sin(0.5 * np.pi * s), -r * np.cos(0.5 * np.pi * s)])

    for iy in range(ny):
        for ix in range(nx):
            X = g.cell_control_points(prob["ctrl"], m, ix, iy)
            for a in (0, 1):
                for b in (0, 1):
                    F, _ = g.map_eval(X, np.array([float(a)]), np.array([float(b)]))
                    np.testing.assert_allclose(F[0], annulus((ix + a) / nx, (iy + b) / ny), rtol=0, atol=1e-14)
