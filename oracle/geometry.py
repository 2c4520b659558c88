"""Cell maps, material and the pulled-back elasticity tensor.

Sec. 2.1: each cell is the unit square mapped into physical space; the maps
come from a shared Bezier control net so neighbouring cells agree on common
edges (untrimmed compatibility).  Sec. 2.2.1: plane linear elasticity with
the isotropic tensor C_ijkl, rewritten on the parametric domain through the
pulled-back tensor  Chat_{i j k l} = j dxi_j/dx_m C_{i m k n} dxi_l/dx_n
(the corrected index order of the pull-back equation).  Sec. 4.1: the fast
assembly interpolates Chat at the (q+1)^2 GLL points; the values there are
the geometry coefficients C_{i1 j1 i2 j2 k3}.
"""
import numpy as np
from .basis import bernstein, bernstein_deriv, interp_nodes


def cell_control_points(ctrl, m, ix, iy):
    """Control points X[b, a, :] of cell (ix, iy) taken from the shared net
    (Bezier extraction of a C^0 spline: cells share boundary rows)."""
    return ctrl[m * iy: m * iy + m + 1, m * ix: m * ix + m + 1, :]


def map_eval(X, xi1, xi2):
    """F(xi) = sum_ab X[b,a] B_a(xi1) B_b(xi2) and J[i, j] = dF_i/dxi_j at
    the points (xi1[k], xi2[k]).  Returns F [k, 2], J [k, 2, 2]."""
    m = X.shape[0] - 1
    B1, B2 = bernstein(m, xi1), bernstein(m, xi2)
    D1, D2 = bernstein_deriv(m, xi1), bernstein_deriv(m, xi2)
    npt = B1.shape[1]
    F = np.zeros((npt, 2))
    J = np.zeros((npt, 2, 2))
    for b in range(m + 1):
        for a in range(m + 1):
            F += np.outer(B1[a] * B2[b], X[b, a])
            J[:, :, 0] += np.outer(D1[a] * B2[b], X[b, a])
            J[:, :, 1] += np.outer(B1[a] * D2[b], X[b, a])
    return F, J


def lame(E, nu):
    """Plane-strain Lame constants (lambda, mu)."""
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def material_tensor(E, nu):
    """Isotropic C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)
    (Sec. 2.2.1)."""
    lam, mu = lame(E, nu)
    d = np.eye(2)
    C = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    C[i, j, k, l] = lam * d[i, j] * d[k, l] + mu * (d[i, k] * d[j, l] + d[i, l] * d[j, k])
    return C


def pulled_back_tensor(J, Cmat):
    """Chat[i1, j1, i2, j2] = det J * Jinv[j1, m] C[i1, m, i2, n] Jinv[j2, n]
    for each point (J [k, 2, 2]); Jinv[j, m] = dxi_j / dx_m."""
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    Jinv = np.linalg.inv(J)
    return np.einsum("k,kam,imjn,kbn->kiajb", det, Jinv, Cmat, Jinv), det


def geometry_coefficients(X, q, Cmat):
    """C_{i1 j1 i2 j2 k3} = Chat_{i1 j1 i2 j2}(xi_k3) at the (q+1)^2 GLL
    interpolation points (Sec. 4.1, interpolation of Chat).  Returns an array
    [2, 2, 2, 2, nL] indexed [i1, j1, i2, j2, k3] and det J at the points."""
    pts = interp_nodes(q)
    _, J = map_eval(X, pts[:, 0], pts[:, 1])
    Ch, det = pulled_back_tensor(J, Cmat)
    return np.moveaxis(Ch, 0, -1), det


def min_det_jacobian(X, n=None):
    """Smallest det J over a (2m+2)^2 Gauss-Legendre sample and the corners
    (regularity check of the map, Sec. 4.1)."""
    m = X.shape[0] - 1
    n = n or 2 * m + 2
    g, _ = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    g = np.concatenate([g, [0.0, 1.0]])
    a, b = np.meshgrid(g, g, indexing="xy")
    _, J = map_eval(X, a.ravel(), b.ravel())
    return float(np.min(J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]))
