"""Trimmed-domain integrals of the fast-assembly tensor.

Sec. 4.2, definition of I(mu): the integral over the trimmed parametric
domain of vec(dB_k1/dxi_j1 dB_k2/dxi_j2 L_k3), with dB the GLL basis
gradients and L the degree-q interpolation basis.  We keep I as an array
indexed [k1, k2, j1, j2, k3]; vec() is C-order flattening, so the position of
(k1, k2, j1, j2, k3) is (((k1*nB + k2)*2 + j1)*2 + j2)*nL + k3.

The integrand is a polynomial of total degree at most 4p - 2 + 2q and of
degree at most 2p + q in each variable.  Both stand-in families are trimmed
by circles or axis-aligned lines, so every integral below is exact up to
rounding:
  * rectangles: tensor Gauss-Legendre with ceil((2p+q+1)/2)+1 points;
  * disks: Gauss-Legendre in the radius (ceil((D+2)/2) points, the measure
    r dr raises the degree by one) times the trapezoidal rule in the angle
    (D + 2 points, exact for trigonometric polynomials of degree <= D).
I_Pi is the same integral over the untrimmed square (Sec. 4.1, stabilisation
term split into square minus trimmed domain).

The level sets of Table 1 with the bilinear threshold (Sec. 2.1.2) trim by
curves that are neither circles nor lines; their cells are integrated by the
implicit-domain quadrature of implicit.py with max(12, p + q + 2) Gauss
points per segment (exact along every segment, since the integrand has
degree at most 2p + q in each variable, and converged to rounding across
segments).
"""
import numpy as np
from .basis import tensor_basis, interp_basis, gauss_legendre
from .implicit import TPMS_FAMILIES, tpms_rule

FAMILY_CIRCLE = 0
FAMILY_CROSS = 1


def integrate_points(p, q, x1, x2, w):
    """I[k1, k2, j1, j2, k3] = sum_k w_k dB[k1,j1](x_k) dB[k2,j2](x_k) L[k3](x_k)."""
    _, dB = tensor_basis(p, x1, x2)
    L = interp_basis(q, x1, x2)
    nB, nL = (p + 1) ** 2, (q + 1) ** 2
    I = np.zeros((nB, nB, 2, 2, nL))
    for j1 in range(2):
        for j2 in range(2):
            for k3 in range(nL):
                I[:, :, j1, j2, k3] = (dB[:, j1, :] * (w * L[k3])) @ dB[:, j2, :].T
    return I


def rect_points(p, q, a0, a1, b0, b1):
    n = (2 * p + q + 1 + 1) // 2 + 1
    x, wx = gauss_legendre(n, a0, a1)
    y, wy = gauss_legendre(n, b0, b1)
    X, Y = np.meshgrid(x, y, indexing="xy")
    W = np.outer(wy, wx)
    return X.ravel(), Y.ravel(), W.ravel()


def disk_points_polar(p, q, cx, cy, r, extra=0):
    D = 4 * p - 2 + 2 * q + extra
    nr = (D + 2 + 1) // 2
    nt = D + 2
    rho, wr = gauss_legendre(nr, 0.0, r)
    th = 2.0 * np.pi * np.arange(nt) / nt
    R, T = np.meshgrid(rho, th, indexing="xy")
    W = np.outer(np.full(nt, 2.0 * np.pi / nt), wr * rho)
    return (cx + R * np.cos(T)).ravel(), (cy + R * np.sin(T)).ravel(), W.ravel()


def disk_points_slices(p, q, cx, cy, r, nphi=None):
    """Second, independent disk rule: horizontal slices y = cy + r sin(phi),
    exact Gauss-Legendre in x on each slice, Gauss-Legendre in phi (the
    integrand is analytic in phi, so this converges to rounding)."""
    D = 4 * p - 2 + 2 * q
    nphi = nphi or 2 * D + 24
    phi, wphi = gauss_legendre(nphi, -0.5 * np.pi, 0.5 * np.pi)
    nx = (2 * p + q + 1 + 1) // 2 + 1
    gx, gw = gauss_legendre(nx, -1.0, 1.0)
    xs, ys, ws = [], [], []
    for ph, wp in zip(phi, wphi):
        h = r * np.cos(ph)
        y = cy + r * np.sin(ph)
        xs.append(cx + h * gx)
        ys.append(np.full(nx, y))
        ws.append(gw * h * (r * np.cos(ph)) * wp)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


def I_square(p, q):
    """I_Pi: the integral over the untrimmed cell."""
    return integrate_points(p, q, *rect_points(p, q, 0.0, 1.0, 0.0, 1.0))


def I_circle(p, q, t, I_pi=None, method="polar"):
    """Circle family: material is the square minus the disk of radius
    1/2 - t centred at (1/2, 1/2); I = I_Pi - I_disk."""
    r = 0.5 - t
    if not (0.0 < r < 0.5):
        raise ValueError("circle family needs 0 < t < 1/2")
    if I_pi is None:
        I_pi = I_square(p, q)
    pts = disk_points_polar(p, q, 0.5, 0.5, r) if method == "polar" else disk_points_slices(p, q, 0.5, 0.5, r)
    return I_pi - integrate_points(p, q, *pts)


def I_cross(p, q, t, method="union"):
    """Cross family: material is the union of the strips |xi1 - 1/2| < t/2
    and |xi2 - 1/2| < t/2.  'union' = inclusion-exclusion of the two strips,
    'pieces' = sum over the five disjoint rectangles."""
    if not (0.0 < t < 1.0):
        raise ValueError("cross family needs 0 < t < 1")
    lo, hi = 0.5 - 0.5 * t, 0.5 + 0.5 * t
    R = lambda a0, a1, b0, b1: integrate_points(p, q, *rect_points(p, q, a0, a1, b0, b1))
    if method == "union":
        return R(lo, hi, 0.0, 1.0) + R(0.0, 1.0, lo, hi) - R(lo, hi, lo, hi)
    return (R(lo, hi, lo, hi) + R(0.0, lo, lo, hi) + R(hi, 1.0, lo, hi)
            + R(lo, hi, 0.0, lo) + R(lo, hi, hi, 1.0))


def tpms_points(p, q, mu, family, extra=0):
    return tpms_rule(family, mu, max(12, p + q + 2) + extra)


def I_tpms(family, p, q, mu):
    """I(mu) of a Table 1 level set with corner thresholds mu[4]."""
    return integrate_points(p, q, *tpms_points(p, q, mu, family))


def param_dim(family):
    """Number of geometric parameters of a cell of `family`."""
    return 4 if int(family) in TPMS_FAMILIES else 1


def I_exact(family, p, q, t, I_pi=None):
    """Exact I(t) for a cell of `family` with parameter t (the thickness of
    the stand-in families, the four corner thresholds of the TPMS ones)."""
    if family == FAMILY_CIRCLE:
        return I_circle(p, q, t, I_pi)
    if family == FAMILY_CROSS:
        return I_cross(p, q, t)
    if int(family) in TPMS_FAMILIES:
        return I_tpms(family, p, q, t)
    raise ValueError(f"unknown family {family}")


def material_points(family, p, q, t, extra=0):
    """Signed quadrature points covering the material region (weights of
    removed parts are negative).  Used by the full-quadrature reference."""
    if int(family) in TPMS_FAMILIES:
        return tpms_points(p, q, t, family, extra=extra)
    if family == FAMILY_CIRCLE:
        n = (2 * p + q + 1 + 1) // 2 + 1 + extra
        x, wx = gauss_legendre(n)
        X, Y = np.meshgrid(x, x, indexing="xy")
        W = np.outer(wx, wx)
        dx, dy, dw = disk_points_polar(p, q, 0.5, 0.5, 0.5 - t, extra=2 * extra)
        return (np.concatenate([X.ravel(), dx]), np.concatenate([Y.ravel(), dy]),
                np.concatenate([W.ravel(), -dw]))
    lo, hi = 0.5 - 0.5 * t, 0.5 + 0.5 * t
    parts = []
    for (a0, a1, b0, b1, s) in [(lo, hi, 0, 1, 1), (0, 1, lo, hi, 1), (lo, hi, lo, hi, -1)]:
        n = (2 * p + q + 1 + 1) // 2 + 1 + extra
        x, wx = gauss_legendre(n, a0, a1)
        y, wy = gauss_legendre(n, b0, b1)
        X, Y = np.meshgrid(x, y, indexing="xy")
        parts.append((X.ravel(), Y.ravel(), s * np.outer(wy, wx).ravel()))
    return tuple(np.concatenate([pp[i] for pp in parts]) for i in range(3))


def square_points(p, q, extra=0):
    n = (2 * p + q + 1 + 1) // 2 + 1 + extra
    x, wx = gauss_legendre(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    return X.ravel(), Y.ravel(), np.outer(wx, wx).ravel()
