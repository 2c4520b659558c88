"""Pins of the implicit-domain quadrature and the Table 1 level sets.

  - the four level sets at points where Table 1's formulas give round values
    by hand, their symmetries, and their gradients against central
    differences; the bilinear threshold takes mu_1..mu_4 at the corners
    bottom-left, bottom-right, top-left, top-right (Sec. 2.1.2);
  - the interval bounds contain every sampled value and derivative;
  - regions with closed-form integrals, given only through a level set:
    the outside of a circle (the circle family's exact polar tensor), a
    half-plane cut by a slanted line (the polygon, triangulated, with
    collapsed Gauss rules exact for polynomials), and the Schwarz Diamond at
    threshold 0, whose region is exactly a union of rectangles (its boundary
    lines cross at saddles of phi, the case the recursion can only bound);
  - area and moments of every family with a non-uniform threshold against
    an independent rule: adaptive Gauss-Kronrod along xi_1 of slice
    integrals whose ends come from dense sign sampling and Brent's method;
  - the rule converges: 12 and 20 points per segment agree to rounding.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import implicit as im
from oracle.basis import gauss_legendre
from oracle.trimmed import I_circle, I_tpms, integrate_points, rect_points

SD, SP, FRD, IWP = im.FAMILY_SCHWARZ_D, im.FAMILY_SCHWARZ_P, im.FAMILY_SCHOEN_FRD, im.FAMILY_SCHOEN_IWP

# a threshold vector inside each family's first parameter box (Sec. 5)
MU = {SD: [0.2, 0.8, 0.4, 0.6], SP: [0.1, 0.5, -0.3, 0.7], FRD: [-3.0, -1.0, -5.0, 0.2], IWP: [-2.0, 1.0, 0.5, 2.0]}


def phi0(fam, x, y):
    return im.TrimmedCell(fam, [0.0] * 4).f(np.atleast_1d(float(x)), np.atleast_1d(float(y)))[0]


@pytest.mark.parametrize("fam,pts", [
    (SD, [((0, 0), 1.0), ((0.5, 0), -1.0), ((0.5, 0.5), 1.0), ((0.25, 0.1), 0.0), ((0.7, 0.75), 0.0)]),
    (SP, [((0, 0), 1.0), ((0.5, 0), -1.0), ((0.5, 0.5), -3.0), ((0.25, 0.25), -1.0)]),
    (FRD, [((0, 0), -1.0), ((0.5, 0), 7.0), ((0.25, 0.25), -1.0), ((0.5, 0.5), -1.0)]),
    (IWP, [((0, 0), 3.0), ((0.5, 0.5), -5.0), ((0.5, 0), -5.0), ((0.25, 0.25), 1.0)]),
])
def test_level_set_values(fam, pts):
    for (x, y), v in pts:
        assert abs(phi0(fam, x, y) - v) < 1e-14
    rng = np.random.default_rng(1)
    for x, y in rng.random((20, 2)):
        # symmetric in xi_1 <-> xi_2, even about 1/2, periodic (trimmed compatibility, Sec. 2.1.3)
        v = phi0(fam, x, y)
        assert abs(phi0(fam, y, x) - v) < 1e-13
        assert abs(phi0(fam, 1 - x, y) - v) < 1e-13
        assert abs(phi0(fam, x + 1, y - 1) - v) < 1e-12


@pytest.mark.parametrize("fam", [SD, SP, FRD, IWP])
def test_gradient_vs_central_differences(fam):
    dom = im.TrimmedCell(fam, MU[fam])
    rng = np.random.default_rng(2)
    x, y = rng.random(50), rng.random(50)
    gx, gy = dom.grad(x, y)
    h = 1e-6
    fx = (dom.f(x + h, y) - dom.f(x - h, y)) / (2 * h)
    fy = (dom.f(x, y + h) - dom.f(x, y - h)) / (2 * h)
    scale = 1 + np.abs(gx).max() + np.abs(gy).max()
    assert np.abs(gx - fx).max() < 1e-7 * scale and np.abs(gy - fy).max() < 1e-7 * scale


def test_bilinear_threshold_corners():
    mu = [0.3, -1.0, 2.0, 0.5]
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for m, (x, y) in zip(mu, corners):
        assert abs(im.bilinear(mu, x, y) - m) < 1e-15
    # linear along the bottom edge, the mean of the corners at the centre
    assert abs(im.bilinear(mu, 0.25, 0) - (0.75 * mu[0] + 0.25 * mu[1])) < 1e-15
    assert abs(im.bilinear(mu, 0.5, 0.5) - sum(mu) / 4) < 1e-15
    d = im.bilinear_grad(mu, 0.3, 0.6)
    h = 1e-6
    assert abs(d[0] - (im.bilinear(mu, 0.3 + h, 0.6) - im.bilinear(mu, 0.3 - h, 0.6)) / (2 * h)) < 1e-9
    assert abs(d[1] - (im.bilinear(mu, 0.3, 0.6 + h) - im.bilinear(mu, 0.3, 0.6 - h)) / (2 * h)) < 1e-9


@pytest.mark.parametrize("fam", [SD, SP, FRD, IWP])
def test_interval_bounds_contain_samples(fam):
    dom = im.TrimmedCell(fam, MU[fam])
    rng = np.random.default_rng(3)
    for _ in range(60):
        x0, y0 = rng.random(2)
        w = 10.0 ** rng.uniform(-3, 0)
        x1, y1 = x0 + w, y0 + w * rng.uniform(0.3, 1.0)
        B, (gx, gy) = dom.bound(x0, x1, y0, y1), dom.gbound(x0, x1, y0, y1)
        X, Y = x0 + (x1 - x0) * rng.random(400), y0 + (y1 - y0) * rng.random(400)
        f = dom.f(X, Y)
        dx, dy = dom.grad(X, Y)
        assert B.lo <= f.min() and f.max() <= B.hi
        assert gx.lo <= dx.min() and dx.max() <= gx.hi
        assert gy.lo <= dy.min() and dy.max() <= gy.hi


class _CircleOutside:
    """phi = r^2 - |xi - c|^2: negative outside the disk."""

    def __init__(self, c, r):
        self.c, self.r2 = c, r * r

    def f(self, x, y):
        return self.r2 - (x - self.c) ** 2 - (y - self.c) ** 2

    def grad(self, x, y):
        return -2 * (x - self.c), -2 * (y - self.c)

    @staticmethod
    def _sq(a, b):
        lo = 0.0 if a <= 0 <= b else min(a * a, b * b)
        return im.Iv(lo, max(a * a, b * b))

    def bound(self, x0, x1, y0, y1):
        return (self.r2 - self._sq(x0 - self.c, x1 - self.c) - self._sq(y0 - self.c, y1 - self.c)).widened()

    def gbound(self, x0, x1, y0, y1):
        return (im.Iv(-2 * (x1 - self.c), -2 * (x0 - self.c)).widened(),
                im.Iv(-2 * (y1 - self.c), -2 * (y0 - self.c)).widened())


class _HalfPlane:
    """phi = a x + b y - c."""

    def __init__(self, a, b, c):
        self.a, self.b, self.c = a, b, c

    def f(self, x, y):
        return self.a * x + self.b * y - self.c

    def grad(self, x, y):
        return np.full_like(x, self.a), np.full_like(y, self.b)

    def bound(self, x0, x1, y0, y1):
        v = [self.a * x + self.b * y - self.c for x in (x0, x1) for y in (y0, y1)]
        return im.Iv(min(v), max(v)).widened()

    def gbound(self, *box):
        return im.Iv(self.a).widened(), im.Iv(self.b).widened()


def _rel(A, B):
    return np.abs(A - B).max() / np.abs(B).max()


@pytest.mark.parametrize("t", [0.15, 0.3])
def test_circle_given_implicitly(t):
    p, q = 4, 2
    I = integrate_points(p, q, *im.implicit_rule(_CircleOutside(0.5, 0.5 - t), 12))
    assert _rel(I, I_circle(p, q, t)) < 1e-12


def _polygon_rule(poly, n):
    """Fan triangulation of a convex polygon, each triangle by the collapsed
    (Duffy) square: x = P0 + u (P1 - P0) + u v (P2 - P1), |det| u du dv."""
    g, w = gauss_legendre(n, 0.0, 1.0)
    U, V = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    xs, ys, ws = [], [], []
    P0 = poly[0]
    for P1, P2 in zip(poly[1:-1], poly[2:]):
        e1, e2 = P1 - P0, P2 - P1
        det = abs(e1[0] * e2[1] - e1[1] * e2[0])
        X = P0[None, None, :] + U[..., None] * e1 + (U * V)[..., None] * e2
        xs.append(X[..., 0].ravel())
        ys.append(X[..., 1].ravel())
        ws.append((W * U * det).ravel())
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


def _clip_square(a, b, c):
    """The unit square's part with a x + b y < c (Sutherland-Hodgman)."""
    sq = [np.array(v, dtype=float) for v in [(0, 0), (1, 0), (1, 1), (0, 1)]]
    out = []
    for i in range(4):
        P, Q = sq[i], sq[(i + 1) % 4]
        fp, fq = a * P[0] + b * P[1] - c, a * Q[0] + b * Q[1] - c
        if fp < 0:
            out.append(P)
        if (fp < 0) != (fq < 0):
            out.append(P + (Q - P) * fp / (fp - fq))
    return out


@pytest.mark.parametrize("line", [(1.0, 0.4, 0.8), (-0.3, 1.0, 0.35), (0.7, -0.9, 0.1)])
def test_half_plane_against_polygon(line):
    p, q = 3, 2
    poly = _clip_square(*line)
    ref = integrate_points(p, q, *_polygon_rule(poly, 2 * p + q + 2))
    I = integrate_points(p, q, *im.implicit_rule(_HalfPlane(*line), 12))
    assert _rel(I, ref) < 1e-12


def test_schwarz_d_zero_threshold_is_rectangles():
    """cos(2 pi x) cos(2 pi y) < 0 exactly where one factor is negative: x in
    (1/4, 3/4) and y outside [1/4, 3/4], or the reverse."""
    p, q = 3, 2
    R = lambda a0, a1, b0, b1: integrate_points(p, q, *rect_points(p, q, a0, a1, b0, b1))
    ref = (R(0.25, 0.75, 0, 0.25) + R(0.25, 0.75, 0.75, 1) + R(0, 0.25, 0.25, 0.75) + R(0.75, 1, 0.25, 0.75))
    I = I_tpms(SD, p, q, [0.0] * 4)
    assert _rel(I, ref) < 1e-12


def _slice_moments(dom, x, nb=3, ns=4001):
    """[int over {y: phi(x, y) < 0} of y^b dy for b < nb]."""
    y = np.linspace(0.0, 1.0, ns)
    f = dom.f(np.full(ns, x), y)
    ends = [0.0]
    for i in np.nonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0]:
        ends.append(optimize.brentq(lambda s: dom.f(np.array([x]), np.array([s]))[0], y[i], y[i + 1], xtol=1e-15, rtol=1e-15))
    ends.append(1.0)
    out = np.zeros(nb)
    for a, b in zip(ends[:-1], ends[1:]):
        if dom.f(np.array([x]), np.array([0.5 * (a + b)]))[0] < 0:
            out += [(b ** (k + 1) - a ** (k + 1)) / (k + 1) for k in range(nb)]
    return out


@pytest.mark.parametrize("fam", [SD, SP, FRD, IWP])
def test_moments_against_slices(fam):
    dom = im.TrimmedCell(fam, MU[fam])
    X, Y, W = im.implicit_rule(dom, 12)
    mine = np.array([(W * X ** a * Y ** b).sum() for a in range(3) for b in range(3)])
    ref, _ = integrate.quad_vec(lambda x: np.outer(x ** np.arange(3), _slice_moments(dom, x)).ravel(),
                                0.0, 1.0, epsabs=1e-13, epsrel=1e-13, limit=4000)
    assert mine[0] > 0.05  # a real trimmed cell, not an empty or full one
    assert np.abs(mine - ref).max() < 1e-10


@pytest.mark.parametrize("fam", [SD, IWP])
def test_rule_converges(fam):
    p, q = 3, 2
    I12 = integrate_points(p, q, *im.tpms_rule(fam, MU[fam], 12))
    I20 = integrate_points(p, q, *im.tpms_rule(fam, MU[fam], 20))
    assert _rel(I12, I20) < 1e-13
