"""Quadrature over an implicitly defined region {phi < 0} of a box.

Test infrastructure: the plain FP64 reference of the library, imported only
by the tests, the smoke check and the benchmark's CPU baseline.

The trimmed parametric cell of a level-set family is the part of the unit
square where phi = phi_0 - mu < 0 (Sec. 2.1.2), phi_0 one of the periodic
level sets of Table 1 and mu the bilinear threshold through the four corner
values.  Its integrals are computed, as the paper does (Sec. 2.2.3, the
height-function quadrature of QUGaR/algoim), by Saye's method (R. I. Saye,
High-order quadrature methods for implicitly defined surfaces and volumes in
hyperrectangles, SIAM J. Sci. Comput. 37 (2015) A993-A1019), in two
dimensions:

  1. bound phi over the box; if it keeps one sign the box lies entirely
     inside (tensor Gauss rule) or outside (no points);
  2. otherwise look for a height direction k in which d phi / d xi_k keeps one
     sign over the box, so that every line along xi_k crosses the boundary at
     most once; without one, split the box into four and start again;
  3. with a height direction: seen from the other (base) direction j, the
     inside part of a line along xi_k changes form only where phi vanishes on
     the two faces xi_k = a_k and xi_k = b_k; those roots split [a_j, b_j]
     into pieces, each gets a Gauss rule in xi_j, and at each of its points
     the root of phi along xi_k (one sign change at most: Newton inside the
     sign-change bracket) ends the
     inside segment, which gets a Gauss rule in xi_k.  The outer rule is made
     adaptive (a piece is halved until halving no longer changes its result),
     so that the oracle reaches rounding level where the height function
     varies fast; Saye's fixed-order rule is the first level of it.

Bounds come from interval arithmetic (exact ranges of cos and sin over an
interval, the bilinear threshold's range from the box corners, products and
sums of intervals), widened by a few ulps, so a box is taken as one-signed or
monotone only when it is.  Where phi and its gradient vanish together on the
boundary (a saddle of phi at the threshold value) no direction becomes
monotone; the recursion stops at depth `max_depth`, and that box, of area
4^-max_depth, keeps only the points of its tensor rule with phi < 0.
"""
import functools
import math

import numpy as np

from .basis import gauss_legendre as _gauss_legendre


@functools.lru_cache(maxsize=None)
def _gauss01(n):
    return _gauss_legendre(n, 0.0, 1.0)


def gauss_legendre(n, a, b):
    """n-point Gauss-Legendre rule on [a, b] (the [0, 1] rule, cached, scaled)."""
    x, w = _gauss01(n)
    return a + (b - a) * x, (b - a) * w

TWO_PI = 2.0 * math.pi

FAMILY_SCHWARZ_D = 2
FAMILY_SCHWARZ_P = 3
FAMILY_SCHOEN_FRD = 4
FAMILY_SCHOEN_IWP = 5
TPMS_FAMILIES = (FAMILY_SCHWARZ_D, FAMILY_SCHWARZ_P, FAMILY_SCHOEN_FRD, FAMILY_SCHOEN_IWP)


class Iv:
    """A closed interval [lo, hi] with the arithmetic the bounds need."""
    __slots__ = ("lo", "hi")

    def __init__(self, lo, hi=None):
        self.lo = float(lo)
        self.hi = float(lo if hi is None else hi)

    @staticmethod
    def of(v):
        return v if isinstance(v, Iv) else Iv(v)

    def __add__(self, o):
        o = Iv.of(o)
        return Iv(self.lo + o.lo, self.hi + o.hi)

    __radd__ = __add__

    def __neg__(self):
        return Iv(-self.hi, -self.lo)

    def __sub__(self, o):
        o = Iv.of(o)
        return Iv(self.lo - o.hi, self.hi - o.lo)

    def __rsub__(self, o):
        return Iv.of(o) - self

    def __mul__(self, o):
        o = Iv.of(o)
        c = (self.lo * o.lo, self.lo * o.hi, self.hi * o.lo, self.hi * o.hi)
        return Iv(min(c), max(c))

    __rmul__ = __mul__

    def widened(self):
        e = 1e-13 * (1.0 + max(abs(self.lo), abs(self.hi)))
        return Iv(self.lo - e, self.hi + e)

    def excludes_zero(self):
        return self.lo > 0.0 or self.hi < 0.0


def iv_cos(u):
    """Exact range of cos over the interval u (radians)."""
    u0, u1 = u.lo, u.hi
    if u1 - u0 >= TWO_PI:
        return Iv(-1.0, 1.0)
    c0, c1 = math.cos(u0), math.cos(u1)
    lo, hi = min(c0, c1), max(c0, c1)
    if TWO_PI * math.ceil(u0 / TWO_PI) <= u1:                      # a maximum 2 k pi inside
        hi = 1.0
    if TWO_PI * math.ceil((u0 - math.pi) / TWO_PI) + math.pi <= u1:  # a minimum (2 k + 1) pi inside
        lo = -1.0
    return Iv(lo, hi)


def iv_sin(u):
    """Exact range of sin over u: sin(v) = cos(v - pi/2)."""
    return iv_cos(Iv(u.lo - 0.5 * math.pi, u.hi - 0.5 * math.pi))


# ---------------------------------------------------------------------------
# The level sets of Table 1, written once for numpy arrays and for intervals:
# C(n, x) = cos(2 pi n x), S(n, x) = sin(2 pi n x).  Each returns
# (phi_0, d phi_0 / d xi_1, d phi_0 / d xi_2).

def _schwarz_d(C, S, x, y):
    return (C(1, x) * C(1, y),
            -TWO_PI * S(1, x) * C(1, y),
            -TWO_PI * C(1, x) * S(1, y))


def _schwarz_p(C, S, x, y):
    return (C(1, x) + C(1, y) - 1.0,
            -TWO_PI * S(1, x),
            -TWO_PI * S(1, y))


def _schoen_frd(C, S, x, y):
    return (C(2, x) * C(2, y) + C(2, y) + C(2, x) - 4.0 * C(1, x) * C(1, y),
            -2.0 * TWO_PI * S(2, x) * C(2, y) - 2.0 * TWO_PI * S(2, x) + 4.0 * TWO_PI * S(1, x) * C(1, y),
            -2.0 * TWO_PI * C(2, x) * S(2, y) - 2.0 * TWO_PI * S(2, y) + 4.0 * TWO_PI * C(1, x) * S(1, y))


def _schoen_iwp(C, S, x, y):
    return (2.0 * (C(1, x) * C(1, y) + C(1, y) + C(1, x)) - C(2, x) - C(2, y) - 1.0,
            -2.0 * TWO_PI * (S(1, x) * C(1, y) + S(1, x)) + 2.0 * TWO_PI * S(2, x),
            -2.0 * TWO_PI * (C(1, x) * S(1, y) + S(1, y)) + 2.0 * TWO_PI * S(2, y))


LEVEL_SETS = {FAMILY_SCHWARZ_D: _schwarz_d, FAMILY_SCHWARZ_P: _schwarz_p,
              FAMILY_SCHOEN_FRD: _schoen_frd, FAMILY_SCHOEN_IWP: _schoen_iwp}


def _np_C(n, x):
    return np.cos(TWO_PI * n * x)


def _np_S(n, x):
    return np.sin(TWO_PI * n * x)


def _iv_C(n, x):
    return iv_cos(Iv(TWO_PI * n * x.lo, TWO_PI * n * x.hi))


def _iv_S(n, x):
    return iv_sin(Iv(TWO_PI * n * x.lo, TWO_PI * n * x.hi))


def bilinear(mu, x, y):
    """mu(xi) = sum_i l_i(xi) mu_i with the corners ordered bottom-left,
    bottom-right, top-left, top-right (Sec. 2.1.2)."""
    return (mu[0] * (1.0 - x) * (1.0 - y) + mu[1] * x * (1.0 - y)
            + mu[2] * (1.0 - x) * y + mu[3] * x * y)


def bilinear_grad(mu, x, y):
    return ((mu[1] - mu[0]) * (1.0 - y) + (mu[3] - mu[2]) * y,
            (mu[2] - mu[0]) * (1.0 - x) + (mu[3] - mu[1]) * x)


class TrimmedCell:
    """phi = phi_0 - mu of one family and one corner-threshold vector."""

    def __init__(self, family, mu):
        self.phi0 = LEVEL_SETS[int(family)]
        self.mu = [float(v) for v in mu]

    def f(self, x, y):
        return self.phi0(_np_C, _np_S, x, y)[0] - bilinear(self.mu, x, y)

    def grad(self, x, y):
        _, gx, gy = self.phi0(_np_C, _np_S, x, y)
        mx, my = bilinear_grad(self.mu, x, y)
        return gx - mx, gy - my

    def bound(self, x0, x1, y0, y1):
        v = self.phi0(_iv_C, _iv_S, Iv(x0, x1), Iv(y0, y1))[0]
        m = [bilinear(self.mu, a, b) for a in (x0, x1) for b in (y0, y1)]
        return (v - Iv(min(m), max(m))).widened()

    def gbound(self, x0, x1, y0, y1):
        _, gx, gy = self.phi0(_iv_C, _iv_S, Iv(x0, x1), Iv(y0, y1))
        mx = [bilinear_grad(self.mu, 0.0, b)[0] for b in (y0, y1)]
        my = [bilinear_grad(self.mu, a, 0.0)[1] for a in (x0, x1)]
        return (Iv.of(gx) - Iv(min(mx), max(mx))).widened(), (Iv.of(gy) - Iv(min(my), max(my))).widened()


# ---------------------------------------------------------------------------

def _root(F, dF, a, b, neg_at_a, max_iter=200):
    """Roots of F (vectorised over its points) between a and b, where F has
    exactly one sign change and is negative at a where neg_at_a: Newton steps
    kept inside the shrinking sign-change bracket (a step that leaves it is
    replaced by the bracket's midpoint), until the step or the bracket is at
    rounding level."""
    lo = np.full(neg_at_a.shape, float(a))
    hi = np.full(neg_at_a.shape, float(b))
    x = 0.5 * (lo + hi)
    for _ in range(max_iter):
        f = F(x)
        same = (f < 0.0) == neg_at_a
        lo = np.where(same, x, lo)
        hi = np.where(same, hi, x)
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = x - f / dF(x)
        bad = ~((xn > lo) & (xn < hi))
        xn = np.where(bad, 0.5 * (lo + hi), xn)
        tol = 4e-16 * (1.0 + np.abs(x))
        done = (np.abs(xn - x) <= tol) | (hi - lo <= tol) | (f == 0.0)
        x = np.where(f == 0.0, x, xn)
        if done.all():
            return x
    raise RuntimeError("implicit quadrature: root iteration did not converge")


def _face_roots(dom, k, face, a, b, depth=0, max_depth=48):
    """Roots in [a, b] of phi restricted to the face xi_k = face, as a function
    of the other coordinate."""
    box = (a, b, face, face) if k == 1 else (face, face, a, b)
    B = dom.bound(*box)
    if B.excludes_zero():
        return []
    if max(abs(B.lo), abs(B.hi)) < 1e-11:
        # phi vanishes on this part of the face to rounding (the face lies on
        # the boundary, e.g. a dyadic box edge on a straight zero line): the
        # inside segments are then the same with or without a break here
        return []
    g = dom.gbound(*box)[1 - k]

    def F(s):
        return dom.f(s, np.full_like(s, face)) if k == 1 else dom.f(np.full_like(s, face), s)

    def dF(s):
        return dom.grad(s, np.full_like(s, face))[0] if k == 1 else dom.grad(np.full_like(s, face), s)[1]

    fa, fb = F(np.array([a]))[0], F(np.array([b]))[0]
    if g.excludes_zero():
        if (fa < 0.0) != (fb < 0.0):
            return [float(_root(F, dF, a, b, np.array([fa < 0.0]))[0])]
        return []
    if depth >= max_depth:
        return [0.5 * (a + b)]
    m = 0.5 * (a + b)
    return _face_roots(dom, k, face, a, m, depth + 1, max_depth) + _face_roots(dom, k, face, m, b, depth + 1, max_depth)


def _tensor(x0, x1, y0, y1, n):
    x, wx = gauss_legendre(n, x0, x1)
    y, wy = gauss_legendre(n, y0, y1)
    X, Y = np.meshgrid(x, y, indexing="xy")
    return X.ravel(), Y.ravel(), np.outer(wy, wx).ravel()


def _height(dom, box, k, n_in, n_out, out, tol=1e-15, max_split=40):
    """Step 3 on a box where d phi / d xi_k has one sign.  The outer integrand
    is analytic on each piece between breaks but can vary fast (two boundary
    branches passing close to each other), so each piece is halved until the
    rule on the halves agrees with the rule on the whole, to `tol`, on the
    moments of the inside segments' ends; the halves are kept."""
    x0, x1, y0, y1 = box
    (ja, jb), (ka, kb) = ((x0, x1), (y0, y1)) if k == 1 else ((y0, y1), (x0, x1))

    def F(s, h):
        return dom.f(s, h) if k == 1 else dom.f(h, s)

    def dF(s, h):
        return dom.grad(s, h)[1] if k == 1 else dom.grad(h, s)[0]

    def segments(s0, s1):
        s, ws = gauss_legendre(n_out, s0, s1)
        fa, fb = F(s, np.full_like(s, ka)), F(s, np.full_like(s, kb))
        lo, hi = np.full_like(s, ka), np.full_like(s, kb)
        na, nb = fa < 0.0, fb < 0.0
        cut = na != nb
        if cut.any():
            sc = s[cut]
            r = _root(lambda h: F(sc, h), lambda h: dF(sc, h), ka, kb, na[cut])
            hi[cut] = np.where(na[cut], r, kb)
            lo[cut] = np.where(na[cut], ka, r)
        keep = na | nb
        s, ws, lo, hi = s[keep], ws[keep], lo[keep], hi[keep]
        mom = np.array([np.sum(ws * (hi ** e - lo ** e) * s ** j) for e in (1, 2, 3) for j in (0, 1)])
        return (s, ws, lo, hi), mom

    def piece(s0, s1, whole, depth):
        m = 0.5 * (s0 + s1)
        left, right = segments(s0, m), segments(m, s1)
        if depth >= max_split or np.abs(left[1] + right[1] - whole[1]).max() <= tol:
            return [left[0], right[0]]
        return piece(s0, m, left, depth + 1) + piece(m, s1, right, depth + 1)

    breaks = {ja, jb}
    for face in (ka, kb):
        breaks.update(_face_roots(dom, k, face, ja, jb))
    breaks = sorted(v for v in breaks if ja <= v <= jb)
    g, gw = gauss_legendre(n_in, 0.0, 1.0)
    for s0, s1 in zip(breaks[:-1], breaks[1:]):
        if not s1 > s0:
            continue
        for s, ws, lo, hi in piece(s0, s1, segments(s0, s1), 0):
            if len(s) == 0:
                continue
            h = lo[:, None] + (hi - lo)[:, None] * g[None, :]
            w = (ws * (hi - lo))[:, None] * gw[None, :]
            S = np.repeat(s, n_in)
            if k == 1:
                out.append((S, h.ravel(), w.ravel()))
            else:
                out.append((h.ravel(), S, w.ravel()))


def implicit_rule(dom, n, n_out=None, box=(0.0, 1.0, 0.0, 1.0), max_depth=24):
    """Points (x, y) and weights of a quadrature over {phi < 0} within `box`:
    n Gauss points along every inside segment and n_out (default n) along the
    base direction of each piece.  `dom` supplies f(x, y),
    grad(x, y), bound(box) and gbound(box) (the ranges of phi and of its two
    partial derivatives over a box)."""
    n_out = n_out or n
    out = []
    stack = [(tuple(box), 0)]
    visited = 0
    while stack:
        b, depth = stack.pop()
        visited += 1
        if visited > 1_000_000:
            raise RuntimeError("implicit_rule: more than 10^6 boxes (a boundary that is not resolved)")
        B = dom.bound(*b)
        if B.hi < 0.0:
            out.append(_tensor(*b, n))
            continue
        if B.lo > 0.0:
            continue
        gx, gy = dom.gbound(*b)
        cand = [(min(abs(gk.lo), abs(gk.hi)), k) for k, gk in enumerate((gx, gy)) if gk.excludes_zero()]
        if cand:
            _height(dom, b, max(cand)[1], n, n_out, out)
            continue
        x0, x1, y0, y1 = b
        if depth >= max_depth:
            X, Y, W = _tensor(*b, n)
            inside = dom.f(X, Y) < 0.0
            out.append((X[inside], Y[inside], W[inside]))
            continue
        xm, ym = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
        stack += [((x0, xm, y0, ym), depth + 1), ((xm, x1, y0, ym), depth + 1),
                  ((x0, xm, ym, y1), depth + 1), ((xm, x1, ym, y1), depth + 1)]
    if not out:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    return tuple(np.concatenate([o[i] for o in out]) for i in range(3))


def tpms_rule(family, mu, n, n_out=None):
    """Quadrature over the trimmed cell {phi_0 < mu} of a Table 1 family."""
    return implicit_rule(TrimmedCell(family, mu), n, n_out)
