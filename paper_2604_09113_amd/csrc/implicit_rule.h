// Quadrature rules over the trimmed cell {phi_0 < mu} of the level sets of
// Table 1 with the bilinear threshold of Sec. 2.1.2, for the offline stage of
// the method (the snapshot integrals of Sec. 4.2).  The paper integrates
// these cells with the height-function quadrature of QUGaR/algoim (Sec.
// 2.2.3), i.e. Saye's method (SIAM J. Sci. Comput. 37 (2015) A993); this is
// that method for two dimensions, written for one thread per rule so that
// the same code runs on the host and in a GPU kernel over thousands of
// parameter vectors at once:
//  * depth-first over boxes starting from the unit cell: interval bounds of
//    phi decide inside (tensor Gauss rule) or outside; otherwise a direction
//    k in which d phi / d xi_k keeps one sign makes phi monotone along xi_k
//    (height direction); without one the box splits into four, down to a
//    depth limit where the box keeps the points of its tensor rule with
//    phi < 0;
//  * in a height box the base interval splits at the roots of phi on the
//    two faces xi_k = const; each piece gets n Gauss points, and at each the
//    root of phi along xi_k (Newton inside the sign-change bracket) ends the
//    inside segment, which gets n Gauss points; a piece is halved until the
//    halves reproduce it (to 1e-15 on six moments of the segment ends).
// Intervals: exact ranges of cos over an interval, sums and products of
// intervals, the bilinear threshold's range from the box corners; every
// bound is widened by 1e-13 (1 + |bound|).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace lbddc {
namespace rule {

#define RULE_HD __host__ __device__ inline

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.1415926535897932384626433832795;

struct Iv {
  double lo, hi;
};
RULE_HD Iv ivc(double a) { return {a, a}; }
RULE_HD Iv operator+(Iv a, Iv b) { return {a.lo + b.lo, a.hi + b.hi}; }
RULE_HD Iv operator-(Iv a, Iv b) { return {a.lo - b.hi, a.hi - b.lo}; }
RULE_HD Iv operator*(Iv a, Iv b) {
  const double p0 = a.lo * b.lo, p1 = a.lo * b.hi, p2 = a.hi * b.lo, p3 = a.hi * b.hi;
  return {fmin(fmin(p0, p1), fmin(p2, p3)), fmax(fmax(p0, p1), fmax(p2, p3))};
}
RULE_HD Iv operator*(double s, Iv a) { return s >= 0.0 ? Iv{s * a.lo, s * a.hi} : Iv{s * a.hi, s * a.lo}; }
RULE_HD Iv operator-(Iv a, double s) { return {a.lo - s, a.hi - s}; }
RULE_HD Iv widen(Iv a) {
  const double e = 1e-13 * (1.0 + fmax(fabs(a.lo), fabs(a.hi)));
  return {a.lo - e, a.hi + e};
}
RULE_HD bool no_zero(Iv a) { return a.lo > 0.0 || a.hi < 0.0; }

// range of cos over [u0, u1]: the end values, widened to 1 where a multiple
// of 2 pi lies inside and to -1 where an odd multiple of pi does
RULE_HD Iv cos_range(double u0, double u1) {
  if (u1 - u0 >= kTwoPi) return {-1.0, 1.0};
  const double c0 = cos(u0), c1 = cos(u1);
  Iv r{fmin(c0, c1), fmax(c0, c1)};
  if (kTwoPi * ceil(u0 / kTwoPi) <= u1) r.hi = 1.0;
  if (kTwoPi * ceil((u0 - kPi) / kTwoPi) + kPi <= u1) r.lo = -1.0;
  return r;
}
// cos(2 pi n x) and sin(2 pi n x) over the interval x
RULE_HD Iv cosn(int n, Iv x) { return cos_range(kTwoPi * n * x.lo, kTwoPi * n * x.hi); }
RULE_HD Iv sinn(int n, Iv x) { return cos_range(kTwoPi * n * x.lo - 0.5 * kPi, kTwoPi * n * x.hi - 0.5 * kPi); }

// A trimmed cell: family id (2 Schwarz Diamond, 3 Schwarz Primitive, 4 Schoen
// FRD, 5 Schoen IWP) and the corner thresholds (bottom-left, bottom-right,
// top-left, top-right).
struct Cell {
  int fam;
  double mu[4];
};

RULE_HD double bilin(const Cell& c, double x, double y) {
  return c.mu[0] * (1.0 - x) * (1.0 - y) + c.mu[1] * x * (1.0 - y) + c.mu[2] * (1.0 - x) * y + c.mu[3] * x * y;
}

// phi = phi_0 - mu and its gradient at a point
RULE_HD void phi_grad(const Cell& c, double x, double y, double& f, double& gx, double& gy) {
  const double c1x = cos(kTwoPi * x), c1y = cos(kTwoPi * y), s1x = sin(kTwoPi * x), s1y = sin(kTwoPi * y);
  double v, dx, dy;
  if (c.fam == 2) {
    v = c1x * c1y;
    dx = -kTwoPi * s1x * c1y;
    dy = -kTwoPi * c1x * s1y;
  } else if (c.fam == 3) {
    v = c1x + c1y - 1.0;
    dx = -kTwoPi * s1x;
    dy = -kTwoPi * s1y;
  } else {
    const double c2x = cos(2.0 * kTwoPi * x), c2y = cos(2.0 * kTwoPi * y);
    const double s2x = sin(2.0 * kTwoPi * x), s2y = sin(2.0 * kTwoPi * y);
    if (c.fam == 4) {
      v = c2x * c2y + c2y + c2x - 4.0 * c1x * c1y;
      dx = -2.0 * kTwoPi * s2x * (c2y + 1.0) + 4.0 * kTwoPi * s1x * c1y;
      dy = -2.0 * kTwoPi * s2y * (c2x + 1.0) + 4.0 * kTwoPi * c1x * s1y;
    } else {
      v = 2.0 * (c1x * c1y + c1y + c1x) - c2x - c2y - 1.0;
      dx = -2.0 * kTwoPi * s1x * (c1y + 1.0) + 2.0 * kTwoPi * s2x;
      dy = -2.0 * kTwoPi * s1y * (c1x + 1.0) + 2.0 * kTwoPi * s2y;
    }
  }
  f = v - bilin(c, x, y);
  gx = dx - ((c.mu[1] - c.mu[0]) * (1.0 - y) + (c.mu[3] - c.mu[2]) * y);
  gy = dy - ((c.mu[2] - c.mu[0]) * (1.0 - x) + (c.mu[3] - c.mu[1]) * x);
}

RULE_HD double phi(const Cell& c, double x, double y) {
  double f, gx, gy;
  phi_grad(c, x, y, f, gx, gy);
  return f;
}

// bounds of phi and of its partial derivatives over [x0,x1] x [y0,y1]
RULE_HD void bounds(const Cell& c, double x0, double x1, double y0, double y1, Iv& B, Iv& Gx, Iv& Gy) {
  const Iv X{x0, x1}, Y{y0, y1};
  const Iv c1x = cosn(1, X), c1y = cosn(1, Y), s1x = sinn(1, X), s1y = sinn(1, Y);
  Iv v, dx, dy;
  if (c.fam == 2) {
    v = c1x * c1y;
    dx = -kTwoPi * (s1x * c1y);
    dy = -kTwoPi * (c1x * s1y);
  } else if (c.fam == 3) {
    v = c1x + c1y - 1.0;
    dx = -kTwoPi * s1x;
    dy = -kTwoPi * s1y;
  } else {
    const Iv c2x = cosn(2, X), c2y = cosn(2, Y), s2x = sinn(2, X), s2y = sinn(2, Y);
    if (c.fam == 4) {
      v = c2x * c2y + c2y + c2x - 4.0 * (c1x * c1y);
      dx = (-2.0 * kTwoPi) * (s2x * (c2y + ivc(1.0))) + (4.0 * kTwoPi) * (s1x * c1y);
      dy = (-2.0 * kTwoPi) * (s2y * (c2x + ivc(1.0))) + (4.0 * kTwoPi) * (c1x * s1y);
    } else {
      v = 2.0 * (c1x * c1y + c1y + c1x) - c2x - c2y - 1.0;
      dx = (-2.0 * kTwoPi) * (s1x * (c1y + ivc(1.0))) + (2.0 * kTwoPi) * s2x;
      dy = (-2.0 * kTwoPi) * (s1y * (c1x + ivc(1.0))) + (2.0 * kTwoPi) * s2y;
    }
  }
  // the bilinear threshold: range at the corners, its x-derivative linear in
  // y (range at y0, y1), its y-derivative linear in x
  const double m00 = bilin(c, x0, y0), m10 = bilin(c, x1, y0), m01 = bilin(c, x0, y1), m11 = bilin(c, x1, y1);
  const Iv M{fmin(fmin(m00, m10), fmin(m01, m11)), fmax(fmax(m00, m10), fmax(m01, m11))};
  const double gx0 = (c.mu[1] - c.mu[0]) * (1.0 - y0) + (c.mu[3] - c.mu[2]) * y0;
  const double gx1 = (c.mu[1] - c.mu[0]) * (1.0 - y1) + (c.mu[3] - c.mu[2]) * y1;
  const double gy0 = (c.mu[2] - c.mu[0]) * (1.0 - x0) + (c.mu[3] - c.mu[1]) * x0;
  const double gy1 = (c.mu[2] - c.mu[0]) * (1.0 - x1) + (c.mu[3] - c.mu[1]) * x1;
  B = widen(v - M);
  Gx = widen(dx - Iv{fmin(gx0, gx1), fmax(gx0, gx1)});
  Gy = widen(dy - Iv{fmin(gy0, gy1), fmax(gy0, gy1)});
}

// Rule settings: n Gauss points per segment and per piece, the [0, 1] Gauss
// rule, the depth limit of the box recursion.
struct Cfg {
  int n;
  const double* gx;  // [n] nodes on [0, 1]
  const double* gw;  // [n] weights
  int max_depth;
};

// A sink receives the points in their order of generation (emit) and keeps an
// error code: 0, 1 capacity exceeded, 2 a root iteration did not converge, 3
// a work stack overflowed.  Out stores them.
struct Out {
  double* x;
  double* y;
  double* w;
  int cap;
  int n;
  int err;
  RULE_HD void emit(double px, double py, double pw) {
    if (n >= cap) {
      err = 1;
      return;
    }
    x[n] = px;
    y[n] = py;
    w[n] = pw;
    ++n;
  }
};

template <class Sink>
RULE_HD void tensor(const Cfg& g, Sink& o, const Cell* masked, double x0, double x1, double y0, double y1) {
  for (int b = 0; b < g.n; ++b)
    for (int a = 0; a < g.n; ++a) {
      const double x = x0 + (x1 - x0) * g.gx[a], y = y0 + (y1 - y0) * g.gx[b];
      if (masked && !(phi(*masked, x, y) < 0.0)) continue;
      o.emit(x, y, (x1 - x0) * (y1 - y0) * g.gw[a] * g.gw[b]);
    }
}

// phi along the height direction k at base coordinate s and height h
RULE_HD void along(const Cell& c, int k, double s, double h, double& f, double& df) {
  double v, gx, gy;
  if (k == 1) {
    phi_grad(c, s, h, v, gx, gy);
    df = gy;
  } else {
    phi_grad(c, h, s, v, gx, gy);
    df = gx;
  }
  f = v;
}

// phi on the face xi_k = face as a function of the base coordinate s
RULE_HD void on_face(const Cell& c, int k, double face, double s, double& f, double& df) {
  double v, gx, gy;
  if (k == 1) {
    phi_grad(c, s, face, v, gx, gy);
    df = gx;
  } else {
    phi_grad(c, face, s, v, gx, gy);
    df = gy;
  }
  f = v;
}

// Newton steps inside the sign-change bracket [a, b] of a function with one
// sign change, negative at a when neg_a; a step leaving the bracket becomes
// the bracket's midpoint.  mode 0: along xi_k at base s; mode 1: on a face.
template <class Sink>
RULE_HD double bracket_root(const Cell& c, int mode, int k, double fix, double a, double b, bool neg_a, Sink& o) {
  double lo = a, hi = b, x = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double f, df;
    if (mode == 0) along(c, k, fix, x, f, df);
    else on_face(c, k, fix, x, f, df);
    if (f == 0.0) return x;
    if ((f < 0.0) == neg_a) lo = x;
    else hi = x;
    double xn = x - f / df;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const double tol = 4e-16 * (1.0 + fabs(x));
    if (fabs(xn - x) <= tol || hi - lo <= tol) return xn;
    x = xn;
  }
  o.err = 2;
  return x;
}

// roots in [a, b] of phi on the face xi_k = face (appended to br[nb..]).
// Depth-first over the bisection tree of [a, b], left half first, without a
// stack: the node at depth d and index i is reached by halving from [a, b]
// along the bits of i, and after a resolved node the walk climbs while it is
// a right half and then steps to the right sibling.  A sign-change bracket
// takes its slot in br when found; its Newton solve is deferred and the
// pending ones run together (up to kPend at a time), so that the lanes of a
// wave, each on its own face, run their solves side by side rather than one
// walk step after another.
template <class Sink>
RULE_HD void face_roots(const Cell& c, int k, double face, double a, double b, double* br, int& nb, int brcap, Sink& o) {
  constexpr int kMaxDepth = 48;
  constexpr int kPend = 8;
  double pa[kPend], pb[kPend];
  int pslot[kPend];
  unsigned pneg = 0;
  int np = 0;
  auto flush = [&]() {
    for (int j = 0; j < np; ++j) br[pslot[j]] = bracket_root(c, 1, k, face, pa[j], pb[j], (pneg >> j) & 1, o);
    np = 0;
    pneg = 0;
  };
  long long i = 0;
  int d = 0;
  for (;;) {
    double u0 = a, u1 = b;
    for (int l = d - 1; l >= 0; --l) {
      const double m = 0.5 * (u0 + u1);
      if ((i >> l) & 1) u0 = m;
      else u1 = m;
    }
    bool split = false;
    Iv B, Gx, Gy;
    if (k == 1) bounds(c, u0, u1, face, face, B, Gx, Gy);
    else bounds(c, face, face, u0, u1, B, Gx, Gy);
    if (no_zero(B)) {
    } else if (fmax(fabs(B.lo), fabs(B.hi)) < 1e-11) {
      // phi vanishes on this part of the face
    } else if (no_zero(k == 1 ? Gx : Gy)) {
      double f0, f1, d0;
      on_face(c, k, face, u0, f0, d0);
      on_face(c, k, face, u1, f1, d0);
      if ((f0 < 0.0) != (f1 < 0.0)) {
        if (nb >= brcap) { flush(); o.err = 3; return; }
        if (np == kPend) flush();
        pa[np] = u0;
        pb[np] = u1;
        if (f0 < 0.0) pneg |= 1u << np;
        pslot[np++] = nb++;
      }
    } else if (d >= kMaxDepth) {
      if (nb >= brcap) { flush(); o.err = 3; return; }
      br[nb++] = 0.5 * (u0 + u1);
    } else {
      split = true;
    }
    if (split) {
      ++d;
      i <<= 1;
      continue;
    }
    while (d > 0 && (i & 1)) {
      i >>= 1;
      --d;
    }
    if (d == 0) {
      flush();
      return;
    }
    ++i;
  }
}

constexpr int kMaxN = 24;

// The inside segments of the n base points of the piece [s0, s1] of a height
// box, and six moments of their ends.
struct Seg {
  double s[kMaxN], ws[kMaxN], lo[kMaxN], hi[kMaxN];
  bool keep[kMaxN];
  double mom[6];
};

template <class Sink>
RULE_HD void segments(const Cell& c, const Cfg& g, int k, double ka, double kb, double s0, double s1, Seg& S, Sink& o) {
  for (int e = 0; e < 6; ++e) S.mom[e] = 0.0;
  for (int i = 0; i < g.n; ++i) {
    const double s = s0 + (s1 - s0) * g.gx[i], ws = (s1 - s0) * g.gw[i];
    double fa, fb, d;
    along(c, k, s, ka, fa, d);
    along(c, k, s, kb, fb, d);
    const bool na = fa < 0.0, nb = fb < 0.0;
    double lo = ka, hi = kb;
    if (na != nb) {
      const double r = bracket_root(c, 0, k, s, ka, kb, na, o);
      if (na) hi = r;
      else lo = r;
    }
    S.s[i] = s;
    S.ws[i] = ws;
    S.lo[i] = lo;
    S.hi[i] = hi;
    S.keep[i] = na || nb;
    if (S.keep[i]) {
      double he = hi, le = lo;
      for (int e = 0; e < 3; ++e) {
        S.mom[2 * e] += ws * (he - le);
        S.mom[2 * e + 1] += ws * (he - le) * s;
        he *= hi;
        le *= lo;
      }
    }
  }
}

template <class Sink>
RULE_HD void emit_segments(const Cfg& g, int k, const Seg& S, Sink& o) {
  for (int i = 0; i < g.n; ++i) {
    if (!S.keep[i]) continue;
    const double len = S.hi[i] - S.lo[i];
    for (int t = 0; t < g.n; ++t) {
      const double h = S.lo[i] + len * g.gx[t], w = S.ws[i] * len * g.gw[t];
      if (k == 1) o.emit(S.s[i], h, w);
      else o.emit(h, S.s[i], w);
    }
  }
}

template <class Sink>
RULE_HD void height(const Cell& c, const Cfg& g, int k, double x0, double x1, double y0, double y1, Sink& o) {
  const double ja = k == 1 ? x0 : y0, jb = k == 1 ? x1 : y1;
  const double ka = k == 1 ? y0 : x0, kb = k == 1 ? y1 : x1;
  double br[64];
  int nb = 0;
  br[nb++] = ja;
  br[nb++] = jb;
  face_roots(c, k, ka, ja, jb, br, nb, 64, o);
  face_roots(c, k, kb, ja, jb, br, nb, 64, o);
  if (o.err) return;
  // sort, drop duplicates and points outside [ja, jb]
  for (int i = 1; i < nb; ++i) {
    const double v = br[i];
    int j = i - 1;
    while (j >= 0 && br[j] > v) {
      br[j + 1] = br[j];
      --j;
    }
    br[j + 1] = v;
  }
  Seg W, L, R;
  double st[64][2];
  int sd[64];
  for (int p = 0; p + 1 < nb; ++p) {
    const double s0 = br[p], s1 = br[p + 1];
    if (!(s1 > s0) || s0 < ja || s1 > jb) continue;
    int top = 0;
    st[0][0] = s0;
    st[0][1] = s1;
    sd[0] = 0;
    top = 1;
    while (top > 0) {
      --top;
      const double a = st[top][0], b = st[top][1];
      const int d = sd[top];
      const double m = 0.5 * (a + b);
      segments(c, g, k, ka, kb, a, b, W, o);
      segments(c, g, k, ka, kb, a, m, L, o);
      segments(c, g, k, ka, kb, m, b, R, o);
      double diff = 0.0;
      for (int e = 0; e < 6; ++e) diff = fmax(diff, fabs(L.mom[e] + R.mom[e] - W.mom[e]));
      if (d >= 40 || diff <= 1e-15) {
        emit_segments(g, k, L, o);
        emit_segments(g, k, R, o);
        continue;
      }
      if (top + 2 > 64) { o.err = 3; return; }
      st[top][0] = m; st[top][1] = b; sd[top] = d + 1; ++top;  // right after left
      st[top][0] = a; st[top][1] = m; sd[top] = d + 1; ++top;
    }
  }
}

// The rule over {phi < 0} in the unit cell.
template <class Sink>
RULE_HD void cell_rule(const Cell& c, const Cfg& g, Sink& o) {
  double st[128][4];
  int sd[128];
  int top = 0;
  st[0][0] = 0.0; st[0][1] = 1.0; st[0][2] = 0.0; st[0][3] = 1.0;
  sd[0] = 0;
  top = 1;
  o.err = 0;
  while (top > 0 && !o.err) {
    --top;
    const double x0 = st[top][0], x1 = st[top][1], y0 = st[top][2], y1 = st[top][3];
    const int d = sd[top];
    Iv B, Gx, Gy;
    bounds(c, x0, x1, y0, y1, B, Gx, Gy);
    if (B.hi < 0.0) {
      tensor(g, o, nullptr, x0, x1, y0, y1);
      continue;
    }
    if (B.lo > 0.0) continue;
    const bool okx = no_zero(Gx), oky = no_zero(Gy);
    if (okx || oky) {
      const double mx = okx ? fmin(fabs(Gx.lo), fabs(Gx.hi)) : -1.0;
      const double my = oky ? fmin(fabs(Gy.lo), fabs(Gy.hi)) : -1.0;
      height(c, g, my >= mx ? 1 : 0, x0, x1, y0, y1, o);
      continue;
    }
    if (d >= g.max_depth) {
      tensor(g, o, &c, x0, x1, y0, y1);
      continue;
    }
    if (top + 4 > 128) { o.err = 3; return; }
    const double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1);
    const double ch[4][4] = {{xm, x1, ym, y1}, {x0, xm, ym, y1}, {xm, x1, y0, ym}, {x0, xm, y0, ym}};
    for (int q = 0; q < 4; ++q) {
      for (int e = 0; e < 4; ++e) st[top][e] = ch[q][e];
      sd[top] = d + 1;
      ++top;
    }
  }
}

#undef RULE_HD

}  // namespace rule
}  // namespace lbddc
