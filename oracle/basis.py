"""Polynomial bases on [0, 1].

GLL Lagrange basis of the cell element (Sec. 2.2.2, the bivariate basis
B_ij = b_i(xi_1) b_j(xi_2)), the degree-q interpolation basis of the fast
assembly (Sec. 4.1, interpolation of the pulled-back tensor at GLL points),
and Bernstein polynomials for the cell maps (Sec. 2.1.3: a spline surface is
used after Bezier extraction).
"""
import numpy as np
from math import comb


def gll_nodes(p):
    """Gauss-Lobatto-Legendre nodes on [0, 1], p+1 of them: the end points
    and the roots of P_p' (Sec. 2.2.2).  Roots by numpy's Legendre companion
    matrix, polished by Newton steps on P_p'."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    leg = np.polynomial.legendre
    c = np.zeros(p + 1)
    c[p] = 1.0
    d1 = leg.legder(c)
    d2 = leg.legder(d1)
    x = np.sort(np.real(leg.legroots(d1)))
    for _ in range(4):
        x = x - leg.legval(x, d1) / leg.legval(x, d2)
    x = np.concatenate([[-1.0], x, [1.0]])
    return 0.5 * (x + 1.0)


def gll_weights(p):
    """GLL quadrature weights on [0, 1]: w_i = 1 / (p (p+1) P_p(x_i)^2),
    the classical formula on [-1, 1] halved."""
    x = 2.0 * gll_nodes(p) - 1.0
    c = np.zeros(p + 1)
    c[p] = 1.0
    P = np.polynomial.legendre.legval(x, c)
    return 1.0 / (p * (p + 1) * P * P)


def gauss_legendre(n, a=0.0, b=1.0):
    """n-point Gauss-Legendre rule on [a, b] (exact to degree 2n-1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return a + (b - a) * 0.5 * (x + 1.0), (b - a) * 0.5 * w


def lagrange(nodes, x):
    """Values L[a, k] = l_a(x_k) of the Lagrange polynomials on `nodes`,
    by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((n, len(x)))
    for a in range(n):
        for m in range(n):
            if m != a:
                L[a] *= (x - nodes[m]) / (nodes[a] - nodes[m])
    return L


def lagrange_deriv(nodes, x):
    """Derivatives dL[a, k] = l_a'(x_k): the product rule applied to the
    product formula, sum over the dropped factor l."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    dL = np.zeros((n, len(x)))
    for a in range(n):
        for l in range(n):
            if l == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[l]))
            for m in range(n):
                if m != a and m != l:
                    term = term * (x - nodes[m]) / (nodes[a] - nodes[m])
            dL[a] += term
    return dL


def bernstein(m, x):
    """Bernstein polynomials of degree m: B[a, k] = C(m,a) x^a (1-x)^(m-a)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([comb(m, a) * x**a * (1.0 - x) ** (m - a) for a in range(m + 1)])


def bernstein_deriv(m, x):
    """Derivatives: B'_a = m (B^{m-1}_{a-1} - B^{m-1}_a)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if m == 0:
        return np.zeros((1, len(x)))
    Bm1 = bernstein(m - 1, x)
    d = np.zeros((m + 1, len(x)))
    for a in range(m + 1):
        if a - 1 >= 0:
            d[a] += m * Bm1[a - 1]
        if a <= m - 1:
            d[a] -= m * Bm1[a]
    return d


def tensor_basis(p, x1, x2):
    """Bivariate GLL basis at points (x1[k], x2[k]) (Sec. 2.2.2):
    B[kk, k] with kk = a + (p+1) b, and its gradient dB[kk, j, k] = dB/dxi_j."""
    nodes = gll_nodes(p)
    L1, L2 = lagrange(nodes, x1), lagrange(nodes, x2)
    D1, D2 = lagrange_deriv(nodes, x1), lagrange_deriv(nodes, x2)
    n = p + 1
    B = np.zeros((n * n, len(x1)))
    dB = np.zeros((n * n, 2, len(x1)))
    for b in range(n):
        for a in range(n):
            kk = a + n * b
            B[kk] = L1[a] * L2[b]
            dB[kk, 0] = D1[a] * L2[b]
            dB[kk, 1] = L1[a] * D2[b]
    return B, dB


def interp_basis(q, x1, x2):
    """Degree-q tensor Lagrange basis on (q+1)^2 GLL points (Sec. 4.1):
    Lq[k3, k], k3 = a + (q+1) b."""
    nodes = gll_nodes(q)
    L1, L2 = lagrange(nodes, x1), lagrange(nodes, x2)
    n = q + 1
    out = np.zeros((n * n, len(x1)))
    for b in range(n):
        for a in range(n):
            out[a + n * b] = L1[a] * L2[b]
    return out


def interp_nodes(q):
    """The (q+1)^2 interpolation points, ordered k3 = a + (q+1) b."""
    g = gll_nodes(q)
    n = q + 1
    pts = np.zeros((n * n, 2))
    for b in range(n):
        for a in range(n):
            pts[a + n * b] = (g[a], g[b])
    return pts
