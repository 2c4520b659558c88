"""Pins of the exact trimmed tensors: two independent quadratures per family,
closed-form moments of the material region, limits and invariants."""
import numpy as np
import pytest
from oracle import trimmed as tr
from oracle.basis import gll_nodes, interp_nodes


@pytest.mark.parametrize("p", [3, 6, 8])
@pytest.mark.parametrize("t", [0.08, 0.2, 0.37])
def test_circle_two_methods(p, t):
    a = tr.I_circle(p, 2, t, method="polar")
    b = tr.I_circle(p, 2, t, method="slices")
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("p", [3, 8])
@pytest.mark.parametrize("t", [0.1, 0.25])
def test_cross_two_methods(p, t):
    a = tr.I_cross(p, 2, t, method="union")
    b = tr.I_cross(p, 2, t, method="pieces")
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def _moments(I, p, q):
    """Use linear precision of the GLL and interpolation bases:
    sum_{k1 k2} x_a(k1) x_b(k2) I[k1,k2,j,l,k3] = delta_aj delta_bl int L_k3,
    and sum_k3 phi(node k3) L_k3 = phi for phi in {1, xi1, xi2} (q >= 1).
    Returns {(a, b, j, l): (int 1, int xi1, int xi2)} over the material."""
    g = gll_nodes(p)
    n = p + 1
    x1 = np.array([g[k % n] for k in range(n * n)])
    x2 = np.array([g[k // n] for k in range(n * n)])
    xs = [x1, x2]
    pts = interp_nodes(q)
    out = {}
    for a in range(2):
        for b in range(2):
            for j in range(2):
                for l in range(2):
                    v = np.einsum("x,y,xyk->k", xs[a], xs[b], I[:, :, j, l, :])
                    out[(a, b, j, l)] = (v.sum(), v @ pts[:, 0], v @ pts[:, 1])
    return out


@pytest.mark.parametrize("t", [0.1, 0.3])
def test_circle_closed_form_moments(t):
    p, q = 6, 2
    r = 0.5 - t
    mom = _moments(tr.I_circle(p, q, t), p, q)
    area = 1 - np.pi * r * r
    for (a, b, j, l), (m0, m1, m2) in mom.items():
        if a == j and b == l:
            assert abs(m0 - area) < 1e-13
            assert abs(m1 - 0.5 * area) < 1e-13   # symmetric about the centre
            assert abs(m2 - 0.5 * area) < 1e-13
        else:
            assert abs(m0) < 1e-13 and abs(m1) < 1e-13


@pytest.mark.parametrize("t", [0.1, 0.3])
def test_cross_closed_form_moments(t):
    p, q = 5, 2
    mom = _moments(tr.I_cross(p, q, t), p, q)
    area = 2 * t - t * t
    m0, m1, _ = mom[(0, 1, 0, 1)]
    assert abs(m0 - area) < 1e-13 and abs(m1 - 0.5 * area) < 1e-13


def test_translation_invariance_and_limits():
    p, q = 4, 2
    for I in (tr.I_circle(p, q, 0.2), tr.I_cross(p, q, 0.2), tr.I_square(p, q)):
        assert np.abs(I.sum(axis=0)).max() < 1e-13
        assert np.abs(I.sum(axis=1)).max() < 1e-13
        assert np.abs(I - np.transpose(I, (1, 0, 3, 2, 4))).max() < 1e-14
    Ipi = tr.I_square(p, q)
    # hole shrinking to nothing, cross filling the cell
    assert np.abs(tr.I_circle(p, q, 0.5 - 1e-9) - Ipi).max() < 1e-12
    assert np.abs(tr.I_cross(p, q, 1 - 1e-12) - Ipi).max() < 1e-10


def test_square_kronecker_closed_form():
    """I_pi summed over k3 equals Kronecker products of 1-D GLL matrices."""
    from oracle.basis import lagrange, lagrange_deriv, gauss_legendre
    p, q = 4, 2
    x, w = gauss_legendre(p + 2)
    g = gll_nodes(p)
    L, D = lagrange(g, x), lagrange_deriv(g, x)
    M = (L * w) @ L.T
    A = (D * w) @ D.T
    X = (D * w) @ L.T   # X[a1, a2] = int b'_a1 b_a2
    S = tr.I_square(p, q).sum(axis=4)
    n = p + 1
    ref = np.zeros_like(S)
    ref[:, :, 0, 0] = np.kron(M, A)
    ref[:, :, 1, 1] = np.kron(A, M)
    ref[:, :, 0, 1] = np.kron(X.T, X)
    ref[:, :, 1, 0] = np.kron(X, X.T)
    assert np.abs(S - ref).max() < 1e-13
