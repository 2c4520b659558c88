"""The oracle's method on a lattice of the paper's own cells: a Schwarz
Diamond lattice with the bilinear threshold through shared vertex values
(d = 4, Sec. 2.1.2), the recipe of the graded workload at a small size.

  - the vertex values are shared: each cell's corners agree with its
    neighbours' (trimmed compatibility, Sec. 2.1.3);
  - PCG with the BDDC preconditioner (Alg. 1) reaches the direct solve of
    the same ROM-assembled system;
  - dJ/dX, dJ/dmu of the discrete adjoint against central differences of the
    compliance along random directions (mu perturbed cell by cell).
"""
import numpy as np
import pytest

from conftest import oracle_roms
from oracle.adjoint import compliance_gradient, fd_directional
from oracle.bddc import Problem
from workloads import make_problem

# the box is wider than the lattice's values, so finite differences stay inside it
ROM = {2: dict(lo=0.05, hi=0.95, n_k=1, n_s=10, n_r=10, r=1, dim=4)}


def small_tpms(**over):
    kw = dict(nx=3, ny=2, p=3, rom=ROM)
    kw.update(over)
    return make_problem(6, **kw)


def test_thresholds_shared_across_edges():
    prob = make_problem(6, nx=5, ny=4, p=3, rom=ROM)
    nx, ny, mu = prob["nx"], prob["ny"], prob["mu"]
    for c in range(nx * ny):
        iy, ix = divmod(c, nx)
        if ix + 1 < nx:
            e = c + 1
            assert mu[c, 1] == mu[e, 0] and mu[c, 3] == mu[e, 2]
        if iy + 1 < ny:
            e = c + nx
            assert mu[c, 2] == mu[e, 0] and mu[c, 3] == mu[e, 1]
    assert mu.min() >= 0.1 and mu.max() <= 0.9


@pytest.mark.slow
def test_pcg_matches_direct_and_gradient_matches_fd():
    prob = small_tpms()
    roms = oracle_roms(prob)
    P = Problem(prob, roms)
    u_dir = P.direct_solve()
    P.setup()
    u_pcg, its, _ = P.solve(rtol=1e-12)
    assert np.abs(u_pcg - u_dir).max() <= 1e-9 * np.abs(u_dir).max()
    J, gX, gt, gmu = compliance_gradient(P, u_dir, thresholds=True)
    assert np.all(gt == 0.0)
    rng = np.random.default_rng(77)
    for _ in range(3):
        dX = rng.normal(size=prob["ctrl"].shape)
        dmu = rng.normal(size=prob["mu"].shape)
        nrm = np.sqrt((dX ** 2).sum() + (dmu ** 2).sum())
        dX, dmu = dX / nrm, dmu / nrm
        fd = fd_directional(prob, roms, dX, np.zeros_like(prob["t"]), h=1e-6, dmu=dmu)
        ad = np.array([(gX[r] * dX).sum() + (gmu[r] * dmu).sum() for r in range(len(J))])
        assert np.all(np.abs(fd - ad) <= 1e-6 * np.abs(ad)), (fd, ad)


def _square(L, m=2):
    """Affine map of the unit square onto [0, L]^2 with degree-m control points."""
    X = np.zeros((m + 1, m + 1, 2))
    for b in range(m + 1):
        for a in range(m + 1):
            X[b, a] = (L * a / m, L * b / m)
    return X


def test_trimmed_edge_rows_fully_material_equal_untrimmed():
    """With phi_0 < mu everywhere on the cell (Schwarz Diamond, phi_0 <= 1 <
    mu) the material part of every edge is the whole edge."""
    from oracle.bddc import edge_constraint_rows
    from oracle.dofs import EDGES
    from oracle.implicit import TrimmedCell
    rng = np.random.default_rng(3)
    X = _square(1.3) + 0.05 * rng.normal(size=(3, 3, 2))
    dom = TrimmedCell(2, (1.2, 1.4, 1.1, 1.3))
    for e in EDGES:
        np.testing.assert_allclose(edge_constraint_rows(X, 6, e, True, dom),
                                   edge_constraint_rows(X, 6, e, True), rtol=0, atol=1e-14)


@pytest.mark.parametrize("mu", [0.0, 0.4, -0.7])
def test_trimmed_edge_rows_closed_form(mu):
    """Schwarz Primitive with a constant threshold on the square [0, L]^2: on
    the left edge phi_0 = cos(2 pi y), so the material part is (a, 1 - a) with
    a = arccos(mu) / (2 pi).  The GLL Lagrange basis reproduces 1 and s, so
    sum_n avg_n = L (1 - 2a), sum_n avg_n s_n = L ((1 - a)^2 - a^2) / 2, and
    on this vertical edge the moment acts on u1 with L (s - 1/2):
    sum_n mom_n s_n = L^2 int_a^{1-a} (s^2 - s/2) ds."""
    from oracle.basis import gll_nodes
    from oracle.bddc import edge_constraint_rows
    from oracle.implicit import TrimmedCell
    p, L = 6, 1.7
    a = np.arccos(mu) / (2 * np.pi)
    rows = edge_constraint_rows(_square(L), p, "left", True, TrimmedCell(3, (mu,) * 4))
    s = gll_nodes(p)
    np.testing.assert_allclose(rows[0, :, 0].sum(), L * (1 - 2 * a), rtol=1e-13)
    np.testing.assert_allclose(rows[1, :, 1], rows[0, :, 0], rtol=0, atol=0)
    np.testing.assert_allclose(rows[0, :, 0] @ s, L * ((1 - a) ** 2 - a ** 2) / 2, rtol=1e-13)
    F = lambda t: t ** 3 / 3 - t ** 2 / 4
    np.testing.assert_allclose(rows[2, :, 0] @ s, L * L * (F(1 - a) - F(a)), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(rows[2, :, 1], 0.0, atol=1e-15)
    assert np.all(rows[0, :, 1] == 0) and np.all(rows[1, :, 0] == 0)


@pytest.mark.parametrize("family", [2, 3, 4, 5])
def test_trimmed_edge_rows_brute_force(family):
    """Every edge of a curved cell with four distinct corner thresholds:
    material intervals from a dense sign scan refined by brentq, integrals by
    adaptive quadrature (scipy), independent of the oracle's interval-checked
    root search and its Gauss rule."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    from oracle.basis import bernstein, bernstein_deriv, gll_nodes, lagrange
    from oracle.bddc import edge_constraint_rows
    from oracle.dofs import EDGES
    from oracle.implicit import TrimmedCell
    rng = np.random.default_rng(10 + family)
    X = _square(2.0) + 0.1 * rng.normal(size=(3, 3, 2))
    mu = {2: (0.1, 0.5, -0.3, 0.7), 3: (0.2, -0.4, 0.5, 0.0),
          4: (0.3, 1.0, -0.5, 0.6), 5: (0.8, -0.2, 0.4, 1.3)}[family]
    dom = TrimmedCell(family, mu)
    p = 5
    nodes = gll_nodes(p)
    P = {"left": X[:, 0], "right": X[:, 2], "bottom": X[0, :], "top": X[2, :]}
    for e in EDGES:
        k, face = (0, float(e == "right")) if e in ("left", "right") else (1, float(e == "top"))
        g = (lambda s: dom.f(np.array([face]), np.array([s]))[0]) if k == 0 else \
            (lambda s: dom.f(np.array([s]), np.array([face]))[0])
        t = np.linspace(0.0, 1.0, 20001)
        v = np.array([g(x) for x in t])
        br = [0.0] + [brentq(g, t[i], t[i + 1], xtol=1e-15)
                      for i in range(len(t) - 1) if (v[i] < 0) != (v[i + 1] < 0)] + [1.0]
        pieces = [(lo, hi) for lo, hi in zip(br[:-1], br[1:]) if g(0.5 * (lo + hi)) < 0]
        xbar = bernstein(2, np.array([0.5]))[:, 0] @ P[e]

        def integrand(s, n, kind):
            x = bernstein(2, np.array([s]))[:, 0] @ P[e]
            dx = bernstein_deriv(2, np.array([s]))[:, 0] @ P[e]
            b = lagrange(nodes, np.array([s]))[n, 0] * np.hypot(*dx)
            return b if kind == 0 else b * ((x[1] - xbar[1]) if kind == 1 else (xbar[0] - x[0]))

        ref = np.zeros((3, p + 1))
        for n in range(p + 1):
            for kind in range(3):
                ref[kind, n] = sum(quad(integrand, lo, hi, args=(n, kind), epsabs=1e-14, epsrel=1e-13)[0]
                                   for lo, hi in pieces)
        rows = edge_constraint_rows(X, p, e, True, dom)
        assert pieces, (family, e)
        np.testing.assert_allclose(rows[0, :, 0], ref[0], rtol=0, atol=1e-11)
        np.testing.assert_allclose(rows[2, :, 0], ref[1], rtol=0, atol=1e-11)
        np.testing.assert_allclose(rows[2, :, 1], ref[2], rtol=0, atol=1e-11)


def test_trimmed_edge_rows_shared_by_neighbours():
    """Trimmed compatibility (Sec. 2.1.3): two cells sharing an edge, its
    control points and its two vertex thresholds see one material part, so
    the right-edge rows of the left cell equal the left-edge rows of the
    right cell, and likewise top and bottom."""
    from oracle.bddc import edge_constraint_rows
    from oracle.implicit import TrimmedCell
    rng = np.random.default_rng(7)
    A = _square(1.0) + 0.05 * rng.normal(size=(3, 3, 2))
    B = _square(1.0) + np.array([1.0, 0.0]) + 0.05 * rng.normal(size=(3, 3, 2))
    B[:, 0] = A[:, 2]
    C = _square(1.0) + np.array([0.0, 1.0]) + 0.05 * rng.normal(size=(3, 3, 2))
    C[0, :] = A[2, :]
    for fam in (2, 3, 4, 5):
        muA = rng.uniform(-0.5, 0.9, 4)
        muB = np.array([muA[1], rng.uniform(-0.5, 0.9), muA[3], rng.uniform(-0.5, 0.9)])
        muC = np.array([muA[2], muA[3], rng.uniform(-0.5, 0.9), rng.uniform(-0.5, 0.9)])
        ra = edge_constraint_rows(A, 4, "right", True, TrimmedCell(fam, muA))
        rb = edge_constraint_rows(B, 4, "left", True, TrimmedCell(fam, muB))
        np.testing.assert_allclose(ra, rb, rtol=0, atol=1e-14)
        ra = edge_constraint_rows(A, 4, "top", True, TrimmedCell(fam, muA))
        rc = edge_constraint_rows(C, 4, "bottom", True, TrimmedCell(fam, muC))
        np.testing.assert_allclose(ra, rc, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mu", [0.0, 0.4, -0.7])
def test_trimmed_traction_closed_form(mu):
    """The traction on the material part of the loaded edge: Schwarz
    Primitive at a constant threshold on [0, L]^2, right edge, material part
    (a, 1 - a) with a = arccos(mu) / (2 pi): the nodal loads sum to
    L (1 - 2a) t and their first moment is L ((1 - a)^2 - a^2) / 2 t; with
    phi_0 < mu everywhere they equal the whole-edge loads."""
    from oracle.basis import gll_nodes
    from oracle.bddc import traction_load
    from oracle.implicit import TrimmedCell
    p, L, t = 6, 1.7, np.array([0.3, -1.1])
    a = np.arccos(mu) / (2 * np.pi)
    f = traction_load(_square(L), p, t, "right", TrimmedCell(3, (mu,) * 4))
    s = gll_nodes(p)
    np.testing.assert_allclose(f.sum(axis=0), L * (1 - 2 * a) * t, rtol=1e-13)
    np.testing.assert_allclose(s @ f, L * ((1 - a) ** 2 - a ** 2) / 2 * t, rtol=1e-13)
    rng = np.random.default_rng(4)
    X = _square(1.2) + 0.05 * rng.normal(size=(3, 3, 2))
    np.testing.assert_allclose(traction_load(X, p, t, "right", TrimmedCell(2, (1.1, 1.3, 1.2, 1.05))),
                               traction_load(X, p, t, "right"), rtol=0, atol=1e-14)


def test_moving_end_term_of_the_load():
    """dJ/dmu of a lattice whose loaded edges are partly void against central
    differences along thresholds of the loaded cells only; without the
    Leibniz term of the moving ends the adjoint misses by far more than the
    tolerance."""
    import oracle.adjoint as A
    prob = small_tpms()
    roms = oracle_roms(prob)
    P = Problem(prob, roms)
    u = P.direct_solve()
    _, _, _, gmu = A.compliance_gradient(P, u, thresholds=True)
    loaded = np.array(sorted(P.load_pos))
    dmu = np.zeros_like(prob["mu"])
    dmu[loaded] = np.random.default_rng(8).normal(size=(len(loaded), 4))
    dmu /= np.linalg.norm(dmu)
    fd = A.fd_directional(prob, roms, np.zeros_like(prob["ctrl"]), np.zeros_like(prob["t"]), h=1e-6, dmu=dmu)[0]
    ad = (gmu[0] * dmu).sum()
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    orig = A._load_end_rate
    try:
        A._load_end_rate = lambda *a: np.zeros(4)
        _, _, _, g0 = A.compliance_gradient(P, u, thresholds=True)
    finally:
        A._load_end_rate = orig
    assert abs(fd - (g0[0] * dmu).sum()) > 1e-3 * abs(ad)
