"""Pins of the ROM with four parameters per cell (the corner thresholds of
the Table 1 level sets, Sec. 2.1.2, 4.2):

  - FindCluster over the n_k^4 clusters of the box: per-coordinate interval
    indices, first coordinate fastest, the box's upper face in the last
    cluster, a point outside the box rejected;
  - Latin-hypercube sampling: in every coordinate each stratum of the
    cluster holds exactly one sample;
  - snapshots that are polynomials of degree <= r in each coordinate, in a
    fixed span of fewer than n_r vectors, are reproduced exactly by the
    surrogate (SVD span, DEIM interpolation and the tensor Lagrange fit are
    exact for them), and so are their derivatives in each coordinate; the
    polynomials are not symmetric, so a coordinate taken in the wrong order
    or a transposed fitting grid fails;
  - on a real Schwarz Diamond cell, the projection error of fresh snapshots
    falls as n_r grows (the indicator of Sec. 5.1.2).
"""
import numpy as np
import pytest

from oracle import rom as R
from oracle.implicit import FAMILY_SCHWARZ_D
from workloads import rom_lhs_draws


def test_find_cluster_4d():
    lo, hi = 0.1, 0.9
    f = lambda x: R.find_cluster_nd(np.array(x), lo, hi, 2)
    assert f([0.1, 0.1, 0.1, 0.1]) == 0
    assert f([0.9, 0.1, 0.1, 0.1]) == 1
    assert f([0.1, 0.9, 0.1, 0.1]) == 2
    assert f([0.1, 0.1, 0.9, 0.1]) == 4
    assert f([0.1, 0.1, 0.1, 0.9]) == 8
    assert f([0.5, 0.5, 0.5, 0.5]) == 15
    assert f([0.4999, 0.5001, 0.2, 0.7]) == 2 + 8
    with pytest.raises(ValueError):
        f([0.1, 0.95, 0.1, 0.1])
    assert R.cluster_box(2 + 8, lo, hi, 2, 4) == [(0.1, 0.5), (0.5, 0.9), (0.1, 0.5), (0.5, 0.9)]


def test_lhs_strata_4d():
    n_s = 9
    u, perm = rom_lhs_draws(FAMILY_SCHWARZ_D, 2, n_s, 4)
    for k in range(16):
        box = R.cluster_box(k, 0.1, 0.9, 2, 4)
        for i, (a, b) in enumerate(box):
            x = R.lhs_samples(a, b, u[k][:, i], perm[k][i])
            strata = np.floor((x - a) / (b - a) * n_s).astype(int)
            assert sorted(strata) == list(range(n_s))


def _poly_exact(V):
    """Snapshots sum_j c_j(x) V[:, j] with c_j polynomials of degree <= 3 in
    each coordinate, and their gradients."""
    def coef(x):
        x1, x2, x3, x4 = x
        return np.array([1.0, x1 * x1 * x2, x3 * x4 + x1, x2 ** 3 - 2 * x4, x1 * x3 ** 2 * x4 ** 3])

    def dcoef(x):
        x1, x2, x3, x4 = x
        return np.array([[0, 2 * x1 * x2, 1, 0, x3 ** 2 * x4 ** 3],
                         [0, x1 * x1, 0, 3 * x2 ** 2, 0],
                         [0, 0, x4, 0, 2 * x1 * x3 * x4 ** 3],
                         [0, 0, x3, -2, 3 * x1 * x3 ** 2 * x4 ** 2]])

    exact = lambda family, p, q, x: V @ coef(np.asarray(x, dtype=float))
    return exact, lambda x: V @ dcoef(x).T


def test_polynomial_snapshots_reproduced():
    rng = np.random.default_rng(11)
    V = rng.normal(size=(60, 5))
    exact, grad = _poly_exact(V)
    u, perm = rom_lhs_draws(FAMILY_SCHWARZ_D, 2, 12, 4)
    rom = R.train(FAMILY_SCHWARZ_D, 2, 1, 0.1, 0.9, 2, 12, 8, 3, u, exact=exact, dim=4, lhs_perm=perm)
    assert all(c["n_used"] == 5 for c in rom["clusters"])
    for x in 0.1 + 0.8 * rng.random((40, 4)):
        k, Ir = R.reduced_coordinates(rom, x)
        U = rom["clusters"][k]["U"]
        ref = exact(None, 0, 0, x)
        assert np.abs(U @ Ir - ref).max() <= 1e-11 * np.abs(ref).max()
        _, dIr = R.reduced_coordinates_dt(rom, x)
        dref = grad(x)
        assert np.abs(U @ dIr.T - dref).max() <= 1e-10 * (1 + np.abs(dref).max())


@pytest.mark.slow
def test_schwarz_d_projection_error_falls_with_rank():
    p, q = 3, 2
    u, perm = rom_lhs_draws(FAMILY_SCHWARZ_D, 1, 24, 4)
    rom = R.train(FAMILY_SCHWARZ_D, p, q, 0.3, 0.7, 1, 24, 20, 1, u, dim=4, lhs_perm=perm)
    U = rom["clusters"][0]["U"]
    from oracle.trimmed import I_exact
    rng = np.random.default_rng(5)
    errs = {4: [], 12: []}
    for x in 0.3 + 0.4 * rng.random((6, 4)):
        I = I_exact(FAMILY_SCHWARZ_D, p, q, x).ravel()
        for n in errs:
            errs[n].append(np.abs(I - U[:, :n] @ (U[:, :n].T @ I)).max() / np.abs(I).max())
    assert np.mean(errs[12]) < 0.2 * np.mean(errs[4])
    assert np.mean(errs[12]) < 1e-2
