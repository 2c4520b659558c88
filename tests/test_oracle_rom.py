"""Pins of the offline MDEIM training and the online surrogate."""
import numpy as np
import pytest
from oracle import rom as R
from oracle.trimmed import I_exact
from oracle.basis import gll_nodes
from workloads import rom_lhs_uniforms


@pytest.fixture(scope="module")
def rom3():
    return R.train(0, 3, 2, 0.1, 0.3, 2, 60, 20, 6, rom_lhs_uniforms(0, 2, 60))


def test_find_cluster_edges():
    assert R.find_cluster(0.1, 0.1, 0.3, 2) == 0
    assert R.find_cluster(0.2, 0.1, 0.3, 2) == 1
    assert R.find_cluster(0.3, 0.1, 0.3, 2) == 1
    assert R.find_cluster(0.19999, 0.1, 0.3, 2) == 0
    with pytest.raises(ValueError):
        R.find_cluster(0.3000001, 0.1, 0.3, 2)
    with pytest.raises(ValueError):
        R.find_cluster(0.05, 0.1, 0.3, 2)


def test_lhs_strata():
    u = np.random.default_rng(0).random(10)
    s = R.lhs_samples(0.2, 0.3, u)
    np.testing.assert_array_equal(np.floor((s - 0.2) / 0.01 + 1e-12).astype(int), np.arange(10))


def test_deim_on_permuted_identity():
    # columns are unit vectors: the greedy must pick their positions in order
    U = np.zeros((7, 3))
    U[4, 0], U[1, 1], U[6, 2] = 1.0, 1.0, 1.0
    np.testing.assert_array_equal(R.deim_points(U), [4, 1, 6])


def test_deim_brute_force():
    # the j-th point is the argmax of the interpolation residual: check by brute force
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.normal(size=(12, 4)))
    m = R.deim_points(U)
    for j in range(1, 4):
        P = m[:j]
        res = U[:, j] - U[:, :j] @ np.linalg.solve(U[P, :j], U[P, j])
        assert np.abs(res[m[j]]) >= np.abs(res).max() - 1e-15


def test_magic_point_reproduction(rom3):
    """U_r I_r(t_k) equals I(t_k) at the magic points at every fitting node."""
    for c in rom3["clusters"]:
        n = c["n_used"]
        for t in c["nodes"]:
            I = I_exact(0, 3, 2, t).ravel()
            rec = R.reconstruct(rom3, min(max(t, rom3["lo"]), rom3["hi"]))
            if R.find_cluster(t, rom3["lo"], rom3["hi"], rom3["n_k"]) != rom3["clusters"].index(c):
                continue
            mg = c["magic"][:n]
            assert np.abs(rec[mg] - I[mg]).max() <= 1e-12 * np.abs(I).max()


def test_full_reproduction_when_snapshots_are_fitting_nodes():
    """With the fitting nodes as the only snapshots and n_r = r + 1, the
    surrogate reproduces I exactly at those nodes."""
    p, q, r = 3, 2, 4
    nodes = 0.1 + 0.1 * gll_nodes(r)
    snaps = np.stack([I_exact(1, p, q, t).ravel() for t in nodes], axis=1)
    U, s = R.signed_svd(snaps)
    m = R.deim_points(U)
    for t in nodes:
        I = I_exact(1, p, q, t).ravel()
        Ir = np.linalg.solve(U[m], I[m])
        assert np.abs(U @ Ir - I).max() <= 1e-12 * np.abs(I).max()


def test_indicator_small(rom3):
    ind = R.offline_indicator(rom3, 0, n_test=6)
    for proj, surr in ind:
        assert proj < 1e-12 and surr < 1e-5


def test_reduced_derivative_fd(rom3):
    t, h = 0.137, 1e-6
    _, d = R.reduced_coordinates_dt(rom3, t)
    fd = (R.reduced_coordinates(rom3, t + h)[1] - R.reduced_coordinates(rom3, t - h)[1]) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-8 * np.abs(d).max())
