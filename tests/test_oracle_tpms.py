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
