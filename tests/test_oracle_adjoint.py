"""Pins of the compliance gradient: central finite differences and the
energy identity."""
import numpy as np
import pytest
from oracle.bddc import Problem
from oracle.adjoint import compliance_gradient, fd_directional
from workloads import make_problem
from conftest import oracle_roms


@pytest.mark.parametrize("cfg,over", [(4, dict(nx=3, ny=2, p=4)), (5, dict(nx=2, ny=2, p=3, nrhs=2))])
def test_gradient_vs_central_fd(cfg, over):
    prob = make_problem(cfg, **over)
    roms = oracle_roms(prob)
    P = Problem(prob, roms)
    u = P.direct_solve()
    J, gX, gt = compliance_gradient(P, u)
    rng = np.random.default_rng(4242)
    for _ in range(4):
        dX = rng.normal(size=prob["ctrl"].shape)
        dt = rng.normal(size=prob["t"].shape)
        nrm = np.sqrt((dX**2).sum() + (dt**2).sum())
        dX, dt = dX / nrm, dt / nrm
        fd = fd_directional(prob, roms, dX, dt)
        ad = np.array([(gX[r] * dX).sum() + (gt[r] * dt).sum() for r in range(len(J))])
        assert np.all(np.abs(fd - ad) <= 1e-5 * np.abs(ad))


def test_energy_identity():
    prob = make_problem(1)
    P = Problem(prob, oracle_roms(prob))
    u = P.direct_solve()[0]
    d = P.dofs
    uf = np.zeros(d.N)
    m = d.free_id >= 0
    uf[2 * d.free_id[m]] = u[m, 0]
    uf[2 * d.free_id[m] + 1] = u[m, 1]
    K = P.global_K()
    f = P.global_f()[:, 0]
    assert abs(f @ uf - uf @ (K @ uf)) < 1e-12 * abs(f @ uf)
