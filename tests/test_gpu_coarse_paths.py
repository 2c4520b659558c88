"""The coarse solve on a lattice large enough for every sweep kernel: a
64 x 64, p = 3 lattice has an 11-level nested-dissection tree whose bottom
levels are swept one subtree per workgroup, whose middle levels have enough
items for the one-item-per-wave kernels, and whose top levels use the
workgroup kernels.  Compared with the oracle: the same PCG (equal iteration
counts) and the displacement of its sparse direct solve."""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu


def test_all_sweep_kernels_against_oracle():
    from gpu_helpers import make_solver
    from oracle.bddc import Problem
    from paper_2604_09113_amd import lbddc
    prob = make_problem(1, nx=64, ny=64, p=3)
    roms = oracle_roms(prob)
    s = make_solver(prob, roms)
    levels, launches = s.query(lbddc.Q_COARSE_LEVELS), s.query(lbddc.Q_COARSE_SWEEP_LAUNCHES)
    print(f"\n[coarse paths] {levels} tree levels, {launches} launches per sweep", flush=True)
    assert launches < levels  # the bottom levels are swept as subtrees
    s.assemble()
    s.setup()
    info = s.solve(rtol=1e-12, max_iter=500)
    print("[coarse paths] oracle setup", flush=True)
    P = Problem(prob, roms)
    P.setup()
    ud = P.direct_solve()[0]
    u = s.displacement(0)
    err = np.abs(u - ud).max() / np.abs(ud).max()
    info8 = s.solve(rtol=1e-8)
    _, it, _ = P.pcg(P.rhs()[:, 0], 1e-8)
    print(f"[coarse paths] iters rtol 1e-12 {info[0]['iters']}, |u - u_direct| {err:.2e}; "
          f"rtol 1e-8 gpu {info8[0]['iters']} oracle {it}")
    assert info[0]["rel_res"] <= 1e-12 and err <= 1e-8
    assert abs(info8[0]["iters"] - it) <= 1
    s.close()
