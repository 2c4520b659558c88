"""Block PCG over several load cases (lbddc_solve) against the same load cases
solved one after another (lbddc_solve_sequential), on small lattices drawn
with the recipe of the eight-load workload (random edge tractions, order-3
warped maps, mixed topologies):

  - each case runs its own recurrence in the same kernels and summation
    orders, so the iteration counts are equal and the solutions agree to
    1e-13 of the largest displacement (bit-for-bit equality is expected);
  - 3 and 8 cases form one block, 11 cases a block of 8 and one of 3;
  - one case has no load: it converges before the first iteration (zero
    solution) while the others iterate;
  - FP64 and mixed-precision preconditioners.
"""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [3, 8, 11])
def test_block_matches_sequential(nrhs, prec):
    from gpu_helpers import cut_to_rank, make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(5, nx=6, ny=5, p=4, nrhs=nrhs)
    zero = min(2, nrhs - 1)
    prob["traction"][zero] = 0.0
    roms = {f: cut_to_rank(r) for f, r in oracle_roms(prob).items()}
    s = make_solver(prob, roms)
    s.assemble()
    s.setup(lbddc.FP64 if prec == "fp64" else lbddc.MIXED)
    print(f"\n[block {nrhs} {prec}] block solve", flush=True)
    ib = s.solve(rtol=1e-10, max_iter=2000)
    ub = [s.displacement(r) for r in range(nrhs)]
    print(f"[block {nrhs} {prec}] sequential solve", flush=True)
    iseq = s.solve(rtol=1e-10, max_iter=2000, sequential=True)
    us = [s.displacement(r) for r in range(nrhs)]
    s.close()
    its_b = [i["iters"] for i in ib]
    its_s = [i["iters"] for i in iseq]
    worst = 0.0
    for r in range(nrhs):
        scale = np.abs(us[r]).max()
        if r == zero:
            assert scale == 0.0 and np.abs(ub[r]).max() == 0.0 and its_b[r] == 0
            continue
        worst = max(worst, np.abs(ub[r] - us[r]).max() / scale)
        assert ib[r]["rel_res"] <= 1e-10 and ib[r]["true_rel_res"] <= 1e-9
    print(f"[block {nrhs} {prec}] iterations block {its_b} sequential {its_s}; worst |u_b - u_s| / |u| {worst:.2e}")
    assert its_b == its_s
    assert worst <= 1e-13
