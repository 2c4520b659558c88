"""Edge cases of the method through the C ABI.

  - The smallest lattices: one cell, one row, one column, two cells.  The
    coarse problem then has a one- to three-node tree and a cell can touch
    the clamped and the loaded edge at once.  Converged displacements against
    the oracle's sparse direct solve (1e-8), iteration counts against the
    oracle's PCG (+-1), gradients against the oracle's adjoint (1e-8), and the
    mixed-precision solve within 1e-8 of the FP64 one.
  - No load: the solve stops before the first iteration with u = 0, and the
    compliance and its gradient are zero.
  - Thickness at the ends of its family's trained box is accepted; past them
    the problem is rejected (Sec. 4.2: the ROM covers its box only).
  - A mirrored control net (det J < 0 in every cell) is rejected (Sec. 4.1:
    regular maps only).
  - Calls out of order are rejected and leave the context usable.
"""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu

SMALL = [(1, 1), (1, 3), (3, 1), (2, 1)]


@pytest.mark.parametrize("nx,ny", SMALL)
def test_small_lattices_against_oracle(nx, ny):
    from gpu_helpers import make_solver
    from oracle.adjoint import compliance_gradient
    from oracle.bddc import Problem
    from paper_2604_09113_amd import lbddc
    prob = make_problem(1, nx=nx, ny=ny, p=3)
    roms = oracle_roms(prob)
    P = Problem(prob, roms)
    P.setup()
    ud = P.direct_solve()
    s = make_solver(prob, roms)
    s.assemble()
    s.setup()
    info = s.solve(rtol=1e-12, max_iter=200)
    u = s.displacement(0)
    err = np.abs(u - ud[0]).max() / np.abs(ud[0]).max()
    info8 = s.solve(rtol=1e-8, max_iter=200)
    _, it, _ = P.pcg(P.rhs()[:, 0], 1e-8)
    s.solve(rtol=1e-12, max_iter=200)
    J, gX, gt = s.compliance_gradient()
    Jo, gXo, gto = compliance_gradient(P, ud)
    eJ = abs(J[0] - Jo[0]) / abs(Jo[0])
    eX = np.linalg.norm(gX - gXo) / np.linalg.norm(gXo)
    et = np.linalg.norm(gt - gto) / np.linalg.norm(gto)
    s.setup(lbddc.MIXED)
    s.solve(rtol=1e-12, max_iter=200)
    dm = np.abs(s.displacement(0) - u).max() / np.abs(u).max()
    print(f"\n[edges {nx}x{ny}] its {info[0]['iters']} |u - u_direct| {err:.2e}; rtol 1e-8 gpu "
          f"{info8[0]['iters']} oracle {it}; J {eJ:.2e} dX {eX:.2e} dt {et:.2e}; mixed {dm:.2e}")
    assert info[0]["rel_res"] <= 1e-12 and err <= 1e-8
    assert abs(info8[0]["iters"] - it) <= 1
    assert eJ <= 1e-10 and eX <= 1e-8 and et <= 1e-8
    assert dm <= 1e-8
    s.close()


def test_no_load_gives_zero_solution_and_gradient():
    from gpu_helpers import make_solver
    prob = make_problem(1, nx=3, ny=2, p=3)
    prob["traction"] = np.zeros_like(prob["traction"])
    s = make_solver(prob, oracle_roms(prob))
    s.assemble()
    s.setup()
    info = s.solve(rtol=1e-10, max_iter=100)
    J, gX, gt = s.compliance_gradient()
    print(f"\n[edges no load] its {info[0]['iters']} rel_res {info[0]['rel_res']}")
    assert info[0]["iters"] == 0 and info[0]["rel_res"] == 0.0
    assert not np.any(s.displacement(0))
    assert J[0] == 0.0 and not np.any(gX) and not np.any(gt)
    s.close()


def test_thickness_box_ends_accepted_and_outside_rejected():
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(1, nx=3, ny=2, p=3)
    roms = oracle_roms(prob)
    r = roms[0]
    t = prob["t"].copy()
    t[0], t[-1] = r["lo"], r["hi"]
    s = make_solver(dict(prob, t=t), roms)
    s.assemble()
    s.setup()
    info = s.solve(rtol=1e-10, max_iter=200)
    assert info[0]["rel_res"] <= 1e-10
    s.close()
    for bad in (r["lo"] - 1e-9, r["hi"] + 1e-9):
        t2 = prob["t"].copy()
        t2[1] = bad
        with pytest.raises(lbddc.LbddcError) as ex:
            make_solver(dict(prob, t=t2), roms)
        assert ex.value.status == lbddc.E_PARAM_RANGE


def test_mirrored_map_rejected():
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(1, nx=3, ny=2, p=3)
    ctrl = prob["ctrl"].copy()
    ctrl[..., 0] = -ctrl[..., 0]
    with pytest.raises(lbddc.LbddcError) as ex:
        make_solver(dict(prob, ctrl=ctrl), oracle_roms(prob))
    assert ex.value.status == lbddc.E_DEGENERATE_MAP


def test_calls_out_of_order_rejected():
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(1, nx=3, ny=2, p=3)
    s = make_solver(prob, oracle_roms(prob))
    for call in (lambda: s.setup(), lambda: s.solve(), lambda: s.compliance_gradient(), lambda: s.displacement(0)):
        with pytest.raises(lbddc.LbddcError) as ex:
            call()
        assert ex.value.status == lbddc.E_STATE
    s.assemble()
    s.setup()
    assert s.solve(rtol=1e-10, max_iter=200)[0]["rel_res"] <= 1e-10
    s.close()


def test_assembly_groups_follow_the_geometry():
    """The assembly reuses its cell sort by ROM cluster while the geometry is
    unchanged: two assemblies give identical K_i; after set_geometry_device
    moves cells across the cluster boundary, K_i equals that of a fresh solver
    built with the new thickness (bit for bit: the same kernels)."""
    import torch
    from gpu_helpers import cut_to_rank, make_solver
    prob = make_problem(3, nx=6, ny=5, p=4)
    roms = {f: cut_to_rank(r) for f, r in oracle_roms(prob).items()}
    ncell = prob["nx"] * prob["ny"]
    s = make_solver(prob, roms)
    s.assemble()
    K0 = s.export(0, 0, ncell)
    s.assemble()
    assert np.array_equal(s.export(0, 0, ncell), K0)
    # every cell to the other half of its family's box (n_k = 2 clusters)
    lo, hi = 0.1, 0.3
    t1 = np.where(prob["t"] < 0.5 * (lo + hi), prob["t"] + 0.09, prob["t"] - 0.09)
    ctrl_d = torch.tensor(prob["ctrl"], dtype=torch.float64, device="cuda")
    t_d = torch.tensor(t1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.set_geometry_device(ctrl_d.data_ptr(), t_d.data_ptr())
    s.assemble()
    K1 = s.export(0, 0, ncell)
    s.close()
    p1 = dict(prob, t=np.ascontiguousarray(t1))
    s1 = make_solver(p1, roms)
    s1.assemble()
    K1_fresh = s1.export(0, 0, ncell)
    s1.close()
    assert not np.array_equal(K1, K0)
    assert np.array_equal(K1, K1_fresh)
