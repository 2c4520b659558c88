"""Boundary conditions and constraint sets through the C ABI, and the
failure contract of the calls that replace a problem or its geometry.

  - Lattices clamped on other sides than the left one, loaded on another
    side than the right one (Sec. 2.2.1), including corner cells with two
    clamped edges and loaded edges that end at clamped vertices: per-cell
    Schur complements, weights, coarse bases, loads against the oracle, the
    converged displacement against its direct solve (1e-8), iteration counts
    against its PCG (+-1) and the compliance gradient against its adjoint
    (1e-8).
  - Constraint sets (Sec. 3.3.1): the two supported ones reach the same
    converged displacement; unsupported sets, an empty clamped set and a
    clamped loaded side are rejected.
  - A rejected set_problem or set_geometry_device leaves the previous problem
    and every computed stage in place, bit for bit.
"""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu

SIDE_CASES = {
    "bottom_clamped_top_loaded_p4": (2, dict(nx=3, ny=4, p=4, m=2, jitter=0.03, clamped=("bottom",),
                                             loaded="top")),
    "right_top_clamped_left_loaded_p6_mixed": (3, dict(nx=4, ny=3, p=6, m=2, jitter=0.03,
                                                       clamped=("right", "top"), loaded="left")),
    "three_sides_clamped_p8_mixed": (3, dict(nx=2, ny=3, p=8, m=2, jitter=0.03,
                                             clamped=("left", "bottom", "top"), loaded="right")),
    "strip_bottom_loaded_p3_no_moments": (1, dict(nx=3, ny=1, p=3, clamped=("left", "right", "top"),
                                                  loaded="bottom")),
}


@pytest.fixture(scope="module", params=list(SIDE_CASES))
def sided(request):
    from oracle.bddc import Problem
    from gpu_helpers import make_solver
    cfg, over = SIDE_CASES[request.param]
    prob = make_problem(cfg, **over)
    roms = oracle_roms(prob)
    P = Problem(prob, roms)
    P.setup()
    print(f"\n[sides {request.param}] building solver", flush=True)
    s = make_solver(prob, roms)
    s.assemble()
    s.setup()
    info = s.solve(rtol=1e-12, max_iter=500)
    yield request.param, prob, roms, P, s, info
    s.close()


def test_sides_counts(sided):
    from paper_2604_09113_amd import lbddc
    name, prob, roms, P, s, _ = sided
    d = P.dofs
    got = (s.query(lbddc.Q_NDOF_FREE), s.query(lbddc.Q_N_SKELETON), s.query(lbddc.Q_N_COARSE))
    assert got == (d.N, d.N_U, d.N_C), (name, got)


def test_sides_cell_parity(sided):
    from gpu_helpers import rel
    name, prob, roms, P, s, _ = sided
    n = P.dofs.ncell
    S, D, Psi, SC, L = (s.export(w, 0, n) for w in (3, 4, 5, 6, 7))
    ws = wd = wp = wc = wl = 0.0
    for c, cell in enumerate(P.cells):
        a, ca = cell.slot_active, cell.coarse_active
        ws = max(ws, rel(S[c][np.ix_(a, a)], cell.S))
        assert np.all(D[c][~a] == 0) and np.all(Psi[c][:, ~ca] == 0)
        wd = max(wd, rel(D[c][a], cell.D))
        wp = max(wp, rel(Psi[c][np.ix_(a, ca)], cell.D[:, None] * cell.Psi))
        wc = max(wc, rel(SC[c][np.ix_(ca, ca)], cell.SC))
        wl = max(wl, rel(L[c][:, a].T, cell.f[cell.U_nat]))
    print(f"[{name}] S {ws:.2e} D {wd:.2e} Psi {wp:.2e} SC {wc:.2e} load {wl:.2e}")
    assert ws <= 1e-10 and wd <= 1e-12 and wl <= 1e-13 and wp <= 1e-9 and wc <= 1e-9


def test_sides_displacement_iterations_gradient(sided):
    from oracle.adjoint import compliance_gradient
    name, prob, roms, P, s, info = sided
    ud = P.direct_solve()
    u = s.displacement(0)
    err = np.abs(u - ud[0]).max() / np.abs(ud[0]).max()
    assert info[0]["rel_res"] <= 1e-12 and err <= 1e-8
    assert np.all(u[P.dofs.node_dirichlet] == 0.0)
    J, gX, gt = s.compliance_gradient()
    Jo, gXo, gto = compliance_gradient(P, ud)
    eJ = abs(J[0] - Jo[0]) / abs(Jo[0])
    eX = np.linalg.norm(gX - gXo) / np.linalg.norm(gXo)
    et = np.linalg.norm(gt - gto) / np.linalg.norm(gto)
    info8 = s.solve(rtol=1e-8)
    _, it, _ = P.pcg(P.rhs()[:, 0], 1e-8)
    print(f"[{name}] |u - u_direct| {err:.2e}; its gpu {info8[0]['iters']} oracle {it}; "
          f"J {eJ:.2e} dX {eX:.2e} dt {et:.2e}")
    assert abs(info8[0]["iters"] - it) <= 1
    assert eJ <= 1e-10 and eX <= 1e-8 and et <= 1e-8


def test_constraint_sets_and_rejections():
    from gpu_helpers import rom_arrays
    from paper_2604_09113_amd import lbddc
    prob = make_problem(2, nx=3, ny=3, p=4, m=2, jitter=0.03)
    roms = oracle_roms(prob)
    s = lbddc.Solver(0)
    for rom in roms.values():
        s.load_rom(**rom_arrays(rom))
    args = (prob["nx"], prob["ny"], prob["p"], prob["q"], prob["m"], prob["ctrl"], prob["family"], prob["t"],
            prob["E"], prob["nu"], prob["rho"], True, prob["traction"])
    us = []
    for cons in (lbddc.CON_CORNERS | lbddc.CON_EDGE_AVG, lbddc.CON_CORNERS | lbddc.CON_EDGE_AVG | lbddc.CON_EDGE_MOMENT):
        s.set_problem(*args, constraints=cons)
        s.assemble()
        s.setup()
        s.solve(rtol=1e-13, max_iter=500)
        us.append(s.displacement(0))
        assert s.query(lbddc.Q_NC_CELL) == (16 if cons == 3 else 20)
    d = np.abs(us[0] - us[1]).max() / np.abs(us[1]).max()
    print(f"\n[constraints] averages only vs averages + moments: |du| / |u| = {d:.2e}")
    assert d <= 1e-10
    for cons, st in ((lbddc.CON_CORNERS, lbddc.E_UNSUPPORTED), (lbddc.CON_EDGE_AVG, lbddc.E_UNSUPPORTED),
                     (lbddc.CON_CORNERS | lbddc.CON_EDGE_MOMENT, lbddc.E_UNSUPPORTED), (0, lbddc.E_UNSUPPORTED),
                     (8, lbddc.E_ARG)):
        with pytest.raises(lbddc.LbddcError) as ei:
            s.set_problem(*args, constraints=cons)
        assert ei.value.status == st, (cons, ei.value)
    with pytest.raises(lbddc.LbddcError) as ei:
        s.set_problem(*args, clamped=())
    assert ei.value.status == lbddc.E_ARG
    with pytest.raises(lbddc.LbddcError) as ei:
        s.set_problem(*args, clamped=("left", "right"), loaded="right")
    assert ei.value.status == lbddc.E_ARG
    # the context still holds the last accepted problem, all stages included
    assert np.array_equal(s.displacement(0), us[1])
    s.close()


def test_rejected_calls_keep_previous_state():
    """set_problem with a mirrored (det J < 0) net and set_geometry_device with
    a folded net or a thickness outside the ROM box are rejected; the previous
    problem keeps its stiffness, setup and solution, bit for bit, and solving
    and assembling again reproduce them."""
    import torch
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(3, nx=4, ny=3, p=4, m=2, jitter=0.03)
    roms = oracle_roms(prob)
    s = make_solver(prob, roms)
    s.assemble()
    s.setup()
    s.solve(rtol=1e-12, max_iter=500)
    n = prob["nx"] * prob["ny"]
    K0, S0, u0 = s.export(0, 0, n), s.export(3, 0, n), s.displacement(0)
    bad = dict(prob)
    bad["ctrl"] = prob["ctrl"] * np.array([-1.0, 1.0])
    with pytest.raises(lbddc.LbddcError) as ei:
        s.set_problem(bad["nx"], bad["ny"], bad["p"], bad["q"], bad["m"], bad["ctrl"], bad["family"], bad["t"],
                      bad["E"], bad["nu"], bad["rho"], bad["moments"], bad["traction"])
    assert ei.value.status == lbddc.E_DEGENERATE_MAP
    assert np.array_equal(s.displacement(0), u0)
    assert np.array_equal(s.export(0, 0, n), K0) and np.array_equal(s.export(3, 0, n), S0)
    # a folded net: one interior control point pushed across its neighbours
    folded = prob["ctrl"].copy()
    folded[2, 2] += np.array([1.6, 0.0])
    for ctrl, t, st in ((folded, prob["t"], lbddc.E_DEGENERATE_MAP),
                        (prob["ctrl"], np.where(np.arange(n) == 5, 0.35, prob["t"]), lbddc.E_PARAM_RANGE)):
        dc = torch.tensor(ctrl, dtype=torch.float64, device="cuda")
        dt = torch.tensor(t, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(lbddc.LbddcError) as ei:
            s.set_geometry_device(dc.data_ptr(), dt.data_ptr())
        assert ei.value.status == st, ei.value
        # every stage is still there: the solution, the stiffness, the setup
        assert np.array_equal(s.displacement(0), u0)
        assert np.array_equal(s.export(0, 0, n), K0) and np.array_equal(s.export(3, 0, n), S0)
        s.solve(rtol=1e-12, max_iter=500)
        assert np.array_equal(s.displacement(0), u0)
    s.assemble()
    assert np.array_equal(s.export(0, 0, n), K0)
    s.close()
