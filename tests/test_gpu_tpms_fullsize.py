"""The Table 1 path at the size of the benchmark: the 128 x 128, p = 8
Schwarz Diamond lattice with the graded four-corner threshold, its ROM (16
clusters x 7^4 fitting nodes, n_r = 40) trained on the GPU:

  - two snapshot tensors I(mu) at p = 8 against the oracle's implicit
    quadrature (1e-12);
  - sampled cells: the stabilised reduced vector against the oracle's
    evaluation of the same ROM (1e-13) and K_i against the oracle's ROM
    stiffness (1e-10);
  - the FP64 solve to rtol 1e-10 has a true residual below 1e-9, and the
    mixed solve at rtol 1e-10 lands within 1e-8 of it;

and the paper's own benchmark lattice (the quarter annulus of 184 x 92
cells): sampled edge rows against the oracle and the FP64 solve.
"""
import numpy as np
import pytest

from workloads import make_problem, rom_lhs_draws

pytestmark = pytest.mark.gpu


def oracle_form(rom):
    """The GPU-trained arrays as an oracle ROM dict (cluster boxes from the box
    and n_k, first threshold fastest)."""
    from oracle.rom import cluster_box
    cl = [dict(U=rom["U"][k], coeff=rom["coeff"][k], box=cluster_box(k, rom["lo"], rom["hi"], rom["n_k"], 4))
          for k in range(rom["n_k"] ** 4)]
    return dict(family=rom["family"], p=rom["p"], q=rom["q"], lo=rom["lo"], hi=rom["hi"], n_k=rom["n_k"],
                n_r=rom["n_r"], r=rom["r"], dim=4, I_pi=rom["I_pi"], clusters=cl)


def test_schwarz_d_128_p8():
    from gpu_helpers import set_problem
    from oracle.assembly import rom_K
    from oracle.geometry import cell_control_points, material_tensor
    from oracle.rom import stabilised_reduced
    from oracle.trimmed import I_tpms
    from paper_2604_09113_amd import lbddc, rom_offline
    prob = make_problem(6)
    sc = prob["rom"][2]
    s = lbddc.Solver(0)
    print("\n[tpms128] snapshot tensors at p = 8", flush=True)
    mus = prob["mu"][[5, 9000]]
    I = s.implicit_tensors(2, 8, 2, mus)
    for k in range(2):
        ref = I_tpms(2, 8, 2, mus[k]).ravel()
        e = np.abs(I[k] - ref).max() / np.abs(ref).max()
        print(f"[tpms128] I(mu) cell {k}: {e:.2e}", flush=True)
        assert e <= 1e-12
    print("[tpms128] training the ROM on the GPU", flush=True)
    u, perm = rom_lhs_draws(2, sc["n_k"], sc["n_s"], 4)
    rom = rom_offline.train_implicit(s, 2, 8, 2, sc["lo"], sc["hi"], sc["n_k"], sc["n_s"], sc["n_r"], sc["r"], u, perm)
    s.load_rom(**rom)
    set_problem(s, prob)
    s.assemble(lbddc.FP64)
    orom = oracle_form(rom)
    Cmat = material_tensor(prob["E"], prob["nu"])
    cells = np.linspace(0, prob["nx"] * prob["ny"] - 1, 12).astype(int)
    e_it = e_K = 0.0
    for c in cells:
        it = s.export(lbddc.X_ITIL, int(c), 1)[0]
        _, ref = stabilised_reduced(orom, prob["mu"][c], prob["rho"])
        e_it = max(e_it, np.abs(it[:len(ref)] - ref).max() / np.abs(ref).max())
        iy, ix = divmod(int(c), prob["nx"])
        Kr = rom_K(cell_control_points(prob["ctrl"], prob["m"], ix, iy), orom, prob["mu"][c], prob["rho"], Cmat)
        K = s.export(lbddc.X_K, int(c), 1)[0]
        e_K = max(e_K, np.abs(K - Kr).max() / np.abs(Kr).max())
    print(f"[tpms128] sampled cells: Itil {e_it:.2e}, K {e_K:.2e}", flush=True)
    assert e_it <= 1e-13 and e_K <= 1e-10
    s.setup(lbddc.FP64)
    inf = s.solve(rtol=1e-10, max_iter=3000)
    u64 = s.displacement(0)
    s.setup(lbddc.MIXED)
    infm = s.solve(rtol=1e-10, max_iter=3000)
    um = s.displacement(0)
    s.close()
    e = np.abs(um - u64).max() / np.abs(u64).max()
    print(f"[tpms128] FP64 {inf[0]['iters']} its, true residual {inf[0]['true_rel_res']:.1e}; mixed {infm[0]['iters']} "
          f"its, |u_mixed - u_fp64| / |u| = {e:.1e}")
    assert inf[0]["true_rel_res"] <= 1e-9 and e <= 1e-8


def test_paper_annulus_184x92_p8():
    """The paper's benchmark geometry at its largest size (184 x 92 cells on
    the quarter annulus, p = 8, order-3 maps): the edge rows on the material
    part of sampled cells against the oracle's (1e-12), and the FP64 solve to
    rtol 1e-8 with a true residual below 1e-8.  The iteration count is
    printed and held to at most 20 (17 when measured; the paper reports 17
    for this lattice, and the whole-edge rows took 46); the mixed-precision
    solve takes at most two more."""
    from gpu_helpers import oracle_rows, set_problem
    from paper_2604_09113_amd import lbddc, rom_offline
    prob = make_problem(7)
    sc = prob["rom"][2]
    s = lbddc.Solver(0)
    print("\n[annulus] training the ROM on the GPU", flush=True)
    u, perm = rom_lhs_draws(2, sc["n_k"], sc["n_s"], 4)
    rom = rom_offline.train_implicit(s, 2, 8, 2, sc["lo"], sc["hi"], sc["n_k"], sc["n_s"], sc["n_r"], sc["r"], u, perm)
    s.load_rom(**rom)
    set_problem(s, prob)
    s.assemble(lbddc.FP64)
    nc = prob["nx"] * prob["ny"]
    worst = 0.0
    for c in np.linspace(0, nc - 1, 24).astype(int):
        rows = s.export(lbddc.X_CONS, int(c), 1)[0]
        ref = oracle_rows(prob, c, prob["p"])
        worst = max(worst, np.abs(rows - ref).max() / np.abs(ref).max())
    print(f"[annulus] sampled edge rows: {worst:.2e}", flush=True)
    assert worst <= 1e-12
    s.setup(lbddc.FP64)
    inf = s.solve(rtol=1e-8, max_iter=500)
    s.setup(lbddc.MIXED)
    infm = s.solve(rtol=1e-8, max_iter=500)
    s.close()
    print(f"[annulus] FP64: {inf[0]['iters']} iterations, true residual {inf[0]['true_rel_res']:.1e}; "
          f"mixed: {infm[0]['iters']} iterations")
    assert inf[0]["true_rel_res"] <= 1e-8 and inf[0]["iters"] <= 20
    # the mixed preconditioner is formed in FP64 and stored in FP32: at the
    # paper's rho its iteration count stays with the FP64 one (an FP32-formed
    # one needed 43)
    assert infm[0]["iters"] <= inf[0]["iters"] + 2
