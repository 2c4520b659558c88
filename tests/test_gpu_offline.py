"""The offline stage on the GPU (lbddc_implicit_tensors: an implicit-domain
quadrature per parameter vector, one thread each, then the snapshot
contraction) against the oracle, and the ROM it trains:

  - whole trimmed tensors I(mu) of the four Table 1 level sets at p = 4,
    q = 2, within 1e-12 of the oracle's (its own height-function rule,
    adaptive to rounding), and the entries mode equal to the whole tensor's
    entries;
  - a Schwarz Diamond ROM trained by rom_offline.train_implicit (the same
    Latin-hypercube draws as the oracle's trainer) reconstructs I at the
    cells of a lattice within 1e-9 of the oracle-trained ROM, with the same
    numerical ranks, and the lattice solved with it matches the
    oracle-trained one.
"""
import numpy as np
import pytest

from oracle import implicit as im
from oracle.trimmed import I_tpms
from workloads import make_problem, rom_lhs_draws

pytestmark = pytest.mark.gpu

MU = {2: [0.2, 0.8, 0.4, 0.6], 3: [0.1, 0.5, -0.3, 0.7], 4: [-3.0, -1.0, -5.0, 0.2], 5: [-2.0, 1.0, 0.5, 2.0]}


@pytest.fixture(scope="module")
def solver():
    from paper_2604_09113_amd import lbddc
    s = lbddc.Solver(0)
    yield s
    s.close()


@pytest.mark.parametrize("fam", [2, 3, 4, 5])
def test_snapshot_tensors(solver, fam):
    p, q = 4, 2
    mus = np.array([MU[fam], [m * 0.9 + 0.01 for m in MU[fam]]])
    print(f"\n[offline fam {fam}] GPU tensors", flush=True)
    I = solver.implicit_tensors(fam, p, q, mus)
    for k in range(len(mus)):
        ref = I_tpms(fam, p, q, mus[k]).ravel()
        e = np.abs(I[k] - ref).max() / np.abs(ref).max()
        print(f"[offline fam {fam}] mu {mus[k]}: |I - I_oracle| / |I| = {e:.2e}")
        assert e <= 1e-12
    ent = np.array([0, 17, 1234, len(I[0]) // 2 + 5, len(I[0]) - 1])
    E = solver.implicit_tensors(fam, p, q, mus, entries=ent)
    assert np.abs(E - I[:, ent]).max() <= 1e-13 * np.abs(I).max()


def test_trained_rom_matches_oracle_rom(solver):
    from conftest import oracle_roms
    from gpu_helpers import make_solver
    from oracle.rom import find_cluster_nd, reconstruct
    from paper_2604_09113_amd import lbddc, rom_offline
    rom_cfg = dict(lo=0.05, hi=0.95, n_k=2, n_s=6, n_r=6, r=1, dim=4)
    prob = make_problem(6, nx=4, ny=3, p=3, topo="schwarz_d", rom={2: rom_cfg})
    oroms = oracle_roms(prob)
    only = sorted({find_cluster_nd(m, 0.05, 0.95, 2) for m in prob["mu"]})
    u, perm = rom_lhs_draws(2, 2, 6, 4)
    print(f"\n[offline rom] training clusters {only} on the GPU", flush=True)
    g = rom_offline.train_implicit(solver, 2, 3, 2, 0.05, 0.95, 2, 6, 6, 1, u, perm, only=set(only))
    o = oroms[2]
    assert g["n_r"] == max(c["n_used"] for c in o["clusters"])
    worst = 0.0
    for m in prob["mu"]:
        k = find_cluster_nd(m, 0.05, 0.95, 2)
        ref = reconstruct(o, m)
        c = o["clusters"][k]
        # the GPU-trained surrogate at m: its cluster's basis times the Lagrange fit
        gl = dict(o, clusters=[dict(cc, U=g["U"][i], coeff=g["coeff"][i]) for i, cc in enumerate(o["clusters"])],
                  n_r=g["n_r"])
        val = reconstruct(gl, m)
        worst = max(worst, np.abs(val - ref).max() / np.abs(ref).max())
    print(f"[offline rom] max |I_gpu-trained - I_oracle-trained| / |I| over the cells: {worst:.2e}")
    assert worst <= 1e-9
    # the lattice solved with either ROM
    s1 = make_solver(prob, oroms)
    s1.assemble()
    s1.setup(lbddc.FP64)
    s1.solve(rtol=1e-13, max_iter=2000)
    u1 = s1.displacement(0)
    s1.close()
    s3 = lbddc.Solver(0)
    s3.load_rom(**g)
    from gpu_helpers import set_problem
    set_problem(s3, prob)
    s3.assemble()
    s3.setup(lbddc.FP64)
    s3.solve(rtol=1e-13, max_iter=2000)
    u3 = s3.displacement(0)
    s3.close()
    e = np.abs(u3 - u1).max() / np.abs(u1).max()
    print(f"[offline rom] |u(GPU-trained ROM) - u(oracle-trained ROM)| / |u| = {e:.2e}")
    assert e <= 1e-8
