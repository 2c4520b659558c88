"""Write the oracle's reference values for the paper's benchmark lattice: the
quarter annulus of 184 x 92 Schwarz Diamond cells (16,928 cells, order-3
maps, thresholds mu = 0.9 - 0.8 xi~_1 at the vertices, E = 5,
nu = 0.25, traction 0.1 downward on the material part of the loaded edges,
corners + averages + moments on the material part of each edge), with
rho = 1e-2: the small ROM below leaves some constrained local problems
singular to rounding at the benchmark's 2e-3.

Calls the oracle only (ROM training with its implicit-domain quadrature, cell
build, BDDC-PCG, interior recovery, compliance adjoint with dJ/dmu), on the
seeded inputs of the workloads module.  The degree is p = 4 and the ROM a
small one (one cluster, 20 Latin-hypercube snapshots, r = 2 per threshold:
101 implicit quadratures), so that the GPU test can train the same ROM with
the oracle in under a minute; the lattice, the geometry, the loads and the
solver are those of the benchmark (which runs p = 8).  PCG runs to a relative residual of 1e-14; the iteration count
at which the same recurrence first reaches 1e-8 is recorded too.

Output: annulus184x92_p4_oracle.json beside this script, holding sizes, the
ROM specification and rank, iteration counts, J, and strided samples of u,
dJ/dX and dJ/dmu.

Run:  python tests/golden/make_annulus184x92_p4.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import make_problem, rom_lhs_draws  # noqa: E402
from oracle.rom import train  # noqa: E402
from oracle.bddc import Problem  # noqa: E402
from oracle.adjoint import compliance_gradient  # noqa: E402

ROM = {2: dict(lo=0.1, hi=0.9, n_k=1, n_s=20, n_r=20, r=2, dim=4)}
P_DEG = 4
RHO = 1e-2
U_STRIDE = 1031
X_STRIDE = 61
MU_STRIDE = 7


def main(out_name="annulus184x92_p4_oracle.json"):
    t0 = time.time()
    prob = make_problem(7, rom=ROM, p=P_DEG, rho=RHO)
    s = ROM[2]
    u_lhs, perm = rom_lhs_draws(2, s["n_k"], s["n_s"], s["dim"])
    roms = {2: train(2, prob["p"], prob["q"], s["lo"], s["hi"], s["n_k"], s["n_s"], s["n_r"], s["r"], u_lhs,
                     dim=s["dim"], lhs_perm=perm)}
    print(f"rom {time.time() - t0:.0f} s", flush=True)
    P = Problem(prob, roms)
    print(f"cells built {time.time() - t0:.0f} s", flush=True)
    P.setup()
    print(f"setup {time.time() - t0:.0f} s", flush=True)
    F = P.rhs()
    x, it, hist = P.pcg(F[:, 0], rtol=1e-14, max_iter=3000)
    it8 = int(np.argmax(hist <= 1e-8))
    print(f"pcg {it} iterations (1e-8 after {it8}) {time.time() - t0:.0f} s", flush=True)
    u = P.recover(x, 0)[None]
    J, gX, gt, gmu = compliance_gradient(P, u, thresholds=True)
    print(f"gradient {time.time() - t0:.0f} s  J = {J[0]!r}", flush=True)
    uf = u[0].ravel()
    gXf = gX[0].ravel()
    gmf = gmu[0].ravel()
    iu = np.arange(0, uf.size, U_STRIDE)
    ix = np.arange(0, gXf.size, X_STRIDE)
    im = np.arange(0, gmf.size, MU_STRIDE)
    d = P.dofs
    res = dict(
        workload="184x92 quarter annulus of Schwarz Diamond cells, p=4, order-3 maps, mu = 0.9 - 0.8 xi~_1",
        nx=prob["nx"], ny=prob["ny"], p=prob["p"], rho=prob["rho"], rom={str(k): v for k, v in ROM.items()},
        N=int(d.N), N_U=int(d.N_U), N_C=int(d.N_C), n_r=int(roms[2]["n_r"]),
        rtol=1e-14, iters=int(it), iters_1e8=it8, history=[float(h) for h in hist],
        J=float(J[0]), u_max=float(np.abs(uf).max()), gX_max=float(np.abs(gXf).max()),
        gmu_max=float(np.abs(gmf).max()),
        u_stride=U_STRIDE, u=[float(v) for v in uf[iu]],
        gX_stride=X_STRIDE, gX=[float(v) for v in gXf[ix]],
        gmu_stride=MU_STRIDE, gmu=[float(v) for v in gmf[im]],
        seconds=round(time.time() - t0, 1),
    )
    with open(os.path.join(HERE, out_name), "w") as fh:
        json.dump(res, fh, indent=0)
    print(f"written in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
