"""Write the oracle's reference values for the 128 x 128, p = 8 mixed
circle/cross lattice (16,384 cells, order-2 jittered map, unit traction on the
right side, left side clamped, rho = 5e-4, corners + averages + moments).

Calls the oracle only (ROM training, cell build, BDDC-PCG, interior recovery,
compliance adjoint), on the seeded inputs of the workloads module.  The ROMs
are the oracle's, cut to their numerical rank (the reduced size the library
runs this lattice with).  PCG runs to a relative residual of 1e-14 (so that
the stored compliance, which is first order in the solver error, is exact to
about 1e-12); the iteration count at which the same recurrence first reaches
1e-8 is recorded too.

Output: lattice128_p8_oracle.json beside this script, holding
  - sizes and the ROM ranks;
  - iteration counts at 1e-8 and 1e-14 and the recurrence history;
  - the compliance J;
  - a strided sample of the nodal displacement u[gy, gx, c] (flat index into
    the [Gy][Gx][2] lattice);
  - dJ/dt of every eighth cell;
  - a strided sample of dJ/dX (flat index into the [(2ny+1)][(2nx+1)][2] net).

Run:  python tests/golden/make_lattice128_p8.py      (about 40 minutes)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import make_problem, rom_lhs_uniforms  # noqa: E402
from oracle.rom import train  # noqa: E402
from oracle.bddc import Problem  # noqa: E402
from oracle.adjoint import compliance_gradient  # noqa: E402

U_STRIDE = 1031     # prime, so the sample visits every node position class
X_STRIDE = 61
T_STRIDE = 8


def cut(rom):
    nr = max(c["n_used"] for c in rom["clusters"])
    out = dict(rom, n_r=nr)
    out["clusters"] = [dict(c, U=c["U"][:, :nr], coeff=c["coeff"][:, :nr]) for c in rom["clusters"]]
    return out


def main(nx=128, out_name="lattice128_p8_oracle.json"):
    t0 = time.time()
    prob = make_problem(3, nx=nx, ny=nx)
    roms = {}
    for f, s in prob["rom"].items():
        roms[f] = cut(train(f, prob["p"], prob["q"], s["lo"], s["hi"], s["n_k"], s["n_s"], s["n_r"], s["r"],
                            rom_lhs_uniforms(f, s["n_k"], s["n_s"])))
    print(f"roms {time.time() - t0:.0f} s", flush=True)
    P = Problem(prob, roms)
    print(f"cells built {time.time() - t0:.0f} s", flush=True)
    P.setup()
    print(f"setup {time.time() - t0:.0f} s", flush=True)
    F = P.rhs()
    x, it, hist = P.pcg(F[:, 0], rtol=1e-14, max_iter=3000)
    it8 = int(np.argmax(hist <= 1e-8))
    print(f"pcg {it} iterations (1e-8 after {it8}) {time.time() - t0:.0f} s", flush=True)
    u = P.recover(x, 0)[None]
    J, gX, gt = compliance_gradient(P, u)
    print(f"gradient {time.time() - t0:.0f} s  J = {J[0]!r}", flush=True)
    uf = u[0].ravel()
    gXf = gX[0].ravel()
    iu = np.arange(0, uf.size, U_STRIDE)
    ix = np.arange(0, gXf.size, X_STRIDE)
    ic = np.arange(0, prob["nx"] * prob["ny"], T_STRIDE)
    d = P.dofs
    res = dict(
        workload="128x128 p=8 mixed circle/cross, order-2 map jitter N(0,0.03), seed 3",
        nx=prob["nx"], ny=prob["ny"], p=prob["p"],
        N=int(d.N), N_U=int(d.N_U), N_C=int(d.N_C),
        n_r={str(f): int(r["n_r"]) for f, r in roms.items()},
        rtol=1e-14, iters=int(it), iters_1e8=it8, history=[float(h) for h in hist],
        J=float(J[0]), u_max=float(np.abs(uf).max()), gX_max=float(np.abs(gXf).max()),
        gt_max=float(np.abs(gt[0]).max()),
        u_stride=U_STRIDE, u=[float(v) for v in uf[iu]],
        gX_stride=X_STRIDE, gX=[float(v) for v in gXf[ix]],
        gt_stride=T_STRIDE, gt=[float(v) for v in gt[0][ic]],
        seconds=round(time.time() - t0, 1),
    )
    with open(os.path.join(HERE, out_name), "w") as fh:
        json.dump(res, fh, indent=0)
    print(f"written in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
