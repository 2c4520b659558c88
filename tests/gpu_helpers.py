"""Shared helpers of the GPU tests: feed the oracle's trained ROM and the
seeded inputs to the C-ABI library, and map oracle per-cell data to the
library's export layouts."""
import numpy as np

from paper_2604_09113_amd import lbddc


def rom_arrays(rom):
    U = np.stack([c["U"] for c in rom["clusters"]])
    coeff = np.stack([c["coeff"] for c in rom["clusters"]])
    return dict(family=rom["family"], p=rom["p"], q=rom["q"], n_k=rom["n_k"], n_r=rom["n_r"], r=rom["r"],
                lo=rom["lo"], hi=rom["hi"], U=U, coeff=coeff, I_pi=rom["I_pi"])


def make_solver(prob, roms, moments=None):
    s = lbddc.Solver(0)
    for f, rom in roms.items():
        s.load_rom(**rom_arrays(rom))
    s.set_problem(prob["nx"], prob["ny"], prob["p"], prob["q"], prob["m"], prob["ctrl"], prob["family"], prob["t"],
                  prob["E"], prob["nu"], prob["rho"], prob["moments"] if moments is None else moments,
                  prob["traction"])
    return s


def rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)


def oracle_fine_operator(P, cell):
    """D [S C^T; C 0]^-1|_u D over the cell's active skeleton dofs, built by
    applying the oracle's Alg. 2 solve to unit vectors."""
    n = len(cell.U_glob)
    F = np.zeros((n, n))
    z = np.zeros(len(cell.C_glob))
    for j in range(n):
        e = np.zeros(n)
        e[j] = cell.D[j]
        x, _ = P.local_solve(cell, e, z)
        F[:, j] = cell.D * x
    return F
