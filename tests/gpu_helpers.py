"""Shared helpers of the GPU tests: feed the oracle's trained ROM and the
seeded inputs to the C-ABI library, and map oracle per-cell data to the
library's export layouts."""
import numpy as np

from paper_2604_09113_amd import lbddc


def rom_arrays(rom):
    U = np.stack([c["U"] for c in rom["clusters"]])
    coeff = np.stack([c["coeff"] for c in rom["clusters"]])
    return dict(family=rom["family"], p=rom["p"], q=rom["q"], n_k=rom["n_k"], n_r=rom["n_r"], r=rom["r"],
                lo=rom["lo"], hi=rom["hi"], U=U, coeff=coeff, I_pi=rom["I_pi"], dim=rom.get("dim", 1))


def set_problem(s, prob, moments=None):
    """set_problem with every field of a workloads problem dict."""
    s.set_problem(prob["nx"], prob["ny"], prob["p"], prob["q"], prob["m"], prob["ctrl"], prob["family"], prob["t"],
                  prob["E"], prob["nu"], prob["rho"], prob["moments"] if moments is None else moments,
                  prob["traction"], clamped=prob.get("clamped", ("left",)), loaded=prob.get("loaded", "right"),
                  mu=prob.get("mu"))


def make_solver(prob, roms, moments=None):
    s = lbddc.Solver(0)
    for f, rom in roms.items():
        s.load_rom(**rom_arrays(rom))
    set_problem(s, prob, moments)
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


def cut_to_rank(rom):
    """The oracle's ROM truncated to its numerical rank (the reduced size the
    library is run with at full size)."""
    nr = max(c["n_used"] for c in rom["clusters"])
    out = dict(rom, n_r=nr)
    out["clusters"] = [dict(c, U=c["U"][:, :nr], coeff=c["coeff"][:, :nr]) for c in rom["clusters"]]
    return out


def oracle_cells(prob, roms, cells):
    """Oracle Cell objects of selected cells only (the oracle's own cell build,
    without building the whole lattice)."""
    from oracle.bddc import Problem
    from oracle.dofs import Dofs, side_cells
    from oracle.geometry import material_tensor
    P = Problem.__new__(Problem)
    P.prob, P.p, P.q, P.m = prob, prob["p"], prob["q"], prob["m"]
    P.nx, P.ny, P.rho, P.moments = prob["nx"], prob["ny"], prob["rho"], prob["moments"]
    P.clamped, P.loaded = tuple(prob.get("clamped", ("left",))), prob.get("loaded", "right")
    P.dofs = Dofs(P.nx, P.ny, P.p, P.moments, P.clamped)
    P.load_pos = {c: k for c, k in side_cells(P.nx, P.ny, P.loaded)}
    P.Cmat = material_tensor(prob["E"], prob["nu"])
    P.roms, P.assembly, P.nrhs = roms, "rom", prob["traction"].shape[0]
    return P, {c: P._build_cell(c) for c in cells}


def sampled_cell_errors(prob, roms, s, cells):
    """Largest relative errors of K, S (active slots), theta and Itil of the
    sampled cells against the oracle."""
    from oracle.geometry import geometry_coefficients
    from oracle.rom import stabilised_reduced
    P, oc = oracle_cells(prob, roms, cells)
    wk = ws = wt = wi = 0.0
    for c in cells:
        cell = oc[c]
        C, _ = geometry_coefficients(cell.X, prob["q"], P.Cmat)
        th = s.export(1, c, 1)[0]
        wt = max(wt, np.abs(th - C).max() / np.abs(C).max())
        _, v = stabilised_reduced(roms[int(prob["family"][c])], float(prob["t"][c]), prob["rho"])
        it = s.export(2, c, 1)[0]
        wi = max(wi, np.abs(it[:len(v)] - v).max() / max(1.0, np.abs(v).max()))
        wk = max(wk, rel(s.export(0, c, 1)[0], cell.K))
        a = cell.slot_active
        ws = max(ws, rel(s.export(3, c, 1)[0][np.ix_(a, a)], cell.S))
    return wk, ws, wt, wi


def compliance_fTu(prob, u, rhs):
    """f_r^T u with the oracle's traction load on the right-edge cells."""
    from oracle.bddc import traction_load
    from oracle.dofs import edge_nodes_local
    from oracle.geometry import cell_control_points
    p, nx, ny, m = prob["p"], prob["nx"], prob["ny"], prob["m"]
    J = 0.0
    for iy in range(ny):
        X = cell_control_points(prob["ctrl"], m, nx - 1, iy)
        fe = traction_load(X, p, prob["traction"][rhs, iy])
        for n, (a, b) in enumerate(edge_nodes_local(p, "right")):
            J += fe[n] @ u[p * iy + b, p * (nx - 1) + a]
    return J


def fp32_contraction_bound(prob, roms, cell_X, c, depth):
    """First-order rounding bound of the FP32 contraction of cell c, entry by
    entry: the library rounds Uhat, Itil and theta to FP32 (3 roundings) and
    accumulates the depth-`depth` reconstruction and the 4 (q+1)^2-term theta
    sum in FP32, so |K32 - K| <= gamma * Kabs with gamma = (depth + ns + 3) u,
    u = 2^-24, and Kabs the same contraction of the absolute values
    |theta| . (|Uhat| |Itil|).  Returns (gamma, Kabs)."""
    from oracle.assembly import contract
    from oracle.geometry import geometry_coefficients, material_tensor
    from oracle.rom import stabilised_reduced
    rom = roms[int(prob["family"][c])]
    k, itil = stabilised_reduced(rom, float(prob["t"][c]), prob["rho"])
    Uhat = np.concatenate([rom["clusters"][k]["U"], rom["I_pi"][:, None]], axis=1)
    p, q = rom["p"], rom["q"]
    nB, nL = (p + 1) ** 2, (q + 1) ** 2
    Iabs = (np.abs(Uhat) @ np.abs(itil)).reshape(nB, nB, 2, 2, nL)
    C, _ = geometry_coefficients(cell_X, q, material_tensor(prob["E"], prob["nu"]))
    Kabs = contract(Iabs, np.abs(C))
    gamma = (depth + 4 * nL + 3) * 2.0 ** -24
    return gamma, Kabs


def assembled_coarse_matrix(s, ncell):
    """S_C = sum_i R_C^(i)T (Psi^T S Psi)^(i) R_C^(i) assembled with
    scipy.sparse from the library's per-cell exports (SC and RC): an
    assembly independent of the library's nested-dissection fronts."""
    import scipy.sparse as sp
    from paper_2604_09113_amd import lbddc
    SC = s.export(lbddc.X_SC, 0, ncell)
    RC = s.export(lbddc.X_RC, 0, ncell).astype(np.int64)
    N = s.query(lbddc.Q_N_COARSE)
    nC = RC.shape[1]
    rows = np.repeat(RC[:, :, None], nC, axis=2)
    cols = np.repeat(RC[:, None, :], nC, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    return sp.csr_matrix((SC[keep], (rows[keep], cols[keep])), shape=(N, N))


def coarse_solve_errors(s, A, nz=3, seed=5):
    """Backward error max ||A g - z||_inf / (||A||_inf ||g||_inf + ||z||_inf)
    of the library's coarse solve for random z, and the g it returned."""
    rng = np.random.default_rng(seed)
    anorm = abs(A).sum(axis=1).max()
    worst, out = 0.0, []
    for _ in range(nz):
        z = rng.normal(size=A.shape[0])
        g = s.coarse_solve(z)
        r = A @ g - z
        worst = max(worst, np.abs(r).max() / (anorm * np.abs(g).max() + np.abs(z).max()))
        out.append((z, g))
    return worst, out


def oracle_rows(prob, c, p):
    """The oracle's edge rows of cell c, [4 edges][nce][p+1][2]."""
    from oracle.bddc import edge_constraint_rows
    from oracle.dofs import EDGES
    from oracle.geometry import cell_control_points
    from oracle.implicit import TrimmedCell
    from oracle.trimmed import param_dim
    iy, ix = divmod(int(c), prob["nx"])
    X = cell_control_points(prob["ctrl"], prob["m"], ix, iy)
    fam = int(prob["family"][c])
    dom = TrimmedCell(fam, prob["mu"][c]) if param_dim(fam) == 4 else None
    return np.stack([edge_constraint_rows(X, p, e, prob["moments"], dom) for e in EDGES])
