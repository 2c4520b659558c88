"""BDDC on the cell skeleton with PCG (Sec. 3, Alg. 1-2).

Per cell (Sec. 3.2): Dirichlet condensation, local Schur complement
S = K_UU - K_UI K_II^-1 K_IU and condensed load f = f_U - K_UI K_II^-1 f_I
through a Cholesky factor of K_II (never inverted).  Global interface
problem S u = f with S = sum R^T S_i R never assembled.

Preconditioner (Sec. 3.3, Eq. of S_BDDC^-1, Alg. 1): partition-of-unity
weights D from the stiffness diagonals, local saddle-point solves of Alg. 2
for the fine correction, coarse basis Psi from local saddle problems with
unit coarse values, and an exact global coarse solve with
S_C = sum R_C^T Psi^T S Psi R_C (the printed S_C formula has a stray
transpose; this is the product the derivation gives).

Alg. 2 as printed removes the cross-point rows and columns, which is exact
when the prescribed corner values are zero (the fine correction).  For the
coarse basis a corner value is one, so its column of S and of C is moved to
the right-hand side before the removal, and the corner multipliers are read
back from the corner rows of the first block equation.

PCG: x0 = 0, stop when ||f - S x||_2 <= rtol ||f||_2 (recurrence residual).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import gll_nodes, lagrange, gauss_legendre, bernstein, bernstein_deriv
from .dofs import Dofs, EDGES, edge_nodes_local, side_cells
from .geometry import cell_control_points, material_tensor, min_det_jacobian
from .assembly import rom_K, fast_K
from .trimmed import param_dim


def edge_map(X, e, xi):
    """Physical points x(xi) and tangents x'(xi) along edge e of the cell map."""
    m = X.shape[0] - 1
    B, dB = bernstein(m, xi), bernstein_deriv(m, xi)
    if e == "left":
        P = X[:, 0, :]
    elif e == "right":
        P = X[:, m, :]
    elif e == "bottom":
        P = X[0, :, :]
    else:
        P = X[m, :, :]
    return B.T @ P, dB.T @ P


def edge_material_intervals(dom, e):
    """The material part {phi < 0} of edge e of a trimmed cell (Sec. 2.1.2),
    as intervals of the edge parameter in [0, 1]: breaks at the roots of phi
    along the edge, kept where phi at the interval midpoint is negative."""
    from .implicit import _face_roots
    k, face = (0, 0.0 if e == "left" else 1.0) if e in ("left", "right") else \
        (1, 0.0 if e == "bottom" else 1.0)
    br = sorted([0.0, 1.0] + _face_roots(dom, k, face, 0.0, 1.0))
    out = []
    for a, b in zip(br[:-1], br[1:]):
        if b <= a:
            continue
        s = np.array([0.5 * (a + b)])
        f = dom.f(np.array([face]), s) if k == 0 else dom.f(s, np.array([face]))
        if f[0] < 0.0:
            out.append((a, b))
    return out


def edge_constraint_rows(X, p, e, moments, dom=None):
    """Coarse-dof rows of edge e over its p+1 nodes x 2 components:
    averages  int_e u_c ds   and moment  int_e f . u ds  with
    f = (x2 - xbar2, xbar1 - x1), xbar = image of the edge midpoint
    (Sec. 3.3.1).  Arc length of the physical edge, Gauss-Legendre with
    2p+2 points.  For a trimmed cell (dom, a TrimmedCell) the domain of the
    edge is its material part, each of its intervals with its own 2p+2
    points.  Returns [nce, p+1, 2]."""
    if dom is None:
        pieces = [(0.0, 1.0)]
    else:
        pieces = edge_material_intervals(dom, e)
    xg, wg = gauss_legendre(2 * p + 2)
    xbar, _ = edge_map(X, e, np.array([0.5]))
    xbar = xbar[0]
    rows = np.zeros((3 if moments else 2, p + 1, 2))
    for a, b in pieces:
        xi, w = a + (b - a) * xg, (b - a) * wg
        x, dx = edge_map(X, e, xi)
        ds = np.sqrt(dx[:, 0] ** 2 + dx[:, 1] ** 2)
        bl = lagrange(gll_nodes(p), xi)          # [p+1, nq]
        rows[0, :, 0] += bl @ (w * ds)
        rows[1, :, 1] += bl @ (w * ds)
        if moments:
            rows[2, :, 0] += bl @ (w * ds * (x[:, 1] - xbar[1]))
            rows[2, :, 1] += bl @ (w * ds * (xbar[0] - x[:, 0]))
    return rows


def traction_load(X, p, trac, e="right", dom=None):
    """Consistent load of a constant traction on edge e of the cell:
    f[node, comp] = int b_node(xi) t_comp |dx/dxi| dxi along the edge,
    nodes in increasing running coordinate, p+2m+2 Gauss points (Sec. 2.2.1,
    external virtual work on the Neumann part of the boundary; traction times
    the curve Jacobian).  The traction acts on the boundary of the material:
    for a trimmed cell (dom, a TrimmedCell) on the material part of the edge
    only, each of its intervals with its own rule; otherwise on the whole
    edge."""
    m = X.shape[0] - 1
    pieces = [(0.0, 1.0)] if dom is None else edge_material_intervals(dom, e)
    xg, wg = gauss_legendre(p + 2 * m + 2)
    f = np.zeros(p + 1)
    for a, b in pieces:
        xi, w = a + (b - a) * xg, (b - a) * wg
        _, dx = edge_map(X, e, xi)
        ds = np.sqrt(dx[:, 0] ** 2 + dx[:, 1] ** 2)
        f += lagrange(gll_nodes(p), xi) @ (w * ds)
    return np.outer(f, trac)  # [p+1, 2]


class Cell:
    pass


class Problem:
    """One lattice problem, built on the oracle's own DoF maps.

    assembly: 'rom' (MDEIM surrogate, the method), 'fast' (exact trimmed
    tensor) or 'full' (full quadrature reference).  The clamped sides
    (prob["clamped"], default the left side) carry homogeneous Dirichlet
    conditions on both components, the loaded side (prob["loaded"], default
    the right side) carries prob["traction"][r, k] on its k-th cell edge, and
    the other sides are traction free (Sec. 2.2.1)."""

    def __init__(self, prob, roms=None, assembly="rom", moments=None):
        self.prob = prob
        self.p, self.q, self.m = prob["p"], prob["q"], prob["m"]
        self.nx, self.ny = prob["nx"], prob["ny"]
        self.rho = prob["rho"]
        self.moments = prob["moments"] if moments is None else moments
        self.clamped = tuple(prob.get("clamped", ("left",)))
        self.loaded = prob.get("loaded", "right")
        if self.loaded in self.clamped:
            raise ValueError("the loaded side is clamped")
        self.dofs = Dofs(self.nx, self.ny, self.p, self.moments, self.clamped)
        self.load_pos = {c: k for c, k in side_cells(self.nx, self.ny, self.loaded)}
        self.Cmat = material_tensor(prob["E"], prob["nu"])
        self.roms = roms
        self.assembly = assembly
        self.nrhs = prob["traction"].shape[0]
        self.cells = []
        for c in range(self.dofs.ncell):
            self.cells.append(self._build_cell(c))

    def control_points(self, c):
        ix, iy = self.dofs.cell_xy(c)
        return cell_control_points(self.prob["ctrl"], self.m, ix, iy)

    def cell_param(self, c):
        """The geometric parameter of cell c: its thickness t, or for a
        Table 1 level set its corner thresholds mu[4] (Sec. 2.1.2)."""
        fam = int(self.prob["family"][c])
        if param_dim(fam) == 4:
            return np.asarray(self.prob["mu"][c], dtype=np.float64)
        return float(self.prob["t"][c])

    def cell_domain(self, c):
        """The trimmed cell {phi_0 < mu} of a Table 1 level set (its edges'
        material parts carry the edge constraints and the traction), or None
        for the one-parameter families (whole edges)."""
        fam = int(self.prob["family"][c])
        if param_dim(fam) == 4:
            from .implicit import TrimmedCell
            return TrimmedCell(fam, self.cell_param(c))
        return None

    def cell_K(self, c):
        X = self.control_points(c)
        fam, t = int(self.prob["family"][c]), self.cell_param(c)
        if self.assembly == "rom":
            return rom_K(X, self.roms[fam], t, self.rho, self.Cmat)
        if self.assembly == "fast":
            return fast_K(X, fam, t, self.rho, self.p, self.q, self.Cmat)
        from .assembly import full_K
        return full_K(X, fam, t, self.rho, self.p, self.q, self.Cmat)

    def _build_cell(self, c):
        d = self.dofs
        p = self.p
        cell = Cell()
        cell.X = self.control_points(c)
        if min_det_jacobian(cell.X) <= 0:
            raise ValueError(f"degenerate map in cell {c}")
        skel_nat, skel_glob, in_nat, cg, free = d.cell_maps(c)
        act = skel_glob >= 0
        cell.slot_active = act
        cell.U_nat = skel_nat[act]
        cell.U_glob = skel_glob[act]
        cell.I_nat = in_nat
        cell.free = free
        cell.K = self.cell_K(c)
        # loads (natural order, nrhs columns): traction on the loaded side
        f = np.zeros((2 * d.nB, self.nrhs))
        if c in self.load_pos:
            k = self.load_pos[c]
            for r in range(self.nrhs):
                fe = traction_load(cell.X, p, self.prob["traction"][r, k], self.loaded, self.cell_domain(c))
                for n, (a, b) in enumerate(edge_nodes_local(p, self.loaded)):
                    for comp in range(2):
                        f[d.natural(a, b, comp), r] += fe[n, comp]
        cell.f = f
        # constraints in canonical coarse order, over active skeleton dofs
        nce = d.nce
        nC_slots = 8 + 4 * nce
        slot_of_nat = {int(n): j for j, n in enumerate(skel_nat)}
        Cfull = np.zeros((nC_slots, len(skel_nat)))
        corners = [(0, 0), (p, 0), (0, p), (p, p)]
        for k, (a, b) in enumerate(corners):
            for comp in range(2):
                Cfull[2 * k + comp, slot_of_nat[d.natural(a, b, comp)]] = 1.0
        dom = self.cell_domain(c)
        for ei, e in enumerate(EDGES):
            rows = edge_constraint_rows(cell.X, p, e, self.moments, dom)
            for n, (a, b) in enumerate(edge_nodes_local(p, e)):
                for comp in range(2):
                    Cfull[8 + nce * ei:8 + nce * (ei + 1), slot_of_nat[d.natural(a, b, comp)]] = rows[:, n, comp]
        cact = cg >= 0
        cell.coarse_active = cact
        cell.C = Cfull[cact][:, act]
        cell.C_glob = cg[cact]
        # corner dofs among active skeleton dofs / corner rows among coarse rows
        cell.corner_pos = np.array([int(np.sum(act[:j])) for j in range(8) if act[j]])
        cell.edge_pos = np.setdiff1d(np.arange(len(cell.U_glob)), cell.corner_pos)
        cell.crow = np.array([int(np.sum(cact[:j])) for j in range(8) if cact[j]])
        cell.erow = np.setdiff1d(np.arange(len(cell.C_glob)), cell.crow)
        # Schur complement via Cholesky of K_II (Sec. 3.2)
        K = cell.K
        KII = K[np.ix_(in_nat, in_nat)]
        KIU = K[np.ix_(in_nat, cell.U_nat)]
        KUU = K[np.ix_(cell.U_nat, cell.U_nat)]
        cell.KII_f = sla.cho_factor(KII, lower=True)
        cell.KIU = KIU
        cell.S = KUU - KIU.T @ sla.cho_solve(cell.KII_f, KIU)
        fI, fU = f[in_nat], f[cell.U_nat]
        cell.fS = fU - KIU.T @ sla.cho_solve(cell.KII_f, fI)
        return cell

    # ---- global interface operator -------------------------------------------------
    def apply_S(self, v):
        w = np.zeros_like(v)
        for cell in self.cells:
            w[cell.U_glob] += cell.S @ v[cell.U_glob]
        return w

    def rhs(self):
        f = np.zeros((self.dofs.N_U, self.nrhs))
        for cell in self.cells:
            f[cell.U_glob] += cell.fS
        return f

    # ---- preconditioner setup ---------------------------------------------------------
    def setup(self):
        d = self.dofs
        Ktot = np.zeros(d.N_U)
        for cell in self.cells:
            Ktot[cell.U_glob] += np.diag(cell.K)[cell.U_nat]
        rows, cols, vals = [], [], []
        for cell in self.cells:
            cell.D = np.diag(cell.K)[cell.U_nat] / Ktot[cell.U_glob]
            nC = len(cell.C_glob)
            Psi = np.zeros((len(cell.U_glob), nC))
            Lam = np.zeros((nC, nC))
            for j in range(nC):
                g = np.zeros(nC)
                g[j] = 1.0
                Psi[:, j], Lam[:, j] = self.local_solve(cell, np.zeros(len(cell.U_glob)), g)
            cell.Psi, cell.Lam = Psi, Lam
            cell.SC = Psi.T @ cell.S @ Psi
            gi = cell.C_glob
            rows.append(np.repeat(gi, nC))
            cols.append(np.tile(gi, nC))
            vals.append(cell.SC.ravel())
        self.SC = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(d.N_C, d.N_C))
        self.SC_lu = spla.splu(self.SC)

    def local_solve(self, cell, f, g):
        """Alg. 2 for [S C^T; C 0][x; lam] = [f; g] (steps 3-9), with the
        prescribed corner values moved to the right-hand side."""
        cp, ep, cr, er = cell.corner_pos, cell.edge_pos, cell.crow, cell.erow
        S, C = cell.S, cell.C
        xc = g[cr]                                   # corner picks fix corner values
        Sh = S[np.ix_(ep, ep)]
        Ch = C[np.ix_(er, ep)]
        fh = f[ep] - S[np.ix_(ep, cp)] @ xc          # step 3 with corners moved right
        gh = g[er] - C[np.ix_(er, cp)] @ xc
        Lf = sla.cho_factor(Sh, lower=True)
        X = sla.cho_solve(Lf, Ch.T)                  # step 4
        T = Ch @ X
        rh = Ch @ sla.cho_solve(Lf, fh) - gh          # step 5
        lamh = sla.cho_solve(sla.cho_factor(T, lower=True), rh)   # step 6
        hh = fh - Ch.T @ lamh                        # step 7
        xh = sla.cho_solve(Lf, hh)                   # step 8
        x = np.zeros(len(f))
        x[cp], x[ep] = xc, xh                        # step 9: undo the removal
        lam = np.zeros(len(g))
        lam[er] = lamh
        lam[cr] = (f - S @ x - C[er].T @ lamh)[cp]
        return x, lam

    def apply_M(self, v):
        """Alg. 1: S_BDDC^-1 v."""
        d = self.dofs
        w = np.zeros(d.N_U)
        z = np.zeros(d.N_C)
        for cell in self.cells:
            vi = cell.D * v[cell.U_glob]
            x, _ = self.local_solve(cell, vi, np.zeros(len(cell.C_glob)))
            w[cell.U_glob] += cell.D * x
            z[cell.C_glob] += cell.Psi.T @ vi
        g = self.SC_lu.solve(z)
        for cell in self.cells:
            w[cell.U_glob] += cell.D * (cell.Psi @ g[cell.C_glob])
        return w

    def pcg(self, f, rtol=1e-8, max_iter=1000, iters=None):
        """Preconditioned CG on S u = f from x0 = 0.  With `iters`, run exactly
        that many iterations (fixed-count parity diagnostic)."""
        x = np.zeros_like(f)
        r = f.copy()
        nf = np.linalg.norm(f)
        z = self.apply_M(r)
        pd = z.copy()
        rz = r @ z
        hist = [1.0]
        it = 0
        while True:
            if iters is None and (hist[-1] <= rtol or it >= max_iter):
                break
            if iters is not None and it >= iters:
                break
            q = self.apply_S(pd)
            alpha = rz / (pd @ q)
            x += alpha * pd
            r -= alpha * q
            it += 1
            hist.append(np.linalg.norm(r) / nf)
            if iters is None and hist[-1] <= rtol:
                break
            z = self.apply_M(r)
            rz_new = r @ z
            pd = z + (rz_new / rz) * pd
            rz = rz_new
        return x, it, np.array(hist)

    def recover(self, uU, rhs_index=0):
        """Interior recovery u_I = K_II^-1 (f_I - K_IU u) per cell; returns the
        full displacement on the node lattice [Gy, Gx, 2] (Dirichlet = 0)."""
        d = self.dofs
        p = self.p
        out = np.zeros((d.Gy, d.Gx, 2))
        for c, cell in enumerate(self.cells):
            ui = np.zeros(2 * d.nB)
            ui[cell.U_nat] = uU[cell.U_glob]
            fI = cell.f[cell.I_nat, rhs_index]
            ui[cell.I_nat] = sla.cho_solve(cell.KII_f, fI - cell.KIU @ uU[cell.U_glob])
            ix, iy = d.cell_xy(c)
            for b in range(p + 1):
                for a in range(p + 1):
                    if d.node_dirichlet[p * iy + b, p * ix + a]:
                        continue
                    out[p * iy + b, p * ix + a, 0] = ui[d.natural(a, b, 0)]
                    out[p * iy + b, p * ix + a, 1] = ui[d.natural(a, b, 1)]
        return out

    def cell_displacement(self, unodes, c):
        """Natural-order local displacement of cell c from the node lattice."""
        d = self.dofs
        p = self.p
        ix, iy = d.cell_xy(c)
        u = np.zeros(2 * d.nB)
        for b in range(p + 1):
            for a in range(p + 1):
                for comp in range(2):
                    u[d.natural(a, b, comp)] = unodes[p * iy + b, p * ix + a, comp]
        return u

    # ---- direct reference (Eq. of the full 2x2 block system) -------------------------
    def global_K(self):
        d = self.dofs
        rows, cols, vals = [], [], []
        for cell in self.cells:
            idx = np.where(cell.free >= 0)[0]
            g = cell.free[idx]
            Kc = cell.K[np.ix_(idx, idx)]
            rows.append(np.repeat(g, len(g)))
            cols.append(np.tile(g, len(g)))
            vals.append(Kc.ravel())
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(d.N, d.N))

    def global_f(self):
        d = self.dofs
        f = np.zeros((d.N, self.nrhs))
        for cell in self.cells:
            idx = np.where(cell.free >= 0)[0]
            f[cell.free[idx]] += cell.f[idx]
        return f

    def direct_solve(self):
        """Sparse direct solve of the assembled system over all free dofs;
        returns u on the node lattice [nrhs, Gy, Gx, 2]."""
        d = self.dofs
        K = self.global_K()
        F = self.global_f()
        U = spla.splu(K).solve(F)
        out = np.zeros((self.nrhs, d.Gy, d.Gx, 2))
        fid = d.free_id
        mask = fid >= 0
        for r in range(self.nrhs):
            out[r, mask, 0] = U[2 * fid[mask], r]
            out[r, mask, 1] = U[2 * fid[mask] + 1, r]
        return out

    def skeleton_from_nodes(self, unodes):
        d = self.dofs
        u = np.zeros(d.N_U)
        m = d.skel_id >= 0
        u[2 * d.skel_id[m]] = unodes[m, 0]
        u[2 * d.skel_id[m] + 1] = unodes[m, 1]
        return u

    def solve(self, rtol=None, max_iter=1000):
        """BDDC-PCG for every load case, then interior recovery.  Returns
        (u [nrhs, Gy, Gx, 2], iterations [nrhs], histories)."""
        rtol = self.prob["rtol"] if rtol is None else rtol
        F = self.rhs()
        us, its, hs = [], [], []
        for r in range(self.nrhs):
            uU, it, h = self.pcg(F[:, r], rtol, max_iter)
            us.append(self.recover(uU, r))
            its.append(it)
            hs.append(h)
        return np.stack(us), its, hs
