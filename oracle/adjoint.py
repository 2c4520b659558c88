"""Compliance J = f^T u and its gradient.

Not in the paper beyond its remark that sensitivities follow directly; this
is the discrete adjoint of the method as implemented.  With K u = f
(assembled over free dofs), dJ = 2 u^T df - u^T dK u (the compliance is
self-adjoint, the adjoint state equals u, so no second solve is needed).
dK is a sum over cells of the derivative of the fast-assembly contraction:

  E_i = u_i^T K_i u_i = sum_{s} sum_{i1 i2} C_i[i1, i2, s] G_i[i1, i2, s],
  G_i[i1, i2, s] = sum_{k1 k2} u_i[i1, k1] u_i[i2, k2] Ieff_i[k1, k2, s],

so  dE/dt = u^T (Uhat dItil/dt) . C u   (ROM surrogate, Lagrange derivative)
and dE/dX = sum_s G . dC/dX with C = Chat(J(xi_k3)) (chain rule through the
pulled-back tensor and the Bernstein map).  The load depends on the
control points of the loaded edge through the curve Jacobian |dx/dxi|.
"""
import numpy as np
from .basis import bernstein, bernstein_deriv, gauss_legendre, gll_nodes, lagrange, interp_nodes
from .geometry import map_eval
from .rom import reduced_coordinates_dt
from .assembly import rom_Ieff, contract
from .bddc import edge_material_intervals, edge_map
from .dofs import edge_nodes_local


def chat_dJ(J, Cmat):
    """dChat[i1, j1, i2, j2] / dJ[p, q] at each point: [k, 2,2,2,2, 2,2]."""
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    A = np.linalg.inv(J)
    Ch = np.einsum("k,kam,imjn,kbn->kiajb", det, A, Cmat, A)
    T1 = np.einsum("kiajb,kqp->kiajbpq", Ch, A)
    T2 = -np.einsum("k,kap,kqm,imjn,kbn->kiajbpq", det, A, A, Cmat, A)
    T3 = -np.einsum("k,kam,imjn,kbp,kqn->kiajbpq", det, A, Cmat, A, A)
    return T1 + T2 + T3


def cell_G(Ieff, u_nat, nB):
    """G[i1, j1, i2, j2, k3] = sum_{k1 k2} u[i1,k1] u[i2,k2] Ieff[k1,k2,j1,j2,k3]."""
    U = u_nat.reshape(2, nB)
    return np.einsum("ia,jb,abxyk->ixjyk", U, U, Ieff)


def compliance_gradient(P, unodes, thresholds=False):
    """Compliance per load case and its gradient w.r.t. the control net and
    the thickness parameters, for an oracle Problem `P` (assembly 'rom') and
    displacements `unodes` [nrhs, Gy, Gx, 2] solving the system.  Returns
    (J [nrhs], dJ_dctrl [nrhs, *ctrl.shape], dJ_dt [nrhs, ncell]), and with
    `thresholds` also dJ_dmu [nrhs, ncell, 4], the gradient with respect to
    the corner thresholds of the cells of Table 1 level sets (zero rows for
    the other cells; their dJ_dt entries are zero)."""
    prob, d = P.prob, P.dofs
    p, q, m, rho = P.p, P.q, P.m, P.rho
    nB = d.nB
    nrhs = unodes.shape[0]
    Fg = P.global_f()
    J = np.zeros(nrhs)
    gX = np.zeros((nrhs,) + prob["ctrl"].shape)
    gt = np.zeros((nrhs, d.ncell))
    gmu = np.zeros((nrhs, d.ncell, 4))
    pts = interp_nodes(q)
    for r in range(nrhs):
        ufree = np.zeros(d.N)
        mask = d.free_id >= 0
        ufree[2 * d.free_id[mask]] = unodes[r][mask, 0]
        ufree[2 * d.free_id[mask] + 1] = unodes[r][mask, 1]
        J[r] = Fg[:, r] @ ufree
    for c, cell in enumerate(P.cells):
        ix, iy = d.cell_xy(c)
        fam, t = int(prob["family"][c]), P.cell_param(c)
        rom = P.roms[fam]
        X = cell.X
        _, Jp = map_eval(X, pts[:, 0], pts[:, 1])
        dCh = chat_dJ(Jp, P.Cmat)                       # [k3, i1 j1 i2 j2, p q]
        D1, D2 = bernstein_deriv(m, pts[:, 0]), bernstein_deriv(m, pts[:, 1])
        B1, B2 = bernstein(m, pts[:, 0]), bernstein(m, pts[:, 1])
        k_cl, Ieff = rom_Ieff(rom, t, rho)
        _, dIr = reduced_coordinates_dt(rom, t)
        Ut = rom["clusters"][k_cl]["U"]
        dIr = np.atleast_2d(dIr)                          # [d, n_r]
        dIeffs = [((1.0 - rho) * (Ut @ row)).reshape(Ieff.shape) for row in dIr]
        from .geometry import geometry_coefficients
        C, _ = geometry_coefficients(X, q, P.Cmat)
        for r in range(nrhs):
            u = P.cell_displacement(unodes[r], c)
            dE = [-u @ contract(dI, C) @ u for dI in dIeffs]
            if len(dE) == 1:
                gt[r, c] = dE[0]
            else:
                gmu[r, c, :] = dE
            G = cell_G(Ieff, u, nB)                      # [i1 j1 i2 j2 k3]
            # dE/dJ[p, q] at node k3
            dEdJ = np.einsum("iajbk,kiajbpq->kpq", G, dCh)
            for b in range(m + 1):
                for a in range(m + 1):
                    dN = np.stack([D1[a] * B2[b], B1[a] * D2[b]], axis=1)   # [k3, q]
                    gX[r, m * iy + b, m * ix + a, :] -= np.einsum("kpq,kq->p", dEdJ, dN)
            if c in P.load_pos:
                e = P.loaded
                trac = prob["traction"][r, P.load_pos[c]]
                dom = P.cell_domain(c)
                pieces = [(0.0, 1.0)] if dom is None else edge_material_intervals(dom, e)
                ue = np.array([[u[d.natural(a, b, comp)] for comp in range(2)]
                               for (a, b) in edge_nodes_local(p, e)])
                ut = ue @ trac                                # [p+1]
                xg, wg = gauss_legendre(p + 2 * m + 2)
                for a0, b0 in pieces:
                    xi, w = a0 + (b0 - a0) * xg, (b0 - a0) * wg
                    _, dx = edge_map(X, e, xi)
                    ds = np.sqrt(dx[:, 0] ** 2 + dx[:, 1] ** 2)
                    bn = lagrange(gll_nodes(p), xi)           # [p+1, nq]
                    dB = bernstein_deriv(m, xi)               # [m+1, nq]
                    # 2 u . df/dX for the control points (beta along the edge) of edge e
                    for beta in range(m + 1):
                        ja, jb = {"left": (0, beta), "right": (m, beta), "bottom": (beta, 0), "top": (beta, m)}[e]
                        for dd in range(2):
                            dds = dx[:, dd] / ds * dB[beta]
                            gX[r, m * iy + jb, m * ix + ja, dd] += 2.0 * ut @ (bn @ (w * dds))
                    # 2 u . df/dmu: the ends of the material part move with the
                    # thresholds (Leibniz rule), s* with phi(s*) = 0 moving by
                    # l_k(s*) / (d phi / d s)(s*) per unit of mu_k
                    if dom is not None:
                        # a break shared by two material intervals is the upper
                        # end of one and the lower end of the other: the two
                        # terms cancel, and are skipped
                        shared = {a for a, _ in pieces} & {b for _, b in pieces}
                        for s_end, sign in ((b0, 1.0), (a0, -1.0)):
                            if s_end <= 0.0 or s_end >= 1.0 or s_end in shared:
                                continue
                            gmu[r, c, :] += sign * 2.0 * _load_end_rate(dom, e, X, p, ut, s_end)
    if thresholds:
        return J, gX, gt, gmu
    return J, gX, gt


def _load_end_rate(dom, e, X, p, ut, s):
    """(sum_n ut_n b_n(s)) |x'(s)| ds/dmu_k at a root s of phi on edge e: the
    rate at which the traction's virtual work on the material part grows as
    the end s moves, per unit of each corner threshold."""
    x0, y0 = {"left": (0.0, s), "right": (1.0, s), "bottom": (s, 0.0), "top": (s, 1.0)}[e]
    gx, gy = dom.grad(np.array([x0]), np.array([y0]))
    dphi_ds = (gy if e in ("left", "right") else gx)[0]
    ell = np.array([(1 - x0) * (1 - y0), x0 * (1 - y0), (1 - x0) * y0, x0 * y0])
    _, dx = edge_map(X, e, np.array([s]))
    g = (ut @ lagrange(gll_nodes(p), np.array([s]))[:, 0]) * np.hypot(dx[0, 0], dx[0, 1])
    return g * ell / dphi_ds


def compliance_direct(prob, roms):
    """J per load case from a direct solve (used for finite differences)."""
    from .bddc import Problem
    P = Problem(prob, roms)
    u = P.direct_solve()
    F = P.global_f()
    d = P.dofs
    out = []
    mask = d.free_id >= 0
    for r in range(u.shape[0]):
        uf = np.zeros(d.N)
        uf[2 * d.free_id[mask]] = u[r][mask, 0]
        uf[2 * d.free_id[mask] + 1] = u[r][mask, 1]
        out.append(F[:, r] @ uf)
    return np.array(out)


def fd_directional(prob, roms, dX, dt, h=1e-6, dmu=None):
    """Central finite difference of J along (dX, dt) (and dmu, the
    per-cell corner thresholds, when given)."""
    pp = dict(prob)
    pm = dict(prob)
    pp["ctrl"] = prob["ctrl"] + h * dX
    pm["ctrl"] = prob["ctrl"] - h * dX
    pp["t"] = prob["t"] + h * dt
    pm["t"] = prob["t"] - h * dt
    if dmu is not None:
        pp["mu"] = prob["mu"] + h * dmu
        pm["mu"] = prob["mu"] - h * dmu
    return (compliance_direct(pp, roms) - compliance_direct(pm, roms)) / (2 * h)
