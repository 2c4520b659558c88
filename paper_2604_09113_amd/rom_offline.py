"""Offline stage of the method: train the MDEIM surrogate of a level-set family.

This is the one-time offline training of Sec. 4.2 (and the offline panel of
the workflow figure): snapshots of the trimmed-domain tensor at Latin-hypercube
samples, a truncated SVD, magic points, and the reduced coordinates at a GLL
grid of each cluster.  It runs on the host before any online work and is not
part of the online path the library accelerates; its output is the input of
lbddc_load_rom.

Both stand-in families are trimmed by circles or axis-aligned lines, so their
snapshots are integrated exactly (to rounding): the integrand is a polynomial
of total degree 4p - 2 + 2q (at most 2p + q per variable), integrated by Gauss
rules over rectangles and a polar Gauss x trapezoid rule over the disk.
The level sets of Table 1 with the bilinear threshold (Sec. 2.1.2) have four
parameters per cell and curved, implicitly given boundaries; their trainer
(train_implicit) runs the snapshot and fitting quadratures on the GPU through
lbddc_implicit_tensors (an implicit-domain quadrature after Saye's method),
with n_k clusters per threshold (n_k^4 in all), Latin-hypercube samples per
cluster and the (r+1)^4 tensor grid of GLL fitting nodes, first threshold
fastest.

Readings shared with the rest of the library: clusters split [lo, hi] evenly;
LHS takes one sample per stratum; columns of the SVD basis are signed so that
their largest entry is positive; the rank is cut where sigma_j / sigma_1 <=
1e-13; magic points follow the DEIM greedy (interpolation residual of each new
basis vector at the earlier points); the fitting grid is r+1 GLL points per
cluster.
"""
import numpy as np
from numpy.polynomial import legendre as npleg

CIRCLE, CROSS = 0, 1


def gll_nodes01(n):
    """n+1 Gauss-Lobatto points on [0, 1] (end points and the extrema of P_n)."""
    if n == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(n + 1)
    c[-1] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c))))
    d1, d2 = npleg.legder(c), npleg.legder(c, 2)
    for _ in range(3):
        inner -= npleg.legval(inner, d1) / npleg.legval(inner, d2)
    return 0.5 * (np.concatenate(([-1.0], inner, [1.0])) + 1.0)


def _bary(nodes):
    diff = nodes[:, None] - nodes[None, :]
    np.fill_diagonal(diff, 1.0)
    return 1.0 / diff.prod(axis=1)


def lagrange_eval(nodes, x):
    """Barycentric evaluation of all Lagrange polynomials: [len(nodes), len(x)]."""
    w = _bary(nodes)
    x = np.asarray(x, dtype=np.float64)
    d = x[None, :] - nodes[:, None]
    exact = np.isclose(d, 0.0, atol=1e-15)
    d[exact] = 1.0
    t = w[:, None] / d
    out = t / t.sum(axis=0, keepdims=True)
    hit = exact.any(axis=0)
    if hit.any():
        out[:, hit] = exact[:, hit].astype(np.float64)
    return out


def diff_matrix(nodes):
    """D[k, j] = l_j'(x_k) from the barycentric weights."""
    w = _bary(nodes)
    n = len(nodes)
    D = np.zeros((n, n))
    for k in range(n):
        for j in range(n):
            if j != k:
                D[k, j] = (w[j] / w[k]) / (nodes[k] - nodes[j])
        D[k, k] = -D[k].sum()
    return D


def _gauss01(n, a=0.0, b=1.0):
    x, w = npleg.leggauss(n)
    return a + (b - a) * 0.5 * (x + 1.0), 0.5 * (b - a) * w


class _Integrator:
    def __init__(self, p, q):
        self.p, self.q = p, q
        self.nodes = gll_nodes01(p)
        self.D = diff_matrix(self.nodes)
        self.qnodes = gll_nodes01(q)
        self.n1 = p + (q + 1) // 2 + 2                     # Gauss points per direction
        self.deg = 4 * p - 2 + 2 * q                        # total degree of the integrand

    def tensor(self, xs, ys, ws):
        """sum_k w_k dB_{k1,j1} dB_{k2,j2} L_{k3} as [nB, nB, 2, 2, nL]."""
        p1, q1 = self.p + 1, self.q + 1
        Lx, Ly = lagrange_eval(self.nodes, xs), lagrange_eval(self.nodes, ys)
        dLx, dLy = self.D.T @ Lx, self.D.T @ Ly              # l_a'(x) = sum_k l_k(x) D[k, a]
        G = np.empty((p1 * p1, 2, len(xs)))
        G[:, 0, :] = (dLx[None, :, :] * Ly[:, None, :]).reshape(p1 * p1, -1)
        G[:, 1, :] = (Lx[None, :, :] * dLy[:, None, :]).reshape(p1 * p1, -1)
        Q = (lagrange_eval(self.qnodes, xs)[None, :, :] * lagrange_eval(self.qnodes, ys)[:, None, :]).reshape(q1 * q1, -1)
        A = G.reshape(p1 * p1 * 2, -1)
        out = np.empty((p1 * p1 * 2, p1 * p1 * 2, q1 * q1))
        for k3 in range(q1 * q1):
            out[:, :, k3] = (A * (ws * Q[k3])) @ A.T
        return out.reshape(p1 * p1, 2, p1 * p1, 2, q1 * q1).transpose(0, 2, 1, 3, 4)

    def rect(self, x0, x1, y0, y1):
        gx, wx = _gauss01(self.n1, x0, x1)
        gy, wy = _gauss01(self.n1, y0, y1)
        X, Y = np.meshgrid(gx, gy)
        return X.ravel(), Y.ravel(), np.outer(wy, wx).ravel()

    def disk(self, r):
        nr, nt = self.deg // 2 + 2, self.deg + 2
        rr, wr = _gauss01(nr, 0.0, r)
        th = np.arange(nt) * (2.0 * np.pi / nt)
        R, T = np.meshgrid(rr, th)
        W = np.outer(np.full(nt, 2.0 * np.pi / nt), wr * rr)
        return (0.5 + R * np.cos(T)).ravel(), (0.5 + R * np.sin(T)).ravel(), W.ravel()

    def regions(self, family, t):
        """Signed point sets whose weighted sum covers the material region."""
        if family == CIRCLE:
            x, y, w = self.rect(0.0, 1.0, 0.0, 1.0)
            dx, dy, dw = self.disk(0.5 - t)
            return np.concatenate([x, dx]), np.concatenate([y, dy]), np.concatenate([w, -dw])
        if family == CROSS:
            a, b = 0.5 - 0.5 * t, 0.5 + 0.5 * t
            parts = [self.rect(a, b, 0.0, 1.0), self.rect(0.0, 1.0, a, b), self.rect(a, b, a, b)]
            sign = [1.0, 1.0, -1.0]
            return (np.concatenate([pp[0] for pp in parts]), np.concatenate([pp[1] for pp in parts]),
                    np.concatenate([s * pp[2] for s, pp in zip(sign, parts)]))
        raise ValueError(f"unknown family {family}")

    def snapshot(self, family, t):
        return self.tensor(*self.regions(family, t)).ravel()

    def untrimmed(self):
        return self.tensor(*self.rect(0.0, 1.0, 0.0, 1.0)).ravel()


def _deim(U):
    pts = [int(np.argmax(np.abs(U[:, 0])))]
    for j in range(1, U.shape[1]):
        c = np.linalg.solve(U[pts, :j], U[pts, j])
        pts.append(int(np.argmax(np.abs(U[:, j] - U[:, :j] @ c))))
    return np.array(pts)


def train(family, p, q, lo, hi, n_k, n_s, n_r, r, lhs_u, rank_tol=1e-13, log=None):
    """Arrays for lbddc_load_rom: U [n_k, n_i, n_r'], coeff [n_k, r+1, n_r'],
    I_pi [n_i], with n_r' <= n_r the largest numerical rank over clusters."""
    integ = _Integrator(p, q)
    w = (hi - lo) / n_k
    bases, coefs, ranks = [], [], []
    for k in range(n_k):
        a, b = lo + k * w, lo + (k + 1) * w
        ts = a + (np.arange(n_s) + lhs_u[k]) * (b - a) / n_s
        snaps = np.stack([integ.snapshot(family, t) for t in ts], axis=1)
        U, s, _ = np.linalg.svd(snaps, full_matrices=False)
        big = np.argmax(np.abs(U), axis=0)
        U = U * np.sign(U[big, np.arange(U.shape[1])])
        rank = min(n_r, int(np.sum(s / s[0] > rank_tol)))
        Ur = U[:, :rank]
        mp = _deim(Ur)
        fit_t = a + (b - a) * gll_nodes01(r)
        coef = np.stack([np.linalg.solve(Ur[mp], integ.snapshot(family, t)[mp]) for t in fit_t])
        bases.append(Ur)
        coefs.append(coef)
        ranks.append(rank)
        if log:
            log(f"family {family} cluster {k}: rank {rank}, sigma ratio {s[rank - 1] / s[0]:.1e}")
    nr = max(ranks)
    n_i = bases[0].shape[0]
    U = np.zeros((n_k, n_i, nr))
    C = np.zeros((n_k, r + 1, nr))
    for k in range(n_k):
        U[k, :, :ranks[k]] = bases[k]
        C[k, :, :ranks[k]] = coefs[k]
    return dict(family=family, p=p, q=q, n_k=n_k, n_r=nr, r=r, lo=lo, hi=hi, U=U, coeff=C,
                I_pi=integ.untrimmed())


def _lhs(a, b, u, perm):
    """One coordinate of a Latin-hypercube sample set: stratum perm[s], offset u[s]."""
    return a + (np.asarray(perm) + u) * (b - a) / len(u)


def train_implicit(solver, family, p, q, lo, hi, n_k, n_s, n_r, r, lhs_u, lhs_perm, rank_tol=1e-13, only=None,
                   log=None):
    """ROM of a Table 1 level set with four corner thresholds per cell, its
    snapshots and fitting values integrated on the GPU (solver: an
    lbddc.Solver).  lhs_u [n_k^4, n_s, 4] offsets and lhs_perm [n_k^4, 4, n_s]
    stratum orders of the Latin-hypercube sampling; `only` restricts training
    to the listed clusters (the others keep zero arrays).  The snapshots of
    four clusters go to the GPU together, and the fitting nodes of all
    clusters in one call (each with its cluster's magic points).  Returns the
    arrays of lbddc_load_rom with dim = 4."""
    ncl = n_k ** 4
    w = (hi - lo) / n_k
    g = gll_nodes01(r)
    todo = [k for k in range(ncl) if only is None or k in only]
    boxes = {}
    for k in todo:
        c = [(k // n_k ** i) % n_k for i in range(4)]
        boxes[k] = [(lo + ci * w, lo + (ci + 1) * w) for ci in c]
    bases, ranks, mps = {}, {}, {}
    for c0 in range(0, len(todo), 4):
        group = todo[c0:c0 + 4]
        X = np.concatenate([np.stack([_lhs(boxes[k][i][0], boxes[k][i][1], lhs_u[k][:, i], lhs_perm[k][i])
                                      for i in range(4)], axis=1) for k in group])
        snaps_all = solver.implicit_tensors(family, p, q, X)
        for j, k in enumerate(group):
            snaps = snaps_all[j * n_s:(j + 1) * n_s].T
            U, s, _ = np.linalg.svd(snaps, full_matrices=False)
            big = np.argmax(np.abs(U), axis=0)
            U = U * np.sign(U[big, np.arange(U.shape[1])])
            rank = min(n_r, int(np.sum(s / s[0] > rank_tol)))
            bases[k] = U[:, :rank]
            ranks[k] = rank
            mps[k] = _deim(bases[k])
            if log:
                log(f"family {family} cluster {k}: rank {rank}, sigma ratio {s[rank - 1] / s[0]:.1e}")
        del snaps_all
    # fitting grids (first threshold fastest) and magic points of every cluster, one GPU call
    nr = max(ranks.values()) if ranks else 1
    nn = (r + 1) ** 4
    grids, ents = [], []
    for k in todo:
        f = [boxes[k][i][0] + (boxes[k][i][1] - boxes[k][i][0]) * g for i in range(4)]
        grids.append(np.array([[f[0][a], f[1][b], f[2][cc], f[3][d]]
                               for d in range(r + 1) for cc in range(r + 1) for b in range(r + 1) for a in range(r + 1)]))
        e = np.zeros(nr, dtype=np.int64)
        e[:ranks[k]] = mps[k]
        ents.append(np.repeat(e[None, :], nn, axis=0))
    vals = solver.implicit_tensors(family, p, q, np.concatenate(grids), entries=np.concatenate(ents))
    n_i = (p + 1) ** 4 * 4 * (q + 1) ** 2
    U = np.zeros((ncl, n_i, nr))
    C = np.zeros((ncl, nn, nr))
    for j, k in enumerate(todo):
        rk = ranks[k]
        v = vals[j * nn:(j + 1) * nn, :rk]
        U[k, :, :rk] = bases[k]
        C[k, :, :rk] = np.linalg.solve(bases[k][mps[k]], v.T).T
    return dict(family=family, p=p, q=q, n_k=n_k, n_r=nr, r=r, lo=lo, hi=hi, U=U, coeff=C,
                I_pi=_Integrator(p, q).untrimmed(), dim=4)
