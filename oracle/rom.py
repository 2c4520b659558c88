"""Offline MDEIM training and online evaluation of the trimmed tensor.

Sec. 4.2 (reduced order modelling) and Alg. 5, for one level-set family with
one parameter t (d = 1):
  * the parameter box [lo, hi] is split into n_k equal clusters; the cluster
    of t is min(floor((t - lo)/w), n_k - 1), and t outside the box is an
    error (the surrogate is only trained inside it);
  * n_s Latin-hypercube samples per cluster (stratified: one sample per
    sub-interval, at an offset given by the supplied U[0,1) draws);
  * exact snapshots I(t_s) (trimmed.py), a thin SVD of the snapshot matrix,
    and the first n_r left singular vectors as U_r.  The paper uses a
    randomized SVD truncated to n_v > n_r; a deterministic thin SVD gives the
    same leading vectors without the randomness.  Columns are signed so that
    their largest-magnitude entry is positive; n_r is cut to the numerical
    rank (sigma_j / sigma_1 > 1e-13) and the cut is reported;
  * magic points: the printed Alg. 3 projects U_j on the span of earlier
    orthonormal columns, which is identically zero, so we read it as the
    standard DEIM greedy of Chaturantabut and Sorensen (cited there): the
    residual of interpolating U_j at the earlier points, argmax |.|, lowest
    index on ties;
  * MDEIM coefficients I_r(t) solve (P^T U_r) I_r = P^T I(t) at r+1 GLL
    points of the cluster interval (tensor GLL fitting grid, d = 1), and the
    online surrogate is their degree-r Lagrange interpolant.
"""
import numpy as np
from .basis import gll_nodes, lagrange, lagrange_deriv
from .trimmed import I_exact, I_square


def cluster_bounds(lo, hi, n_k):
    w = (hi - lo) / n_k
    return [(lo + k * w, lo + (k + 1) * w) for k in range(n_k)]


def find_cluster(t, lo, hi, n_k):
    """FindCluster of Alg. 5 for d = 1."""
    if not (lo <= t <= hi):
        raise ValueError(f"parameter {t} outside the trained box [{lo}, {hi}]")
    w = (hi - lo) / n_k
    return min(int(np.floor((t - lo) / w)), n_k - 1)


def lhs_samples(a, b, u):
    """Stratified Latin-hypercube samples in [a, b] for d = 1."""
    n = len(u)
    return a + (np.arange(n) + u) * (b - a) / n


def signed_svd(M):
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    for j in range(U.shape[1]):
        i = np.argmax(np.abs(U[:, j]))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U, s


def deim_points(U):
    """Magic points by the DEIM greedy (reading of Alg. 3)."""
    n, r = U.shape
    idx = [int(np.argmax(np.abs(U[:, 0])))]
    for j in range(1, r):
        P = np.array(idx)
        c = np.linalg.solve(U[P, :j], U[P, j])
        res = U[:, j] - U[:, :j] @ c
        idx.append(int(np.argmax(np.abs(res))))
    return np.array(idx, dtype=np.int64)


def train(family, p, q, lo, hi, n_k, n_s, n_r, r, lhs_u, exact=I_exact, rank_tol=1e-13):
    """Train the per-cluster ROMs of one family.  `lhs_u` [n_k, n_s] are the
    U[0,1) offsets of the LHS.  Returns a dict with the untrimmed tensor I_pi
    [n_i], and per cluster: U [n_i, n_r] (zero-padded when the numerical rank
    is lower), coeff [r+1, n_r] (I_r at the fitting nodes), magic [n_r],
    nodes [r+1], sigma, rank."""
    Ipi = I_square(p, q).ravel()
    clusters = []
    for k, (a, b) in enumerate(cluster_bounds(lo, hi, n_k)):
        ts = lhs_samples(a, b, lhs_u[k])
        snaps = np.stack([exact(family, p, q, t).ravel() for t in ts], axis=1)
        U, s = signed_svd(snaps)
        rank = int(np.sum(s / s[0] > rank_tol))
        nr = min(n_r, rank)
        Ur = U[:, :nr]
        magic = deim_points(Ur)
        PU = Ur[magic, :]
        nodes = a + (b - a) * gll_nodes(r)
        coeff = np.stack([np.linalg.solve(PU, exact(family, p, q, t).ravel()[magic]) for t in nodes])
        Upad = np.zeros((Ur.shape[0], n_r))
        Upad[:, :nr] = Ur
        cpad = np.zeros((r + 1, n_r))
        cpad[:, :nr] = coeff
        mpad = np.zeros(n_r, dtype=np.int64)
        mpad[:nr] = magic
        clusters.append(dict(a=a, b=b, U=Upad, coeff=cpad, magic=mpad, nodes=nodes,
                             sigma=s, rank=rank, n_used=nr, samples=ts))
    return dict(family=family, p=p, q=q, lo=lo, hi=hi, n_k=n_k, n_r=n_r, r=r,
                I_pi=Ipi, clusters=clusters)


def reduced_coordinates(rom, t):
    """I_r(t): cluster, Lagrange interpolation of the fitted coefficients
    (Alg. 5).  Returns (cluster index, I_r [n_r])."""
    k = find_cluster(t, rom["lo"], rom["hi"], rom["n_k"])
    c = rom["clusters"][k]
    tau = (t - c["a"]) / (c["b"] - c["a"])
    ell = lagrange(gll_nodes(rom["r"]), [tau])[:, 0]
    return k, ell @ c["coeff"]


def reduced_coordinates_dt(rom, t):
    """d I_r / dt from the derivative of the Lagrange interpolant."""
    k = find_cluster(t, rom["lo"], rom["hi"], rom["n_k"])
    c = rom["clusters"][k]
    h = c["b"] - c["a"]
    tau = (t - c["a"]) / h
    dell = lagrange_deriv(gll_nodes(rom["r"]), [tau])[:, 0] / h
    return k, dell @ c["coeff"]


def reconstruct(rom, t):
    """I(t) ~ U_r I_r(t) (Alg. 5)."""
    k, Ir = reduced_coordinates(rom, t)
    return rom["clusters"][k]["U"] @ Ir


def stabilised_reduced(rom, t, rho):
    """The (n_r + 1)-vector [(1 - rho) I_r(t), rho] that multiplies
    [U_r | I_pi]: the stabilised tensor (1 - rho) I + rho I_pi of Alg. 4."""
    k, Ir = reduced_coordinates(rom, t)
    return k, np.concatenate([(1.0 - rho) * Ir, [rho]])


def offline_indicator(rom, family, n_test=50, seed=7, exact=I_exact):
    """Mean over fresh samples of the relative projection error
    ||I - U_r U_r^T I||_inf / ||I||_inf per cluster (Sec. 5, ROM accuracy
    indicator), plus the same for the full MDEIM surrogate."""
    rng = np.random.default_rng(seed)
    out = []
    for c in rom["clusters"]:
        ts = c["a"] + (c["b"] - c["a"]) * rng.random(n_test)
        proj, surr = [], []
        for t in ts:
            I = exact(family, rom["p"], rom["q"], t).ravel()
            nrm = np.abs(I).max()
            proj.append(np.abs(I - c["U"] @ (c["U"].T @ I)).max() / nrm)
            surr.append(np.abs(I - reconstruct(rom, t)).max() / nrm)
        out.append((float(np.mean(proj)), float(np.mean(surr))))
    return out
