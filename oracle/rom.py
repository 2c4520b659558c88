"""Offline MDEIM training and online evaluation of the trimmed tensor.

Sec. 4.2 (reduced order modelling) and Alg. 5, for one level-set family
whose cells carry d parameters: d = 1 (one thickness t per cell, the
stand-in families) or d = 4 (the corner thresholds mu_1..mu_4 of the
bilinear threshold function, Sec. 2.1.2, for the level sets of Table 1):
  * every parameter range [lo, hi] is split into n_k equal intervals, so the
    parameter box holds n_k^d clusters (Sec. 4.2.1); the cluster of a
    parameter vector takes, per coordinate, min(floor((x_i - lo)/w), n_k - 1),
    numbered with the first coordinate fastest; a parameter outside the box
    is an error (the surrogate is only trained inside it);
  * n_s Latin-hypercube samples per cluster: per coordinate one sample per
    sub-interval, at offsets given by the supplied U[0,1) draws, the strata
    of coordinate i visited in the order of a supplied permutation (d = 1:
    the identity);
  * exact snapshots I(x_s) (trimmed.py), a thin SVD of the snapshot matrix,
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
  * MDEIM coefficients I_r(x) solve (P^T U_r) I_r = P^T I(x) at the tensor
    grid of (r+1)^d GLL points of the cluster box (Sec. 4.2.3; 7^4 = 2401 for
    r = 6, d = 4), node (a_1, .., a_d) stored at a_1 + (r+1) a_2 + ..., and
    the online surrogate is their tensor-product Lagrange interpolant of
    degree r per coordinate.
"""
import numpy as np
from .basis import gll_nodes, lagrange, lagrange_deriv
from .trimmed import I_exact, I_square


def cluster_bounds(lo, hi, n_k):
    w = (hi - lo) / n_k
    return [(lo + k * w, lo + (k + 1) * w) for k in range(n_k)]


def find_cluster(t, lo, hi, n_k):
    """FindCluster of Alg. 5 for one coordinate."""
    if not (lo <= t <= hi):
        raise ValueError(f"parameter {t} outside the trained box [{lo}, {hi}]")
    w = (hi - lo) / n_k
    return min(int(np.floor((t - lo) / w)), n_k - 1)


def find_cluster_nd(x, lo, hi, n_k):
    """FindCluster of Alg. 5 for a parameter vector: the per-coordinate
    cluster indices combined with the first coordinate fastest."""
    k = 0
    for i in reversed(range(len(x))):
        k = k * n_k + find_cluster(float(x[i]), lo, hi, n_k)
    return k


def cluster_box(k, lo, hi, n_k, dim):
    """Per-coordinate intervals [(a_i, b_i)] of cluster k."""
    b = cluster_bounds(lo, hi, n_k)
    out = []
    for _ in range(dim):
        out.append(b[k % n_k])
        k //= n_k
    return out


def tensor_weights(vecs):
    """Products v_1[a_1] v_2[a_2] ... in the node order a_1 + (r+1) a_2 + ..."""
    w = np.ones(1)
    for v in vecs:
        w = np.outer(v, w).ravel()
    return w


def lhs_samples(a, b, u, perm=None):
    """Stratified Latin-hypercube samples of one coordinate in [a, b]: sample
    s lies in stratum perm[s] (the identity by default) at offset u[s]."""
    n = len(u)
    strata = np.arange(n) if perm is None else np.asarray(perm)
    return a + (strata + u) * (b - a) / n


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


def train(family, p, q, lo, hi, n_k, n_s, n_r, r, lhs_u, exact=I_exact, rank_tol=1e-13, dim=1, lhs_perm=None,
          only=None):
    """Train the per-cluster ROMs of one family.  `lhs_u` holds the U[0,1)
    offsets of the LHS, [n_k] x [n_s] for d = 1 and [n_k^d, n_s, d] for d > 1,
    with `lhs_perm` [n_k^d, d, n_s] the stratum order of each coordinate.
    Returns a dict with the untrimmed tensor I_pi [n_i], and per cluster: U
    [n_i, n_r] (zero-padded when the numerical rank is lower), coeff
    [(r+1)^d, n_r] (I_r at the fitting nodes), magic [n_r], nodes (the r+1
    GLL points of each coordinate interval), sigma, rank.  With `only` (a set
    of cluster indices) the other clusters are left untrained: zero U and
    coefficients, n_used 0 (a test that visits few of the n_k^d clusters
    trains just those)."""
    Ipi = I_square(p, q).ravel()
    clusters = []
    ncl = n_k ** dim
    g = gll_nodes(r)
    n_i = Ipi.size
    for k in range(ncl):
        box = cluster_box(k, lo, hi, n_k, dim)
        if only is not None and k not in only:
            cl = dict(a=box[0][0], b=box[0][1]) if dim == 1 else {}
            cl.update(U=np.zeros((n_i, n_r)), coeff=np.zeros(((r + 1) ** dim, n_r)),
                      magic=np.zeros(n_r, dtype=np.int64), nodes=None, box=box, sigma=None, rank=0, n_used=0,
                      samples=None, untrained=True)
            clusters.append(cl)
            continue
        if dim == 1:
            (a, b), = box
            samples = lhs_samples(a, b, lhs_u[k])
            fit = [a + (b - a) * g]
            pars = list(fit[0])
        else:
            samples = np.stack([lhs_samples(box[i][0], box[i][1], lhs_u[k][:, i], lhs_perm[k][i])
                                for i in range(dim)], axis=1)
            fit = [box[i][0] + (box[i][1] - box[i][0]) * g for i in range(dim)]
            # tensor grid, first coordinate fastest
            mesh = np.meshgrid(*fit, indexing="ij")
            pars = list(np.stack([m.transpose(tuple(reversed(range(dim)))).ravel() for m in mesh], axis=1))
        snaps = np.stack([exact(family, p, q, x).ravel() for x in samples], axis=1)
        U, s = signed_svd(snaps)
        rank = int(np.sum(s / s[0] > rank_tol))
        nr = min(n_r, rank)
        Ur = U[:, :nr]
        magic = deim_points(Ur)
        PU = Ur[magic, :]
        coeff = np.stack([np.linalg.solve(PU, exact(family, p, q, x).ravel()[magic]) for x in pars])
        Upad = np.zeros((Ur.shape[0], n_r))
        Upad[:, :nr] = Ur
        cpad = np.zeros((coeff.shape[0], n_r))
        cpad[:, :nr] = coeff
        mpad = np.zeros(n_r, dtype=np.int64)
        mpad[:nr] = magic
        cl = dict(a=box[0][0], b=box[0][1]) if dim == 1 else {}
        cl.update(U=Upad, coeff=cpad, magic=mpad, nodes=fit[0] if dim == 1 else fit,
                  box=box, sigma=s, rank=rank, n_used=nr, samples=samples)
        clusters.append(cl)
    return dict(family=family, p=p, q=q, lo=lo, hi=hi, n_k=n_k, n_r=n_r, r=r, dim=dim,
                I_pi=Ipi, clusters=clusters)


def _dim(rom):
    return rom.get("dim", 1)


def reduced_coordinates(rom, t):
    """I_r(x): cluster, Lagrange interpolation of the fitted coefficients
    (Alg. 5).  `t` is the parameter (d = 1) or the parameter vector.
    Returns (cluster index, I_r [n_r])."""
    if _dim(rom) == 1:
        k = find_cluster(t, rom["lo"], rom["hi"], rom["n_k"])
        c = rom["clusters"][k]
        tau = (t - c["a"]) / (c["b"] - c["a"])
        ell = lagrange(gll_nodes(rom["r"]), [tau])[:, 0]
        return k, ell @ c["coeff"]
    x = np.asarray(t, dtype=np.float64)
    k = find_cluster_nd(x, rom["lo"], rom["hi"], rom["n_k"])
    c = rom["clusters"][k]
    if c.get("untrained"):
        raise ValueError(f"cluster {k} of this ROM was not trained")
    g = gll_nodes(rom["r"])
    ells = [lagrange(g, [(x[i] - a) / (b - a)])[:, 0] for i, (a, b) in enumerate(c["box"])]
    return k, tensor_weights(ells) @ c["coeff"]


def reduced_coordinates_dt(rom, t):
    """d I_r / dt from the derivative of the Lagrange interpolant (d = 1);
    for d > 1 the rows d I_r / d x_i, [d, n_r]."""
    if _dim(rom) == 1:
        k = find_cluster(t, rom["lo"], rom["hi"], rom["n_k"])
        c = rom["clusters"][k]
        h = c["b"] - c["a"]
        tau = (t - c["a"]) / h
        dell = lagrange_deriv(gll_nodes(rom["r"]), [tau])[:, 0] / h
        return k, dell @ c["coeff"]
    x = np.asarray(t, dtype=np.float64)
    k = find_cluster_nd(x, rom["lo"], rom["hi"], rom["n_k"])
    c = rom["clusters"][k]
    g = gll_nodes(rom["r"])
    taus = [(x[i] - a) / (b - a) for i, (a, b) in enumerate(c["box"])]
    ells = [lagrange(g, [tau])[:, 0] for tau in taus]
    dells = [lagrange_deriv(g, [tau])[:, 0] / (b - a) for tau, (a, b) in zip(taus, c["box"])]
    rows = []
    for i in range(len(x)):
        vecs = [dells[j] if j == i else ells[j] for j in range(len(x))]
        rows.append(tensor_weights(vecs) @ c["coeff"])
    return k, np.stack(rows)


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
        if _dim(rom) == 1:
            ts = c["a"] + (c["b"] - c["a"]) * rng.random(n_test)
        else:
            ts = [np.array([a + (b - a) * rng.random() for (a, b) in c["box"]]) for _ in range(n_test)]
        proj, surr = [], []
        for t in ts:
            I = exact(family, rom["p"], rom["q"], t).ravel()
            nrm = np.abs(I).max()
            proj.append(np.abs(I - c["U"] @ (c["U"].T @ I)).max() / nrm)
            surr.append(np.abs(I - reconstruct(rom, t)).max() / nrm)
        out.append((float(np.mean(proj)), float(np.mean(surr))))
    return out
