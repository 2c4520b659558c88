"""The five lattice workloads and a generator for small variants.

Each problem is a plain dict of numpy arrays and scalars:

  nx, ny       cells along x and y (cell (ix, iy) has index iy*nx + ix)
  p, q         GLL degree of the cell element and of the coefficient
               interpolation used by the fast assembly
  m            Bernstein order of the map; the shared control net has
               (m*ny+1) x (m*nx+1) points, ctrl[jy, jx] = (x, y)
  ctrl         float64 [(m*ny+1), (m*nx+1), 2]
  family       int32 [ncell] level-set family per cell (0 circle, 1 cross,
               2-5 the level sets of Table 1: Schwarz Diamond, Schwarz
               Primitive, Schoen FRD, Schoen IWP)
  t            float64 [ncell] thickness parameter per cell (circle, cross)
  mu           float64 [ncell, 4] corner thresholds of each cell (bottom-left,
               bottom-right, top-left, top-right) taken from one value per
               lattice vertex, so neighbouring cells share them (trimmed
               compatibility); zeros when no cell uses a Table 1 level set
  E, nu, rho   material (plane strain) and stabilisation factor
  traction     float64 [nrhs, n_side, 2] constant traction on the edge of
               each cell along the loaded side (physical units); n_side = ny
               for the left and right sides, nx for the bottom and top
  clamped      tuple of clamped sides ("left", "right", "bottom", "top")
  loaded       the loaded side
  moments      whether edge-moment coarse dofs are used
  rtol         PCG relative residual tolerance
  rom          {family: dict(lo, hi, n_k, n_s, n_r, r)} ROM settings

By default the left side x = 0 is clamped and the right side carries the
traction; the other outer sides are traction free.  The `clamped` and
`loaded` overrides select other sides.
"""
import numpy as np

FAMILY_NAMES = {0: "circle", 1: "cross", 2: "schwarz_d", 3: "schwarz_p", 4: "schoen_frd", 5: "schoen_iwp"}
TPMS_TOPOLOGY = {"schwarz_d": 2, "schwarz_p": 3, "schoen_frd": 4, "schoen_iwp": 5}
# first threshold box of each Table 1 level set (Sec. 5.1.2)
TPMS_BOX = {2: (0.1, 0.9), 3: (-0.5, 0.8), 4: (-6.5, 0.5), 5: (-2.5, 2.5)}


def family_name(f):
    return FAMILY_NAMES[int(f)]


CONFIGS = {
    # plain FP64 method, tiny: affine (identity) map, circle holes r~U[0.2,0.4]
    1: dict(nx=4, ny=4, p=3, q=2, m=1, jitter=0.0, warp=0.0, topo="circle",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=0.0, moments=False,
            rtol=1e-8, nrhs=1, load="unit",
            rom={0: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=20, r=6)}),
    # plain FP64 at scale: order-2 jittered map, hole radius graded in x
    2: dict(nx=64, ny=64, p=6, q=2, m=2, jitter=0.03, warp=0.0, topo="circle",
            t_mode="graded", t_lo=0.08, t_hi=0.37, rho=5e-4, moments=True,
            rtol=1e-10, nrhs=1, load="unit",
            rom={0: dict(lo=0.05, hi=0.40, n_k=2, n_s=300, n_r=40, r=6)}),
    # the measured workload: 128x128 p=8, mixed circle/cross topologies
    3: dict(nx=128, ny=128, p=8, q=2, m=2, jitter=0.03, warp=0.0, topo="mixed",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=5e-4, moments=True,
            rtol=1e-8, nrhs=1, load="unit",
            rom={0: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=40, r=6),
                 1: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=40, r=6)}),
    # differentiation: order-3 map, circle, t~U[0.1,0.3]
    4: dict(nx=64, ny=64, p=6, q=2, m=3, jitter=0.02, warp=0.0, topo="circle",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=5e-4, moments=True,
            rtol=1e-13, nrhs=1, load="unit",
            rom={0: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=40, r=6)}),
    # large multi-RHS: order-3 sinusoidal warp, two topologies, 8 loads
    5: dict(nx=256, ny=256, p=8, q=2, m=3, jitter=0.0, warp=0.05, topo="mixed",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=5e-4, moments=True,
            rtol=1e-8, nrhs=8, load="random",
            rom={0: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=40, r=6),
                 1: dict(lo=0.1, hi=0.3, n_k=2, n_s=100, n_r=40, r=6)}),
    # the paper's own cells: a Schwarz Diamond lattice with the bilinear
    # threshold (d = 4), graded across the lattice like the paper's benchmark
    # (mu = 0.9 - 0.8 x / L at the vertices) plus U[-0.05, 0.05], clipped to
    # the box [0.1, 0.9]; 2 clusters per threshold (16), r = 6 (7^4 nodes).
    # rho = 2e-3: with n_r = 40 the surrogate's error (up to ~4e-4 of |I| with
    # 100 snapshots per cluster) outweighs rho = 5e-4 on these jittered cells
    # with noisy thresholds and leaves the coarse matrix or the interface
    # operator indefinite (also with 200 snapshots)
    6: dict(nx=128, ny=128, p=8, q=2, m=2, jitter=0.03, warp=0.0, topo="schwarz_d",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=2e-3, moments=True,
            rtol=1e-8, nrhs=1, load="unit", mu_mode="graded", mu_noise=0.05,
            rom={2: dict(lo=0.1, hi=0.9, n_k=2, n_s=100, n_r=40, r=6, dim=4)}),
    # the paper's benchmark geometry (Sec. 5.2): a quarter annulus r in
    # [0.6, 1] of 184 x 92 = 16,928 cells (twice as many along xi~_1), Schwarz
    # Diamond cells with mu = 0.9 - 0.8 xi~_1 at the vertices, E = 5, nu = 0.25,
    # xi~_1 = 0 clamped and a traction of 0.1 pointing down (-y) on xi~_1 = 1;
    # the map of every cell is an order-3 Bezier patch whose control points lie
    # on the (mirrored) annulus at the uniform grid of the auxiliary coordinates;
    # the paper's rho = 5e-4, which 200 Latin-hypercube snapshots per cluster
    # keep positive definite (100 do not)
    7: dict(nx=184, ny=92, p=8, q=2, m=3, jitter=0.0, warp=0.0, topo="schwarz_d", map="annulus",
            t_mode="uniform", t_lo=0.1, t_hi=0.3, rho=5e-4, moments=True, E=5.0, nu=0.25,
            rtol=1e-8, nrhs=1, load="down", load_value=0.1, mu_mode="graded", mu_noise=0.0,
            rom={2: dict(lo=0.1, hi=0.9, n_k=2, n_s=200, n_r=40, r=6, dim=4)}),
}


def _uniform_net(nx, ny, m):
    gx = np.arange(m * nx + 1, dtype=np.float64) / m
    gy = np.arange(m * ny + 1, dtype=np.float64) / m
    net = np.zeros((m * ny + 1, m * nx + 1, 2))
    net[:, :, 0] = gx[None, :]
    net[:, :, 1] = gy[:, None]
    return net


def make_problem(config=1, seed=None, **overrides):
    """Build the seeded inputs of workload `config` (1..5).

    `overrides` replace entries of the config table (e.g. nx=8, ny=4, p=4)
    so tests can draw smaller lattices with the same recipe.  The seed
    defaults to the config number.
    """
    cfg = dict(CONFIGS[config])
    cfg["rom"] = {k: dict(v) for k, v in cfg["rom"].items()}
    cfg.update(overrides)
    if seed is None:
        seed = config
    rng = np.random.default_rng(seed)
    nx, ny, m = cfg["nx"], cfg["ny"], cfg["m"]
    net = _uniform_net(nx, ny, m)
    if cfg.get("map") == "annulus":
        # the quarter annulus r = 0.6 + 0.4 u, angle pi/2 s at the net's uniform
        # auxiliary coordinates s = jx / (m nx), u = jy / (m ny), mirrored in x
        # (x = -r sin(pi/2 s), y = -r cos(pi/2 s)): the paper's orientation has
        # det J < 0, and the library takes positively oriented maps
        s_ = net[:, :, 0] / nx
        u_ = net[:, :, 1] / ny
        rad = 0.6 + 0.4 * u_
        net = np.stack([-rad * np.sin(0.5 * np.pi * s_), -rad * np.cos(0.5 * np.pi * s_)], axis=2)
    interior = np.zeros(net.shape[:2], dtype=bool)
    interior[1:-1, 1:-1] = True
    jit = rng.normal(0.0, 1.0, size=net.shape)
    if cfg["jitter"] > 0:
        net = net + cfg["jitter"] * jit * interior[:, :, None]
    if cfg["warp"] > 0:
        gxy = _uniform_net(nx, ny, m)
        wx = np.sin(2 * np.pi * gxy[:, :, 1] / ny)
        wy = np.sin(2 * np.pi * gxy[:, :, 0] / nx)
        net[:, :, 0] += cfg["warp"] * wx * interior
        net[:, :, 1] += cfg["warp"] * wy * interior
    ncell = nx * ny
    coin = rng.random(ncell)
    if cfg["topo"] == "circle":
        family = np.zeros(ncell, dtype=np.int32)
    elif cfg["topo"] == "cross":
        family = np.ones(ncell, dtype=np.int32)
    elif cfg["topo"] in TPMS_TOPOLOGY:
        family = np.full(ncell, TPMS_TOPOLOGY[cfg["topo"]], dtype=np.int32)
    else:
        family = (coin < 0.5).astype(np.int32)
    u = rng.random(ncell)
    if cfg["t_mode"] == "graded":
        # hole radius r = 0.15 + 0.25 * xc / nx + U[-0.02, 0.02], t = 1/2 - r
        ix = np.arange(ncell) % nx
        r = 0.15 + 0.25 * (ix + 0.5) / nx + (u * 0.04 - 0.02)
        t = 0.5 - r
    else:
        t = cfg["t_lo"] + (cfg["t_hi"] - cfg["t_lo"]) * u
    mu = np.zeros((ncell, 4))
    if cfg["topo"] in TPMS_TOPOLOGY:
        lo, hi = cfg.get("mu_box", TPMS_BOX[TPMS_TOPOLOGY[cfg["topo"]]])
        vx = np.arange(nx + 1)[None, :] / nx
        v = np.broadcast_to(hi - (hi - lo) * vx, (ny + 1, nx + 1)).copy()
        if cfg.get("mu_mode", "graded") == "uniform":
            v = lo + (hi - lo) * rng.random((ny + 1, nx + 1))
        else:
            noise = cfg.get("mu_noise", 0.05) * (hi - lo) / 0.8
            v += noise * (2.0 * rng.random((ny + 1, nx + 1)) - 1.0)
        v = np.clip(v, lo, hi)
        iy, ix = np.divmod(np.arange(ncell), nx)
        mu = np.stack([v[iy, ix], v[iy, ix + 1], v[iy + 1, ix], v[iy + 1, ix + 1]], axis=1)
    nrhs = cfg["nrhs"]
    clamped = tuple(cfg.get("clamped", ("left",)))
    loaded = cfg.get("loaded", "right")
    n_side = ny if loaded in ("left", "right") else nx
    if cfg["load"] == "down":
        traction = np.zeros((nrhs, n_side, 2))
        traction[:, :, 1] = -cfg.get("load_value", 1.0)
    elif cfg["load"] == "unit":
        # unit traction along the outward normal of the loaded side
        traction = np.zeros((nrhs, n_side, 2))
        normal = {"left": (-1.0, 0.0), "right": (1.0, 0.0), "bottom": (0.0, -1.0), "top": (0.0, 1.0)}[loaded]
        traction[:, :, :] = normal
    else:
        traction = rng.normal(0.0, 1.0, size=(nrhs, n_side, 2))
    present = sorted(set(int(f) for f in np.unique(family)))
    rom = {f: cfg["rom"][f] for f in cfg["rom"] if f in present or len(present) == 0}
    return dict(config=config, seed=seed, nx=nx, ny=ny, p=cfg["p"], q=cfg["q"],
                m=m, ctrl=np.ascontiguousarray(net), family=family,
                t=np.ascontiguousarray(t, dtype=np.float64), mu=np.ascontiguousarray(mu),
                E=cfg.get("E", 1.0), nu=cfg.get("nu", 0.3),
                rho=cfg["rho"], moments=cfg["moments"], rtol=cfg["rtol"],
                traction=np.ascontiguousarray(traction), clamped=clamped, loaded=loaded, rom=rom)


def rom_lhs_uniforms(family, n_k, n_s):
    """The U[0,1) draws of the stratified Latin-hypercube sampling of each
    cluster of `family` (d = 1): returns [n_k, n_s]."""
    rng = np.random.default_rng(100 + int(family))
    return rng.random((n_k, n_s))


def rom_lhs_draws(family, n_k, n_s, dim):
    """The draws of the Latin-hypercube sampling of each of the n_k^dim
    clusters of a family with dim parameters: U[0,1) offsets [n_cl, n_s, dim]
    and, per coordinate, a random order of the strata [n_cl, dim, n_s]."""
    rng = np.random.default_rng(100 + int(family))
    ncl = n_k ** dim
    u = rng.random((ncl, n_s, dim))
    perm = np.stack([np.stack([rng.permutation(n_s) for _ in range(dim)]) for _ in range(ncl)])
    return u, perm
