"""DoF classification, restriction maps and coarse dofs (Sec. 3.1, 3.3.1).

Global GLL nodes form a (p nx + 1) x (p ny + 1) lattice; node (gx, gy) of
cell (ix, iy) is local node (a, b) = (gx - p ix, gy - p iy), k = a + (p+1) b.

Classification (reading of Sec. 3.1 that reproduces every dof count printed
in the scaling study and the 17k-cell statistics):
  * Dirichlet: nodes on the clamped sides of the lattice (Sec. 2.2.1, the
    Dirichlet part of the boundary), strong, whole side; the benchmark clamps
    the side x = 0 (gx = 0), which is the default;
  * interior u_I: the (p-1)^2 nodes strictly inside a cell;
  * skeleton u: every other node (any cell boundary, including the outer
    traction-free and loaded sides).
Coarse dofs (Sec. 3.3.1): two displacement values at every non-Dirichlet
grid vertex, and per non-Dirichlet cell edge two averages plus (optionally)
one moment.

Canonical local orders (also the export order of per-cell results):
  skeleton slots: nodes [BL, BR, TL, TR, left edge b=1..p-1, right edge,
                  bottom edge a=1..p-1, top edge], dof slot = 2*node + comp;
  coarse slots:   [BL.x, BL.y, BR.x, BR.y, TL.x, TL.y, TR.x, TR.y] then per
                  edge [left, right, bottom, top]: [avg x, avg y, (moment)];
  interior slots: node (b-1)(p-1) + (a-1), dof slot = 2*node + comp.
Slots of Dirichlet nodes (e.g. the left side of first-column cells) are
inactive, as are the coarse slots of Dirichlet vertices and edges.
"""
import numpy as np

EDGES = ("left", "right", "bottom", "top")
SIDES = EDGES   # sides of the lattice, in the same order as a cell's edges


def skeleton_nodes_local(p):
    """Local (a, b) of the canonical skeleton node slots."""
    nodes = [(0, 0), (p, 0), (0, p), (p, p)]
    nodes += [(0, b) for b in range(1, p)]
    nodes += [(p, b) for b in range(1, p)]
    nodes += [(a, 0) for a in range(1, p)]
    nodes += [(a, p) for a in range(1, p)]
    return nodes


def interior_nodes_local(p):
    return [(a, b) for b in range(1, p) for a in range(1, p)]


def edge_nodes_local(p, e):
    """The p+1 nodes of edge e in increasing running coordinate."""
    if e == "left":
        return [(0, b) for b in range(p + 1)]
    if e == "right":
        return [(p, b) for b in range(p + 1)]
    if e == "bottom":
        return [(a, 0) for a in range(p + 1)]
    return [(a, p) for a in range(p + 1)]


class Dofs:
    """All index maps of an nx x ny lattice of degree-p cells."""

    def __init__(self, nx, ny, p, moments=True, clamped=("left",)):
        self.nx, self.ny, self.p, self.moments = nx, ny, p, moments
        self.clamped = tuple(clamped)
        for sd in self.clamped:
            if sd not in SIDES:
                raise ValueError(f"unknown side {sd}")
        self.ncell = nx * ny
        self.nB = (p + 1) ** 2
        Gx, Gy = p * nx + 1, p * ny + 1
        self.Gx, self.Gy = Gx, Gy
        gx, gy = np.meshgrid(np.arange(Gx), np.arange(Gy), indexing="xy")
        cl = self.clamped
        dir_ = (("left" in cl) & (gx == 0)) | (("right" in cl) & (gx == Gx - 1)) \
            | (("bottom" in cl) & (gy == 0)) | (("top" in cl) & (gy == Gy - 1))
        inter = (gx % p != 0) & (gy % p != 0)
        skel = ~dir_ & ~inter
        self.node_dirichlet = dir_
        self.skel_id = -np.ones((Gy, Gx), dtype=np.int64)
        self.skel_id[skel] = np.arange(int(skel.sum()))
        self.N_U = 2 * int(skel.sum())
        self.free_id = -np.ones((Gy, Gx), dtype=np.int64)
        self.free_id[~dir_] = np.arange(int((~dir_).sum()))
        self.N = 2 * int((~dir_).sum())
        self.N_I = 2 * (p - 1) ** 2 * self.ncell
        self.sk_local = skeleton_nodes_local(p)
        self.in_local = interior_nodes_local(p)
        # coarse numbering: non-Dirichlet vertices, horizontal edges, vertical
        # edges (a vertex or edge on a clamped side carries no coarse dof)
        self.nce = 3 if moments else 2
        on_x = lambda vx: (("left" in cl) and vx == 0) or (("right" in cl) and vx == nx)
        on_y = lambda vy: (("bottom" in cl) and vy == 0) or (("top" in cl) and vy == ny)
        cid = 0
        self.vert_id = -np.ones((ny + 1, nx + 1), dtype=np.int64)
        for vy in range(ny + 1):
            for vx in range(nx + 1):
                if not (on_x(vx) or on_y(vy)):
                    self.vert_id[vy, vx] = cid
                    cid += 2
        self.hedge_id = -np.ones((ny + 1, nx), dtype=np.int64)
        for vy in range(ny + 1):
            for ex in range(nx):
                if not on_y(vy):
                    self.hedge_id[vy, ex] = cid
                    cid += self.nce
        self.vedge_id = -np.ones((ny, nx + 1), dtype=np.int64)
        for ey in range(ny):
            for vx in range(nx + 1):
                if not on_x(vx):
                    self.vedge_id[ey, vx] = cid
                    cid += self.nce
        self.N_C = cid

    def cell_xy(self, c):
        return c % self.nx, c // self.nx

    def natural(self, a, b, comp):
        """Natural local dof index comp*nB + a + (p+1) b."""
        return comp * self.nB + a + (self.p + 1) * b

    def cell_maps(self, c):
        """Per-cell index maps in canonical order:
        skel_nat[j], skel_glob[j] (-1 for Dirichlet), in_nat[j],
        coarse_glob[j] (-1 for inactive), and the natural index of every
        dof's global free id (free_glob[natural] or -1)."""
        p = self.p
        ix, iy = self.cell_xy(c)
        skel_nat, skel_glob = [], []
        for (a, b) in self.sk_local:
            g = self.skel_id[p * iy + b, p * ix + a]
            for comp in range(2):
                skel_nat.append(self.natural(a, b, comp))
                skel_glob.append(2 * g + comp if g >= 0 else -1)
        in_nat = []
        for (a, b) in self.in_local:
            for comp in range(2):
                in_nat.append(self.natural(a, b, comp))
        cg = []
        corners = [(ix, iy), (ix + 1, iy), (ix, iy + 1), (ix + 1, iy + 1)]
        for (vx, vy) in corners:
            v = self.vert_id[vy, vx]
            cg += [v, v + 1] if v >= 0 else [-1, -1]
        for e in EDGES:
            if e == "left":
                g = self.vedge_id[iy, ix]
            elif e == "right":
                g = self.vedge_id[iy, ix + 1]
            elif e == "bottom":
                g = self.hedge_id[iy, ix]
            else:
                g = self.hedge_id[iy + 1, ix]
            cg += [g + k for k in range(self.nce)] if g >= 0 else [-1] * self.nce
        free = -np.ones(2 * self.nB, dtype=np.int64)
        for b in range(p + 1):
            for a in range(p + 1):
                f = self.free_id[p * iy + b, p * ix + a]
                if f >= 0:
                    for comp in range(2):
                        free[self.natural(a, b, comp)] = 2 * f + comp
        return (np.array(skel_nat), np.array(skel_glob), np.array(in_nat),
                np.array(cg, dtype=np.int64), free)


def side_cells(nx, ny, side):
    """Cells along a side of the lattice with their position along it:
    [(cell, k)], k = iy on the left and right sides, ix on the bottom and top."""
    if side == "left":
        return [(iy * nx, iy) for iy in range(ny)]
    if side == "right":
        return [(iy * nx + nx - 1, iy) for iy in range(ny)]
    if side == "bottom":
        return [(ix, ix) for ix in range(nx)]
    if side == "top":
        return [((ny - 1) * nx + ix, ix) for ix in range(nx)]
    raise ValueError(f"unknown side {side}")
