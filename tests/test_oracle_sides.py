"""Pins of the oracle's boundary conditions on any side of the lattice
(Sec. 2.2.1: homogeneous Dirichlet conditions on the clamped part of the
boundary, a traction on the loaded part, the rest traction free)."""
import numpy as np
import pytest

from oracle.bddc import Problem, traction_load
from oracle.dofs import Dofs, side_cells
from oracle.adjoint import compliance_gradient
from workloads import make_problem
from conftest import oracle_roms


def transpose_problem(prob):
    """The same lattice mirrored across the diagonal x1 = x2: cell (ix, iy)
    becomes cell (iy, ix), control point (jx, jy) becomes (jy, jx) with its
    coordinates swapped, the left side becomes the bottom side and the right
    side the top side, and every traction has its components swapped."""
    nx, ny = prob["nx"], prob["ny"]
    out = dict(prob)
    out["nx"], out["ny"] = ny, nx
    out["ctrl"] = np.ascontiguousarray(np.transpose(prob["ctrl"], (1, 0, 2))[:, :, ::-1])
    idx = np.arange(nx * ny)
    ix, iy = idx % nx, idx // nx
    tcell = ix * ny + iy          # new index of old cell (ix, iy): (ix' , iy') = (iy, ix)
    t = np.empty_like(prob["t"])
    fam = np.empty_like(prob["family"])
    t[tcell], fam[tcell] = prob["t"], prob["family"]
    out["t"], out["family"] = t, fam
    side = {"left": "bottom", "right": "top", "bottom": "left", "top": "right"}
    out["clamped"] = tuple(side[s] for s in prob.get("clamped", ("left",)))
    out["loaded"] = side[prob.get("loaded", "right")]
    out["traction"] = np.ascontiguousarray(prob["traction"][:, :, ::-1])
    return out, tcell


@pytest.fixture(scope="module")
def mirrored():
    prob = make_problem(2, nx=2, ny=3, p=4, m=2, jitter=0.03)
    roms = oracle_roms(prob)
    probT, tcell = transpose_problem(prob)
    res = []
    for pr in (prob, probT):
        P = Problem(pr, roms)
        P.setup()
        u, its, _ = P.solve(rtol=1e-13)
        res.append((P, u, its))
    return prob, probT, tcell, res


def test_mirror_displacement(mirrored):
    """Clamping the bottom and loading the top of the mirrored lattice gives
    the mirrored displacement of the left-clamped, right-loaded lattice.  The
    circle family is symmetric under xi1 <-> xi2, so its trimmed tensor, its
    snapshots and hence its reduced basis are invariant under the swap."""
    _, probT, _, res = mirrored
    assert probT["clamped"] == ("bottom",) and probT["loaded"] == "top"
    (_, u, _), (_, uT, _) = res
    uT_back = np.transpose(uT[0], (1, 0, 2))[:, :, ::-1]
    assert np.abs(uT_back - u[0]).max() <= 1e-10 * np.abs(u[0]).max()


def test_mirror_compliance_gradient(mirrored):
    _, _, tcell, res = mirrored
    (P, u, _), (PT, uT, _) = res
    J, gX, gt = compliance_gradient(P, u)
    JT, gXT, gtT = compliance_gradient(PT, uT)
    assert abs(J[0] - JT[0]) <= 1e-10 * abs(J[0])
    np.testing.assert_allclose(gtT[0][tcell], gt[0], rtol=0, atol=1e-9 * np.abs(gt).max())
    gXT_back = np.transpose(gXT[0], (1, 0, 2))[:, :, ::-1]
    np.testing.assert_allclose(gXT_back, gX[0], rtol=0, atol=1e-9 * np.abs(gX).max())


def _closed_form_counts(nx, ny, p, clamped, moments):
    kx = ("left" in clamped) + ("right" in clamped)
    ky = ("bottom" in clamped) + ("top" in clamped)
    N = 2 * (p * nx + 1 - kx) * (p * ny + 1 - ky)
    V = (nx + 1 - kx) * (ny + 1 - ky)
    E = nx * (ny + 1 - ky) + ny * (nx + 1 - kx)
    N_C = 2 * V + (3 if moments else 2) * E
    N_I = 2 * (p - 1) ** 2 * nx * ny
    return N, N - N_I, N_C


@pytest.mark.parametrize("clamped", [("left",), ("bottom",), ("right", "top"), ("left", "bottom", "top"),
                                     ("left", "right", "bottom", "top")])
@pytest.mark.parametrize("moments", [True, False])
def test_counts_closed_form(clamped, moments):
    for nx, ny, p in ((3, 2, 4), (1, 1, 3), (5, 4, 2)):
        d = Dofs(nx, ny, p, moments, clamped)
        N, N_U, N_C = _closed_form_counts(nx, ny, p, clamped, moments)
        assert (d.N, d.N_U, d.N_C) == (N, N_U, N_C), (clamped, nx, ny, p)
        # restriction maps: every skeleton and coarse id is used by some cell
        seen_u, seen_c = set(), set()
        for c in range(d.ncell):
            _, ug, _, cg, _ = d.cell_maps(c)
            seen_u |= set(int(g) for g in ug if g >= 0)
            seen_c |= set(int(g) for g in cg if g >= 0)
        assert seen_u == set(range(d.N_U)) and seen_c == set(range(d.N_C))


@pytest.mark.parametrize("clamped,loaded", [(("right", "top"), "left"), (("left", "bottom", "top"), "right"),
                                            (("bottom", "right"), "top")])
def test_pcg_equals_direct_any_sides(clamped, loaded):
    """BDDC-PCG to 1e-13 reproduces the direct solve, for lattices whose
    corner cells have two clamped edges and whose loaded edges end at clamped
    vertices; the partition of unity holds on every skeleton dof."""
    prob = make_problem(2, nx=3, ny=3, p=4, m=2, jitter=0.03, clamped=clamped, loaded=loaded)
    P = Problem(prob, oracle_roms(prob))
    P.setup()
    u, its, _ = P.solve(rtol=1e-13)
    ud = P.direct_solve()
    assert np.abs(u - ud).max() <= 1e-10 * np.abs(ud).max()
    s = np.zeros(P.dofs.N_U)
    for cell in P.cells:
        s[cell.U_glob] += cell.D
    np.testing.assert_allclose(s, 1.0, atol=1e-14)
    # Dirichlet nodes stay zero
    assert np.all(u[0][P.dofs.node_dirichlet] == 0.0)


@pytest.mark.parametrize("side", ["left", "right", "bottom", "top"])
def test_load_resultant_each_side(side):
    """On straight edges sum_k int b_k t ds = t times the edge length
    (partition of unity of the GLL basis); over a side of the unit-cell
    lattice the resultant is t times the side's length."""
    nx, ny, p = 3, 2, 5
    prob = make_problem(1, nx=nx, ny=ny, p=p, m=1)
    tr = np.array([0.7, -1.3])
    tot = np.zeros(2)
    for c, _ in side_cells(nx, ny, side):
        ix, iy = c % nx, c // nx
        X = prob["ctrl"][iy: iy + 2, ix: ix + 2, :]
        tot += traction_load(X, p, tr, side).sum(axis=0)
    length = ny if side in ("left", "right") else nx
    np.testing.assert_allclose(tot, tr * length, atol=1e-13)
