"""Pins of the oracle's BDDC: exact identities of the Schur/recovery path,
BDDC algebra invariants and the converged fixed point vs a direct solve."""
import numpy as np
import pytest
import scipy.linalg as sla
from oracle.bddc import Problem, traction_load
from oracle.dofs import Dofs
from workloads import make_problem
from conftest import oracle_roms


@pytest.fixture(scope="module")
def small():
    prob = make_problem(2, nx=4, ny=3, p=4, m=2, jitter=0.03)
    P = Problem(prob, oracle_roms(prob))
    P.setup()
    return P


def test_dof_counts_match_paper():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "dof_counts.txt")
    for line in open(path):
        if line.startswith("#"):
            continue
        nx, ny, N, NU, NI, NC = map(int, line.split())
        d = Dofs(nx, ny, 8)
        assert d.N == N and d.N_C == NC
        assert NU < 0 or d.N_U == NU
        assert NI < 0 or d.N_I == NI


def test_schur_recovery_equals_direct(small):
    P = small
    d = P.dofs
    S = np.zeros((d.N_U, d.N_U))
    for cell in P.cells:
        S[np.ix_(cell.U_glob, cell.U_glob)] += cell.S
    f = P.rhs()[:, 0]
    u = np.linalg.solve(S, f)
    full = P.recover(u)
    ud = P.direct_solve()[0]
    assert np.abs(full - ud).max() <= 1e-11 * np.abs(ud).max()


def test_pcg_converges_to_direct(small):
    u, its, _ = small.solve(rtol=1e-13)
    ud = small.direct_solve()
    assert np.abs(u - ud).max() <= 1e-10 * np.abs(ud).max()
    assert its[0] < 40


def test_partition_of_unity(small):
    s = np.zeros(small.dofs.N_U)
    for cell in small.cells:
        s[cell.U_glob] += cell.D
    np.testing.assert_allclose(s, 1.0, atol=1e-14)


def test_coarse_basis_identities(small):
    for cell in small.cells[:6]:
        nC = len(cell.C_glob)
        assert np.abs(cell.C @ cell.Psi - np.eye(nC)).max() < 1e-10
        sc = cell.Psi.T @ cell.S @ cell.Psi
        assert np.abs(sc + cell.Lam).max() < 1e-9 * np.abs(sc).max()


def test_local_solve_vs_dense_saddle(small):
    rng = np.random.default_rng(4)
    for cell in small.cells[:6]:
        nU, nC = len(cell.U_glob), len(cell.C_glob)
        f, g = rng.normal(size=nU), rng.normal(size=nC)
        A = np.block([[cell.S, cell.C.T], [cell.C, np.zeros((nC, nC))]])
        ref = np.linalg.solve(A, np.r_[f, g])
        x, lam = small.local_solve(cell, f, g)
        np.testing.assert_allclose(np.r_[x, lam], ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())


def test_bddc_spectrum_lower_bound():
    """BDDC theory: the eigenvalues of S_BDDC^-1 S are >= 1."""
    prob = make_problem(1)
    P = Problem(prob, oracle_roms(prob))
    P.setup()
    n = P.dofs.N_U
    E = np.eye(n)
    S = np.stack([P.apply_S(E[:, j]) for j in range(n)], axis=1)
    M = np.stack([P.apply_M(E[:, j]) for j in range(n)], axis=1)
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    lam = sla.eigh(S, np.linalg.inv(M), eigvals_only=True)
    assert lam.min() > 1 - 1e-8
    assert lam.max() < 50


def test_single_cell_exact_preconditioner():
    prob = make_problem(1, nx=1, ny=1)
    P = Problem(prob, oracle_roms(prob))
    P.setup()
    _, its, _ = P.solve(rtol=1e-12)
    assert its[0] == 1


def test_constraint_set_does_not_change_solution():
    prob = make_problem(2, nx=3, ny=3, p=4)
    roms = oracle_roms(prob)
    outs = []
    for mom in (True, False):
        P = Problem(prob, roms, moments=mom)
        P.setup()
        outs.append(P.solve(rtol=1e-13)[0])
    assert np.abs(outs[0] - outs[1]).max() <= 1e-10 * np.abs(outs[0]).max()


def test_load_resultant():
    prob = make_problem(1)
    P = Problem(prob, oracle_roms(prob))
    F = P.global_f()
    # unit x-traction on the straight right side of length ny
    fx = F[0::2, 0].sum()
    fy = F[1::2, 0].sum()
    assert abs(fx - prob["ny"]) < 1e-13 and abs(fy) < 1e-13


def test_stabilisation_consistency_is_order_rho():
    """The rho-stabilised solution differs from the unstabilised one by
    O(rho) (the paper's consistency-error trend)."""
    base = make_problem(1, nx=2, ny=2, p=4)
    errs = []
    u0 = None
    for rho in (0.0, 1e-2, 1e-3, 1e-4):
        prob = dict(base, rho=rho)
        P = Problem(prob, None, assembly="fast")
        u = P.direct_solve()
        if u0 is None:
            u0 = u
        else:
            errs.append(np.abs(u - u0).max() / np.abs(u0).max())
    slopes = np.diff(np.log10(errs)) / -1.0
    assert np.all(np.abs(slopes - 1.0) < 0.15)


def test_edge_constraint_rows_closed_form():
    """Straight edge of length L, uniform parametrisation: averages are
    L * GLL weights and the moment row is L^2 w_k (1/2 - xi_k) on the
    component normal to the edge (GLL quadrature is exact here)."""
    from oracle.bddc import edge_constraint_rows
    from oracle.basis import gll_weights
    p, L = 5, 1.7
    X = np.zeros((2, 2, 2))
    X[0, 1] = (L, 0.0)
    X[1, 0] = (0.0, 1.0)
    X[1, 1] = (L, 1.0)
    rows = edge_constraint_rows(X, p, "bottom", True)
    w, xi = gll_weights(p), gll_nodes_p(p)
    np.testing.assert_allclose(rows[0, :, 0], L * w, atol=1e-14)
    np.testing.assert_allclose(rows[1, :, 1], L * w, atol=1e-14)
    np.testing.assert_allclose(rows[2, :, 0], 0.0, atol=1e-14)
    np.testing.assert_allclose(rows[2, :, 1], L * L * w * (0.5 - xi), atol=1e-14)
    # right edge (vertical, length 1): moment acts on u1 with (x2 - xbar2)
    rows = edge_constraint_rows(X, p, "right", True)
    np.testing.assert_allclose(rows[2, :, 0], w * (xi - 0.5), atol=1e-14)
    np.testing.assert_allclose(rows[2, :, 1], 0.0, atol=1e-14)


def gll_nodes_p(p):
    from oracle.basis import gll_nodes
    return gll_nodes(p)


def test_traction_load_closed_form():
    from oracle.basis import gll_weights
    p = 6
    X = np.zeros((3, 3, 2))
    for b in range(3):
        for a in range(3):
            X[b, a] = (2.0 + a / 2, 3.0 + 1.5 * b / 2)   # right edge of length 1.5
    f = traction_load(X, p, np.array([1.0, -2.0]))
    np.testing.assert_allclose(f[:, 0], 1.5 * gll_weights(p), atol=1e-14)
    np.testing.assert_allclose(f[:, 1], -3.0 * gll_weights(p), atol=1e-14)
