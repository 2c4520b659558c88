"""Pins of the cell stiffness: symmetry, rigid-body kernel, affine exactness
of the fast assembly, a textbook element and the ROM reconstruction."""
import numpy as np
import pytest
from oracle import assembly as A
from oracle.geometry import material_tensor
from oracle.basis import gll_nodes
from oracle.rom import train
from workloads import rom_lhs_uniforms


def _affine(p_shift=(0.3, -0.2)):
    X = np.zeros((2, 2, 2))
    X[0, 0] = (0.0, 0.0)
    X[0, 1] = (1.3, 0.1)
    X[1, 0] = (0.2, 1.0)
    X[1, 1] = X[0, 1] + X[1, 0]
    return X + np.array(p_shift)


def _rigid_modes(X, p):
    from oracle.geometry import map_eval
    g = gll_nodes(p)
    n = p + 1
    xi1 = np.array([g[k % n] for k in range(n * n)])
    xi2 = np.array([g[k // n] for k in range(n * n)])
    F, _ = map_eval(X, xi1, xi2)
    nB = n * n
    tx = np.r_[np.ones(nB), np.zeros(nB)]
    ty = np.r_[np.zeros(nB), np.ones(nB)]
    rot = np.r_[-F[:, 1], F[:, 0]]
    return tx, ty, rot


@pytest.mark.parametrize("fam", [0, 1])
def test_affine_fast_equals_full_and_kernel(fam):
    p, q = 4, 2
    Cm = material_tensor(1.0, 0.3)
    X = _affine()
    K = A.fast_K(X, fam, 0.2, 1e-3, p, q, Cm)
    Kf = A.full_K(X, fam, 0.2, 1e-3, p, q, Cm)
    nrm = np.abs(K).max()
    assert np.abs(K - Kf).max() < 1e-12 * nrm
    assert np.abs(K - K.T).max() < 1e-14 * nrm
    for v in _rigid_modes(X, p):
        assert np.abs(K @ v).max() < 1e-12 * nrm * np.abs(v).max()
    assert np.linalg.eigvalsh(K)[3] > 1e-6 * nrm


def test_curved_translation_kernel_and_interpolation_error():
    p, q = 4, 2
    Cm = material_tensor(1.0, 0.3)
    rng = np.random.default_rng(5)
    X = np.stack(np.meshgrid(np.arange(3) / 2, np.arange(3) / 2, indexing="xy"), -1)
    X[1, 1] += 0.05 * rng.normal(size=2)
    K = A.fast_K(X, 0, 0.2, 0.0, p, q, Cm)
    Kf = A.full_K(X, 0, 0.2, 0.0, p, q, Cm)
    nrm = np.abs(K).max()
    tx, ty, rot = _rigid_modes(X, p)
    assert np.abs(K @ tx).max() < 1e-12 * nrm and np.abs(K @ ty).max() < 1e-12 * nrm
    # degree-2 interpolation of a smooth Chat: small but nonzero error
    assert np.abs(K - Kf).max() < 1e-2 * nrm


def test_q4_textbook_stiffness():
    """p = 1 on the untrimmed unit square equals the bilinear quadrilateral
    stiffness B^T D B built in Voigt notation with 2x2 Gauss points."""
    E, nu = 1.0, 0.3
    Cm = material_tensor(E, nu)
    X = _affine((0, 0))
    X = np.zeros((2, 2, 2)); X[0, 1] = (1, 0); X[1, 0] = (0, 1); X[1, 1] = (1, 1)
    K = A.fast_K(X, 1, 0.999999999999, 0.0, 1, 1, Cm)   # cross with t -> 1 fills the cell
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    D = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
    g = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    nodes = [(0, 0), (1, 0), (0, 1), (1, 1)]
    Kt = np.zeros((8, 8))
    for x in g:
        for y in g:
            dN = np.array([[(2 * a - 1) * (y if b else 1 - y), (2 * b - 1) * (x if a else 1 - x)] for (a, b) in nodes])
            B = np.zeros((3, 8))
            for k in range(4):
                B[0, k] = dN[k, 0]          # ux dofs first (component-major, as the oracle)
                B[1, 4 + k] = dN[k, 1]
                B[2, k] = dN[k, 1]
                B[2, 4 + k] = dN[k, 0]
            Kt += 0.25 * B.T @ D @ B
    assert np.abs(K - Kt).max() < 1e-10


@pytest.mark.parametrize("fam", [0, 1])
def test_rom_symmetry_kernel_and_accuracy(fam):
    p, q, rho = 3, 2, 5e-4
    rom = train(fam, p, q, 0.1, 0.3, 2, 40, 20, 6, rom_lhs_uniforms(fam, 2, 40))
    Cm = material_tensor(1.0, 0.3)
    X = _affine()
    for t in (0.13, 0.27):
        K = A.rom_K(X, rom, t, rho, Cm)
        Kx = A.fast_K(X, fam, t, rho, p, q, Cm)
        nrm = np.abs(K).max()
        assert np.abs(K - K.T).max() < 1e-13 * nrm
        for v in _rigid_modes(X, p):
            assert np.abs(K @ v).max() < 1e-11 * nrm * np.abs(v).max()
        assert np.abs(K - Kx).max() < 1e-5 * nrm
