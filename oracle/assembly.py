"""Cell stiffness matrices.

Fast assembly (Sec. 4.1): K[(i1,k1),(i2,k2)] = sum_{j1 j2 k3} I[k1,k2,j1,j2,k3]
C[i1,j1,i2,j2,k3], with the alpha-stabilisation folded in as Alg. 4 does:
K = (I + rho (I_pi - I)) . C = ((1 - rho) I + rho I_pi) . C.  The ROM variant
replaces I by U_r I_r(t) (Alg. 5).  The full-quadrature reference integrates
dB Chat(xi) dB directly over the material (weight 1) and the void (weight
rho), without interpolating Chat (Sec. 2.2.3 stabilisation term).

Local dof order of every matrix here: index i*nB + k, component i, node
k = a + (p+1) b (the paper's (i, k) indexing).
"""
import numpy as np
from .basis import tensor_basis
from .geometry import geometry_coefficients, map_eval, pulled_back_tensor
from .trimmed import I_exact, I_square, material_points, square_points
from .rom import stabilised_reduced


def contract(Ieff, C):
    """K[i1 k1, i2 k2] = sum_s Ieff[k1, k2, s] C[i1, i2, s], s = (j1, j2, k3)."""
    nB = Ieff.shape[0]
    K = np.einsum("abjlk,ijmlk->iamb", Ieff, C)
    return K.reshape(2 * nB, 2 * nB)


def fast_K(X, family, t, rho, p, q, Cmat, I_pi=None):
    """Fast assembly with the exact trimmed tensor (no ROM)."""
    if I_pi is None:
        I_pi = I_square(p, q)
    I = I_exact(family, p, q, t, I_pi)
    C, _ = geometry_coefficients(X, q, Cmat)
    return contract((1.0 - rho) * I + rho * I_pi, C)


def rom_Ieff(rom, t, rho):
    """Stabilised reconstruction Uhat Itil with Uhat = [U_r | I_pi] and
    Itil = [(1 - rho) I_r(t), rho]; returns (cluster, Ieff as a 5-index array)."""
    k, Itil = stabilised_reduced(rom, t, rho)
    Uhat = np.concatenate([rom["clusters"][k]["U"], rom["I_pi"][:, None]], axis=1)
    p, q = rom["p"], rom["q"]
    nB, nL = (p + 1) ** 2, (q + 1) ** 2
    return k, (Uhat @ Itil).reshape(nB, nB, 2, 2, nL)


def rom_K(X, rom, t, rho, Cmat):
    """Alg. 4 with Alg. 5: the online ROM stiffness of one cell."""
    _, Ieff = rom_Ieff(rom, t, rho)
    C, _ = geometry_coefficients(X, rom["q"], Cmat)
    return contract(Ieff, C)


def _quad_K(X, p, x1, x2, w, Cmat):
    _, dB = tensor_basis(p, x1, x2)
    _, J = map_eval(X, x1, x2)
    Ch, _ = pulled_back_tensor(J, Cmat)
    nB = (p + 1) ** 2
    K = np.einsum("k,ajk,kijml,blk->iamb", w, dB, Ch, dB)
    return K.reshape(2 * nB, 2 * nB)


def full_K(X, family, t, rho, p, q, Cmat, extra=6):
    """Full-quadrature reference: material part plus rho times the void part,
    Chat evaluated at the quadrature points.  Exact for affine maps; for
    curved maps Chat is rational and this is a high-order approximation."""
    Km = _quad_K(X, p, *material_points(family, p, q, t, extra=extra), Cmat)
    Ks = _quad_K(X, p, *square_points(p, q, extra=extra), Cmat)
    return (1.0 - rho) * Km + rho * Ks
