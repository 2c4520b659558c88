import os
import sys
import functools

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@functools.lru_cache(maxsize=None)
def _trained(family, p, q, lo, hi, n_k, n_s, n_r, r, dim=1, only=None):
    from oracle.rom import train
    from workloads import rom_lhs_uniforms, rom_lhs_draws
    if dim == 1:
        return train(family, p, q, lo, hi, n_k, n_s, n_r, r, rom_lhs_uniforms(family, n_k, n_s))
    u, perm = rom_lhs_draws(family, n_k, n_s, dim)
    return train(family, p, q, lo, hi, n_k, n_s, n_r, r, u, dim=dim, lhs_perm=perm,
                 only=None if only is None else set(only))


def oracle_roms(prob):
    """Oracle-trained ROMs for every family of a problem (cached).  A family
    with four parameters per cell trains only the clusters its cells visit
    (each of its snapshots needs the implicit quadrature)."""
    from oracle.rom import find_cluster_nd
    out = {}
    for f, s in prob["rom"].items():
        dim = s.get("dim", 1)
        only = None
        if dim > 1:
            cells = np.nonzero(prob["family"] == f)[0]
            only = tuple(sorted({find_cluster_nd(prob["mu"][c], s["lo"], s["hi"], s["n_k"]) for c in cells}))
        out[f] = _trained(f, prob["p"], prob["q"], s["lo"], s["hi"], s["n_k"], s["n_s"], s["n_r"], s["r"],
                          dim, only)
    return out


@pytest.fixture(scope="session")
def roms_for():
    return oracle_roms
