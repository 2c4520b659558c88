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
def _trained(family, p, q, lo, hi, n_k, n_s, n_r, r):
    from oracle.rom import train
    from workloads import rom_lhs_uniforms
    return train(family, p, q, lo, hi, n_k, n_s, n_r, r, rom_lhs_uniforms(family, n_k, n_s))


def oracle_roms(prob):
    """Oracle-trained ROMs for every family of a problem (cached)."""
    out = {}
    for f, s in prob["rom"].items():
        out[f] = _trained(f, prob["p"], prob["q"], s["lo"], s["hi"], s["n_k"], s["n_s"], s["n_r"], s["r"])
    return out


@pytest.fixture(scope="session")
def roms_for():
    return oracle_roms
