"""lbddc_assemble_fp32_noalloc through the C ABI: the FP32 contraction into a
caller buffer with the library's static device scratch, against the existing
entry point lbddc_assemble(LBDDC_FP32_CONTRACTION) + export, bit for bit, on
two calls in a row (the second on a smaller lattice, so the scratch holds
the previous call's larger contents), plus the size limit and the promise
that the call leaves every stage of the context as it was."""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu


def unpack(packed, p):
    """The documented packed layout [ncell][npair][4] -> dense [ncell][2nB][2nB]
    in the natural order (component i, node a + (p+1) b)."""
    nB = (p + 1) ** 2
    order = [(a, b) for b in range(1, p) for a in range(1, p)]
    order += [(0, 0), (p, 0), (0, p), (p, p)]
    order += [(0, b) for b in range(1, p)] + [(p, b) for b in range(1, p)]
    order += [(a, 0) for a in range(1, p)] + [(a, p) for a in range(1, p)]
    nat = np.array([a + (p + 1) * b for a, b in order])
    n1, n2 = np.tril_indices(nB)            # row-major over n1, n2 <= n1: pair P = n1 (n1+1)/2 + n2
    out = np.zeros((packed.shape[0], 2 * nB, 2 * nB))
    for i1 in range(2):
        for i2 in range(2):
            v = packed[:, :, 2 * i1 + i2].astype(np.float64)
            r, c = i1 * nB + nat[n1], i2 * nB + nat[n2]
            out[:, r, c] = v
            rr, cc = i2 * nB + nat[n2], i1 * nB + nat[n1]
            out[:, rr, cc] = v
    return out


def run_noalloc(s, prob):
    import torch
    from paper_2604_09113_amd import lbddc
    n = prob["nx"] * prob["ny"]
    npair = s.query(lbddc.Q_NPAIR)
    buf = torch.full((n, npair, 4), float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    s.assemble_fp32_noalloc(buf.data_ptr())
    torch.cuda.synchronize()
    return buf.cpu().numpy()


def test_noalloc_matches_fp32_entry_point_twice():
    from gpu_helpers import make_solver, set_problem
    from paper_2604_09113_amd import lbddc
    big = make_problem(3, nx=6, ny=5, p=8, m=2, jitter=0.03)
    small = make_problem(3, nx=3, ny=2, p=8, m=2, jitter=0.03, seed=11)
    roms = oracle_roms(big)
    s = make_solver(big, roms)
    s.assemble()
    s.setup()
    s.solve(rtol=1e-10, max_iter=500)
    u0 = s.displacement(0)
    n = big["nx"] * big["ny"]
    K64 = s.export(lbddc.X_K, 0, n)
    print(f"\n[noalloc] call 1: {n} cells", flush=True)
    got = unpack(run_noalloc(s, big), big["p"])
    # every stage is still there
    assert np.array_equal(s.displacement(0), u0) and np.array_equal(s.export(lbddc.X_K, 0, n), K64)
    s.solve(rtol=1e-10, max_iter=500)
    assert np.array_equal(s.displacement(0), u0)
    s.assemble(lbddc.FP32_CONTRACTION)
    ref = s.export(lbddc.X_K, 0, n)
    assert np.array_equal(got, ref)
    # the second call, on a smaller lattice
    set_problem(s, small)
    m = small["nx"] * small["ny"]
    print(f"[noalloc] call 2: {m} cells", flush=True)
    got = unpack(run_noalloc(s, small), small["p"])
    s.assemble(lbddc.FP32_CONTRACTION)
    ref = s.export(lbddc.X_K, 0, m)
    assert np.array_equal(got, ref)
    s.close()


def test_noalloc_rejects_lattices_beyond_the_scratch():
    """90,000 cells take at least 704 tiles of 128 cells, more than the 680
    that the scratch holds at q = 2: rejected before any device work."""
    import torch
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(2, nx=300, ny=300, p=2, m=1, jitter=0.0, moments=False)
    s = make_solver(prob, oracle_roms(prob))
    buf = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(lbddc.LbddcError) as ei:
        s.assemble_fp32_noalloc(buf.data_ptr())
    assert ei.value.status == lbddc.E_UNSUPPORTED
    assert "static scratch" in str(ei.value)
    s.close()
