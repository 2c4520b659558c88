"""Phase timing of the PCG loop (lbddc_set_timing): the events it records
change neither the iterates nor the solution, phases that are not timed
report zero, sampled timing (one iteration in eight, scaled to all) reports
the same per-application times to within the spread of the launches, and
unknown bits are rejected."""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu


def test_timing_mask_changes_nothing_but_the_times():
    from gpu_helpers import make_solver
    from paper_2604_09113_amd import lbddc
    prob = make_problem(4, nx=5, ny=4, p=4)
    s = make_solver(prob, oracle_roms(prob))
    s.assemble()
    s.setup(lbddc.MIXED)
    pcg = ("op_kernel", "pre_kernel", "coarse_solve", "coarse_fwd_sweep", "coarse_bwd_sweep")
    runs = {}
    for mask in (lbddc.TIME_ALL, 0, lbddc.TIME_COARSE, lbddc.TIME_OP | lbddc.TIME_PRE,
                 lbddc.TIME_ALL | lbddc.TIME_SAMPLE):
        s.set_timing(mask)
        inf = s.solve(rtol=1e-10, max_iter=500)
        runs[mask] = (inf[0]["iters"], s.displacement(0), s.phase_times())
        ph = runs[mask][2]
        print(f"[timing] mask {mask}: {inf[0]['iters']} its, " + " ".join(f"{k} {ph[k]:.4f}" for k in pcg))
    it0, u0, _ = runs[lbddc.TIME_ALL]
    for mask, (it, u, ph) in runs.items():
        assert it == it0 and np.array_equal(u, u0)
        timed = {"op_kernel": mask & lbddc.TIME_OP, "pre_kernel": mask & lbddc.TIME_PRE,
                 "coarse_solve": mask & lbddc.TIME_COARSE, "coarse_fwd_sweep": mask & lbddc.TIME_COARSE,
                 "coarse_bwd_sweep": mask & lbddc.TIME_COARSE}
        for k in pcg:
            assert (ph[k] > 0) if timed[k] else (ph[k] == 0), (mask, k, ph[k])
        assert ph["solve"] > 0
    full, sampled = runs[lbddc.TIME_ALL][2], runs[lbddc.TIME_ALL | lbddc.TIME_SAMPLE][2]
    for k in pcg:
        assert 0.5 * full[k] <= sampled[k] <= 2.0 * full[k], (k, full[k], sampled[k])
    with pytest.raises(lbddc.LbddcError):
        s.set_timing(16)
    s.close()
