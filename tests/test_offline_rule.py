"""The offline stage's implicit-domain rule (the code the GPU kernels run,
compiled for the host through a test entry of the library) against the
oracle's quadrature: the trimmed tensors of the four Table 1 level sets with
non-uniform thresholds, and the Schwarz Diamond at threshold 0 (boundary lines
crossing at saddles), agree to 1e-13 of their largest entry.  Both follow
Saye's method but share no code; they make different refinement choices in
places, so their point sets differ while the integrals agree."""
import numpy as np
import pytest

from oracle import implicit as im
from oracle.trimmed import integrate_points

MU = {2: [0.2, 0.8, 0.4, 0.6], 3: [0.1, 0.5, -0.3, 0.7], 4: [-3.0, -1.0, -5.0, 0.2], 5: [-2.0, 1.0, 0.5, 2.0]}


@pytest.mark.parametrize("fam,mu", list(MU.items()) + [(2, [0.0] * 4)])
def test_offline_rule_matches_oracle(fam, mu):
    from paper_2604_09113_amd import lbddc
    x, y, w = lbddc.implicit_rule_host(fam, mu, 12)
    I = integrate_points(3, 2, x, y, w)
    Io = integrate_points(3, 2, *im.tpms_rule(fam, mu, 12))
    assert np.abs(I - Io).max() <= 1e-13 * np.abs(Io).max()
