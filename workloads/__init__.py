"""Seeded synthetic lattice workloads.

This module only draws and lays out inputs (grid sizes, control nets, cell
topologies and thickness parameters, tractions, the uniform draws that the
offline Latin-hypercube sampling consumes).  It contains none of the solver's
arithmetic, so both the CPU oracle and the GPU library may use it.

Geometry follows the paper's construction (Sec. 2.1): unit parametric cells
mapped by a shared Bernstein/Bezier control net (a spline surface after Bezier
extraction) and trimmed by a per-cell level set.  Two level-set families stand
in for the paper's TPMS cells (Table 1), because both admit exact quadrature:

* family 0, circular hole: material where |xi - (1/2, 1/2)| > 1/2 - t;
* family 1, cross of two struts: material where |xi_1 - 1/2| < t/2 or
  |xi_2 - 1/2| < t/2.

The scalar thickness t plays the role of the threshold parameter mu (d = 1).

The paper's own cells are available too: families 2-5 are the level sets of
Table 1 (Schwarz Diamond, Schwarz Primitive, Schoen FRD, Schoen IWP) with the
bilinear threshold through one value per lattice vertex (d = 4, Sec. 2.1.2);
their quadrature is implicit (the oracle's height-function rule).
"""
from .configs import CONFIGS, TPMS_BOX, make_problem, rom_lhs_uniforms, rom_lhs_draws, family_name

__all__ = ["CONFIGS", "TPMS_BOX", "make_problem", "rom_lhs_uniforms", "rom_lhs_draws", "family_name"]
