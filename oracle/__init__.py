"""CPU oracle for the ROM-accelerated BDDC method (arXiv 2604.09113).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64
implementation of what the GPU library computes, written step by step from
the paper so that a reader can check it against the text.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
GPU library never does, and it shares no code with it.

Modules (each function cites the passage it follows):
  basis     GLL nodes, Lagrange and Bernstein polynomials     (Sec. 2.2.2, 2.1)
  geometry  map, Jacobian, pulled-back tensor, coefficients   (Sec. 2.2.1, Eq. pull-back; Sec. 4.1)
  trimmed   exact trimmed integrals I(t) and I_Pi             (Sec. 4.1-4.2)
  implicit  Table 1 level sets, bilinear threshold, implicit-
            domain quadrature (Saye's height-function method) (Sec. 2.1.2, 2.2.3, Table 1)
  rom       offline MDEIM training and online evaluation,
            one or four parameters per cell                   (Sec. 4.2, Alg. 3, Alg. 5)
  assembly  fast/ROM stiffness, full-quadrature reference     (Sec. 4.1, Alg. 4)
  dofs      DoF classification, restriction maps, coarse dofs (Sec. 3.1, 3.3.1)
  bddc      Schur complements, constraints, coarse basis,
            weights, preconditioner, PCG, recovery, direct    (Sec. 3, Alg. 1-2)
  adjoint   compliance and its gradient, finite differences   (choice of the build; see module)

Parity status: every function here is pinned by a test under tests/ against
closed forms, invariants, brute force or an independent second method,
except where a function's docstring says "parity unpinned".
"""
