"""Plain, slow FP64 CPU oracle for explicit mapped tent pitching (MTP) with
structure-aware Taylor (SAT) time stepping for DG Maxwell.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
this package: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the GPU library; the only common module is ``mtp_inputs``
(meshes, exact solutions), which holds none of the method's arithmetic.

Independent choices made here on purpose (the GPU path makes different ones):
  * modal basis: Legendre products orthonormalised on the reference simplex,
  * collapsed-coordinate Gauss-Jacobi quadrature,
  * per-tent quadrature assembly of M(t), M' and A as block matrices,
  * generic dense LU solves for M_i U = rhs (no closed-form inverse),
  * face integrals by mapping physical face points into both elements
    (no node matching),
  * its own tent pitcher implementing the same documented pitching rule.

Parity status of every function is stated in its docstring; functions without a
pin say "parity unpinned".
"""
