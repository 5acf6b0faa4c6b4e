"""Plain FP64 CPU oracle of the discrete free-surface problem.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark may import anything from this package; the product library
never does, and this package never imports the product library (apart from the
shared seeded input generators in ``paper_1709_08803_amd.workloads``, which hold
none of the method's arithmetic).

Modules:
  residual  -- the nonlinear residual F(u) of Section 3.1 (C sums in bie_sums.c)
  linear    -- the linearised system of Section 4.2 / Appendix B, its Jacobian,
               the block-banded preconditioner of Appendix A, and the linear start
  jfnk      -- damped inexact Newton + right-preconditioned GMRES (Section 3.2)
  fourier   -- linear-theory reference values (Section 4.1)
  pressure  -- the bottom pressure of eq. (bottompressure) and the force on the
               topography (Section 2.1)
"""
