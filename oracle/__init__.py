"""CPU FP64 oracle for the space-time BDF1 method (test infrastructure only).

This package is the independent reference the HIP path is checked against. It is
plain NumPy/SciPy in float64, written from the paper's equations, and shares no
code with the HIP library or its Python binding. Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never does.

Modules
  discretization  Eq. (3) residual and the Jacobian blocks A_n = I + tau dF/du
                  (Section 3, Eq. (5)-(6)) for one time level.
  sequential      the sequential BDF1 time stepper with Newton at every step
                  (Section 2): the reference solution.
  allatonce       the all-at-once system (Section 3, Eq. (4)-(6)), one global
                  Newton step by a sparse direct solve of the whole space-time
                  Jacobian, by the block inverse of Eq. (7), and by the decoupled
                  system of Theorem 1 / Eq. (8)-(9) with explicit products.
  condition       the condition-number estimate of Section 7, Eq. (cond).
  coarse          the coarse-grid initial iterate of Section 4 (sequential solve on a
                  grid coarsened by c_f in space and time, 1-D cubic splines back).
  neural          FP64 reference forward/backward of the spectral neural operator
                  used for the learned initial iterate.

Parity status of every function is stated in its module header.
"""
