"""Oracle: a plain, slow, FP64 CPU implementation of the Elder-box time step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the HIP library never does, and the two
share no code.  Every function cites the passage of the paper it follows.

Modules:
  elder   - grid, coefficients, FV residual and analytic Jacobian (Section 2)
  newton  - implicit Euler + Newton with line search, exact sparse solves (Section 2.3)
  stats   - weighted mean, variance and exceedance probability (Section 3, eqs. pdestat,
            numer_var; Section 3.2 exceedance estimate)
  gradient - salt mass in a subregion and its tangent-linear gradient in xi
  gpc     - Legendre polynomial chaos surrogate: projection, moments, exceedance
            (Section 3.1 and the appendix)
"""
from . import elder, gpc, gradient, newton, stats  # noqa: F401
