"""FP64 CPU oracle for the integral-form radiative transfer hot path.

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the CPU
baseline leg of `bench.py` may import, call, link or execute anything in this
package.  The GPU library shares no code with it and never calls it.

Modules:
  quadrature  symmetric simplex rules derived from their moment equations
  core        C core: P1 kappa, exact optical depths, kernel entries
  solve       Planck function, band weights, fixed point, direct solve
  htree       cluster tree and block tree (index work, compared bit-exactly)
"""
