"""Plain FP64 CPU oracle for the multigrid CP decomposition hot path.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
or call this package.  It shares no code with the HIP path and imports nothing
from it; both sides take their inputs from the seeded generators only.

Everything here is NumPy in float64, written to be read against the paper
(De Sterck & Miller, "An adaptive algebraic multigrid algorithm for low-rank
canonical tensor decomposition"):

* ``oracle.cp``  -- Section 2 (matricization, Khatri-Rao product), Section 3
  (gradient eq. (6)-(8), ALS as block nonlinear Gauss-Seidel, normalization
  eq. (10), sorting), the objective eq. (2) and the stopping measure eq. (30).
* ``oracle.amg`` -- Section 4 (Galerkin coarse tensor eq. (13)/(15), Cholesky
  transform, prolongation eq. (18)/(22), geometric coarsening Sec. 4.3,
  least-squares interpolation eq. (19)-(20), Algorithm 1 CP-AMG-mult) and
  Section 5 (FAS operators eq. (23)-(28), relaxation eq. (29) with ten
  Gauss-Seidel iterations, Algorithm 2 CP-FAS, Algorithm 3 FMG-CP-FAS) and the
  Section 6.1 driver rules.

Parity status: every function is pinned by tests against brute force, closed
forms or invariants, except the least-squares interpolation heuristic
(``amg.ls_interp_weights`` / ``amg.build_interp``), whose absolute quality is
"parity unpinned" beyond its exactness cases (see the tests).
"""
from . import cp, amg  # noqa: F401
