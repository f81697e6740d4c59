"""Plain CPU oracle for Blanes, "Parallel computation of functions of matrices
and their action on vectors" (arXiv:2210.03714).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct FP64
reference that the GPU library is checked against.  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code, tables or constants with the GPU library (``paper_2210_03714_amd``) and
imports nothing from it; the library never imports this package.

Modules
-------
coefficients  exact rational shift/weight sets (Vandermonde system of §2)
theta         forward error bound and the admissible-norm table θ (§3)
method        the algorithm itself: norm, plan, shifted LU solves, round-off
              form combination, squaring / N-step recurrence (§1, §2, §4.3)
banded        the N-step action for a tridiagonal A with tridiagonal LU
              solves (§2.1, §5)

Every function cites the passage of the paper it follows.
"""

from . import coefficients, theta, method, banded  # noqa: F401
