"""FP64 CPU oracle for the regularized Newton ground-state method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  The
GPU library never calls into this package and shares no code with it.

Plain, slow, obviously-correct NumPy/SciPy code in float64 / complex128:

* ``discretization`` -- grid, trap, Fourier and sine pseudospectral and
  finite-difference operators (§2.1, §2.2, §2.3).
* ``unified``        -- the unified problem F(X) on the unit sphere, its
  gradient and Hessian (§3, Lemma 3.1), chemical potential and residual.
* ``feasible``       -- the Cayley curve (Theorem 3.3) and the feasible
  gradient method with BB steps and nonmonotone search (§3.1, Algorithm 1).
* ``newton``         -- the regularized Newton method (§3.2, Algorithm 2).
* ``cascade``        -- Fourier prolongation and the cascadic multigrid
  (Algorithm 3).

Every function is pinned by a ``-m "not gpu"`` test against closed forms,
printed values of the paper, invariants or brute force; see the tests.
"""
from .discretization import (axis_points, grid_coords, h_vol, potential,  # noqa: F401
                             kinetic, h_lin, h_full)
from .unified import UnifiedProblem, re_dot  # noqa: F401
from .feasible import cayley_coefficients, cayley_point, feasible_gradient  # noqa: F401
from .newton import regularized_newton, Options  # noqa: F401
from .cascade import prolong_fourier, cascadic  # noqa: F401
