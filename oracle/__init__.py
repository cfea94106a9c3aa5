"""Plain, slow, FP64 CPU oracle for the RASPEN hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The HIP
library never calls it and shares no code with it; the only thing both sides
share are the seeded input generators in ``synth``.

Everything is written from the paper (Ciaramella, Kartmann, Mueller,
"Solving semi-linear elliptic optimal control problems with L1-cost via
regularization and RAS-preconditioned Newton methods"): NumPy / SciPy sparse,
float64, sequential, with sparse direct solves (``scipy.sparse.linalg``) where
the paper uses a direct solver.

Modules
  pointwise  -- proj, P_eps, P'_eps, the smoothed soft-threshold u(p), phi family
  system     -- 5-point A, F_eps(x) and F'_eps(x) on the whole grid
  newton     -- Algorithm 1 (damped Newton, relaxed backtracking, eps-continuation)
  krylov     -- restarted GMRES(m), written out (Arnoldi-MGS + Givens)
  schwarz    -- partition, R_i / P_i / P~_i, local corrections, Algorithms 2-4

Parity status: every function is pinned by ``tests/test_oracle_pins.py``
(closed forms, eigenfunctions, manufactured solutions, the linear-quadratic
direct solve, RASPEN versus global Newton, finite-difference Jacobians).
"""
from . import pointwise, system, newton, krylov, schwarz  # noqa: F401
