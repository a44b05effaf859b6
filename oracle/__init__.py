"""Plain, slow FP64 CPU oracle of non-Hermitian FEAST (Kestyn, Polizzi, Tang).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
anything in this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or tables); both sides receive their
inputs from the separate ``workloads`` module.

Everything is complex128 NumPy/SciPy, written step by step in the order and
notation of the paper's complete algorithm figure (non-Hermitian FEAST, steps
0-5):

* ``contour``  -- trapezoidal nodes and weights on a circle or ellipse, the
  rational filter rho_a (eq:rational), the inside test and alpha of eq:res.
* ``linsolve`` -- direct solves of the shifted systems with one factorization
  per node and a conjugate-transpose solve for the left side (Section 2.4),
  plus ILU(0) written out from its definition (used to pin the preconditioner
  factors of the iterative path).
* ``feast``    -- the contour filter (eq:qr, eq:ql), B_Q, spurious detection
  (Section 2.7), resize and B-bi-orthonormalization (Sections 2.5, 2.6),
  Rayleigh-Ritz with QZ (step 4), residuals eq:res and the convergence test.

Parity status of each function is stated in its docstring; every function here
is pinned by a test in ``tests/test_oracle_*.py`` against closed forms,
prescribed spectra, brute-force eigendecompositions or invariants.
"""
from . import contour, linsolve, feast  # noqa: F401
