"""CPU reference ("oracle") for residual-based Chebyshev filtered subspace iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library (no kernels, headers, helpers, constant generators or pre/post
processing); the only common dependency is the seeded input module
``workloads``, which holds no eigensolver arithmetic.

Everything here is plain, slow, obviously-correct NumPy/SciPy in float64,
following the paper (arXiv 2503.22652) step by step:

* ``chebyshev``  -- affine map, scaled Chebyshev polynomials C_k, the scaling
  coefficients sigma_k and the recurrence coefficients a_k, b_k, c_k
  (Section 2.1, eq. ChFSIrecurrence; Section 3.2, eq. ChFSIrecurrenceSEPMP).
* ``filters``    -- Algorithm 2 (Chebyshev filter) and Algorithm 3 (residual
  based Chebyshev filter).
* ``rr``         -- Rayleigh-Ritz on the non-orthogonal filtered basis
  (Algorithm 1, step 2) with the column-scaled / SVQB treatment of a
  numerically singular Gram matrix, and residual norms (Algorithm 1).
* ``solver``     -- the outer loop of Algorithm 1 with either filter.
* ``jacobi``     -- brute-force cyclic Jacobi eigensolver for tiny matrices
  (an independent pin for the library eigensolver used in ``rr``).
* ``stencil``    -- periodic 27-point operator application for grid pencils.
* ``cstencil``   -- the same grid pencil and Algorithm 3 as plain C loops with
  OpenMP (oracle/stencil27.c), FP64, for the CPU baseline at full grid size.
* ``angles``     -- maximum principal angle (Definition 2.1).
* ``bounds``     -- k-step Lanczos estimates of the spectrum of B^{-1} A,
  the filter's bounds (Section 2.1 treats them as estimates).
* ``diagnostics`` -- filtering error, angle and both sides of the convergence
  condition of Section 3.1 with Theorem 3.1's bound, per outer iteration
  (the check of Section 4.1.3).

Parity status of each function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""
from . import chebyshev, filters, rr, solver, jacobi, stencil, angles, diagnostics, bounds  # noqa: F401
