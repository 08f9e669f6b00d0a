"""CPU FP64 oracle for the space-time inexact Uzawa method (Neumüller & Smears,
"Time-parallel iterative solvers for parabolic evolution equations").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library;
the only common dependency is the seeded input generator package ``synth``,
which holds no solver arithmetic.

Everything here is plain, slow and written to be checked against the paper by
eye: numpy/scipy in float64, library primitives (sparse LU, dense matmul,
eigensolvers) used as single steps, no blocking or fusion.

Modules
  fd         finite-difference operator -div(kappa grad) and its assembly
  euler      sequential implicit Euler, eq. (2.1) -- the result the method reaches
  dst        the time transforms Phi, Phi^{-1} of eqs. (4.2)-(4.3), mu_k of (4.5)
  spacetime  time-global K, A, B, saddle-point matrix, S, P, H (Section 2, eq. (4.4))
  mg         the geometric multigrid V-cycle used as spatial preconditioner
  precond    A-tilde^{-1} (eq. (3.2)) and H-tilde^{-1} (eq. (4.6))
  uzawa      the inexact Uzawa iteration, eq. (3.1)
  spectral   eigenvalues of H^{-1} S (Section 8.1, Table 1) and Theorem 3.1's rate
  fem1d      1-D P1 finite-element mass/stiffness matrices (Section 8.1 workload)

Parity status: the multigrid V-cycle is not specified by the paper beyond
"one or two V-cycles with Jacobi smoothers" (Section 8.2); its definition here
is this project's reading, pinned by a dense matrix construction and by its
symmetry/contraction properties, not by a value the paper prints.
"""
