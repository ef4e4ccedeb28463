"""FP64 CPU oracle for the MGR-preconditioned FGMRES hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct restatement of
what the method computes (Bui, Osei-Kuffuor, Castelletto, White, "A Scalable Multigrid
Reduction Framework for Multiphase Poromechanics of Heterogeneous Media", Sec. 5), used to
check the GPU library.  Only the test suite, the smoke check and the benchmark's CPU
baseline may import it; the product path never does, and it shares no code with the HIP
library.

Modules
  sparse  - a minimal CSR container, submatrices, transpose, and the sparse product with a
            pinned summation order (ascending inner index, separate multiply and add)
  mgr     - C/F splitting, Jacobi interpolation / injection restriction, the coarse-grid
            correction product, the dropping operator G, the merge S = A_CC - G(.),
            level recursion, and the multi-level V-cycle of Algorithm 2
  amg     - smoothed-aggregation AMG used for the F-relaxation of displacement and for the
            coarsest (pressure) grid: strength, MIS(2), aggregation, smoothed P, Galerkin
            coarse operators, l1-Jacobi V-cycle, dense LU at the coarsest level
  krylov  - flexible GMRES(m) with modified Gram-Schmidt and Givens rotations
  ilu     - ILU(k) pattern by levels of fill, factors by synchronous fine-grained
            fixed-point sweeps, triangular solves exact or by Jacobi sweeps (the global
            smoother of Sec. 5.3 / Sec. 6)
  assembly - residual F(x) and exact Jacobian of the two-phase poromechanics model of
            Sec. 2-3 (Q1 displacement, TPFA upwind mass balances, backward Euler)
  newton  - Newton's method with backtracking for one time step (Sec. 4, eq. newton)

Parity pins: every function is checked in tests/ against closed forms, identities of
Sec. 5.1, brute force on tiny inputs, or textbook special cases.  End-to-end iteration
counts against the paper are "parity unpinned": the paper's result tables are not
available as numbers.
"""
