"""CPU oracle for nonlinear FEAST (Gavin, Miedlar, Polizzi, "FEAST Eigensolver for
Nonlinear Eigenvalue Problems", arXiv 1801.09794).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct complex128
implementation of what the GPU library computes.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  The HIP library and its Python
binding never import, call or link anything in here, and nothing in here imports them.

Modules
  quadrature  contour nodes and weights (Sec. 3, eq. feast_sum; Algorithm 1 inputs)
  problem     the matrix function T(lambda) = sum_j f_j(lambda) A_j and the block
              residual T(X, Lambda) (Sec. 2 eq. polynomialeig; Sec. 4.2)
  reduced     Step 1/2 of Algorithm 1: the projected problem solved by linearisation
              (Sec. 2 first companion form; Sec. 4.2), selection of m0 pairs
  nlfeast     Algorithm 1 itself, Steps 0-5
  dense       plain reference definitions of the linear-algebra steps the GPU path
              performs one by one (assembly, LU with partial pivoting, solves, the
              Step 4 sum, projections) so that each step can be compared on its own
  brute       brute-force ground truth: eigenvalues of the full companion
              linearisation, shift-invert Arnoldi near a point, winding-number count

Every function states the passage of the paper it follows.  Where the paper is silent
the reading taken is stated in the docstring.
"""
