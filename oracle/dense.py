"""Plain definitions of the linear-algebra steps inside Step 4 and Steps 1/5 of
Algorithm 1 (oracle; test infrastructure only).  The GPU library performs these steps
as separate kernels; each function here is the textbook definition, written so that
a reader can check it by eye, and is used to compare the steps one at a time.
"""
import numpy as np

from .problem import f_eval


def assemble(terms, mats, z):
    """T(z_k) = sum_j f_j(z_k) A_j for every node z_k (the matrices T(z_j) whose
    inverses Step 4 applies)."""
    out = []
    for zk in np.atleast_1d(z):
        T = np.zeros_like(mats[0], dtype=complex)
        for (kind, p), A in zip(terms, mats):
            T = T + complex(f_eval(kind, p, zk)) * A
        out.append(T)
    return out


def lu_partial_pivot(A):
    """Unblocked right-looking LU with partial pivoting (Gaussian elimination with a row
    interchange at every step).  The pivot is the entry of largest |Re| + |Im| in the
    column (the LAPACK convention for complex matrices), the first such row on ties.
    Returns (LU, ipiv): unit-lower L below the diagonal and U on and above it, packed
    in one matrix; ipiv[k] is the row exchanged with row k at step k (LAPACK
    convention, 0-based).  P A = L U where P applies the exchanges in order."""
    LU = np.array(A, dtype=complex, copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(n, dtype=np.int64)
    for k in range(n):
        p = k + int(np.argmax(np.abs(LU[k:, k].real) + np.abs(LU[k:, k].imag)))
        ipiv[k] = p
        if p != k:
            LU[[k, p], :] = LU[[p, k], :]
        piv = LU[k, k]
        if piv == 0:
            raise ZeroDivisionError("zero pivot at column %d" % k)
        LU[k + 1:, k] /= piv
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, ipiv


def apply_pivots(ipiv, B):
    """P B for the row exchanges ipiv (in order)."""
    B = np.array(B, dtype=complex, copy=True)
    for k, p in enumerate(ipiv):
        if p != k:
            B[[k, p], :] = B[[p, k], :]
    return B


def lu_solve(LU, ipiv, B):
    """x = A^{-1} B from the packed factors: forward substitution with unit L, then
    back substitution with U."""
    Y = apply_pivots(ipiv, B)
    n = LU.shape[0]
    for i in range(n):
        Y[i] -= LU[i, :i] @ Y[:i]
    for i in range(n - 1, -1, -1):
        Y[i] = (Y[i] - LU[i, i + 1:] @ Y[i + 1:]) / LU[i, i]
    return Y


def step4_sum(X, solves, lam, z, omega):
    """Q = sum_k omega_k (X - Y_k) (z_k I - Lambda)^{-1} with Y_k = T(z_k)^{-1} T(X, Lambda)
    (Algorithm 1, Step 4, quadrature form)."""
    Q = np.zeros_like(X, dtype=complex)
    for Yk, zk, wk in zip(solves, z, omega):
        Q = Q + wk * (X - Yk) / (zk - lam)[None, :]
    return Q


def block_residual(terms, mats, X, lam):
    """T(X, Lambda) = sum_j A_j X f_j(Lambda) and its column 2-norms (Steps 3, 4)."""
    R = np.zeros_like(X, dtype=complex)
    for (kind, p), A in zip(terms, mats):
        R = R + (A @ X) * f_eval(kind, p, lam)[None, :]
    return R, np.linalg.norm(R, axis=0)


def project(mats, Q):
    """Q^H A_j Q (Algorithm 1, Step 1)."""
    return [Q.conj().T @ A @ Q for A in mats]
