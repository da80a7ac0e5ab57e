"""Brute-force ground truth for the eigenvalues inside a contour (oracle; test
infrastructure only).

* polynomial T: every eigenvalue of the full first companion linearisation (Sec. 2),
  or, for large n, the eigenvalues nearest a point from shift-invert Arnoldi (ARPACK)
  on that linearisation, applying (L(sigma))^{-1} through one LU of T(sigma) by block
  elimination;
* any T: the number of eigenvalues inside C as the winding number of det T(z) along C
  (argument principle), with log det T(z) taken from LU factors.
"""
import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

from .problem import Problem
from .reduced import companion_first, reduced_coeffs_about, taylor_degree


def poly_coeffs(problem):
    """C_0..C_k of a polynomial Problem."""
    if not problem.is_polynomial:
        raise ValueError("not polynomial")
    k = problem.degree
    C = [np.zeros((problem.n, problem.n), dtype=complex) for _ in range(k + 1)]
    for (_, p), A in zip(problem.terms, problem.mats):
        C[int(p)] = C[int(p)] + A
    return C


def companion_eigs(problem):
    """All k n eigenvalues of the polynomial problem (inf where B is singular), by QZ on
    the first companion form; when the leading coefficient is exactly the identity, B = I
    and the pencil is the standard eigenproblem of -A (same eigenvalues, cheaper QR)."""
    A, B = companion_first(poly_coeffs(problem))
    if np.array_equal(B, np.eye(B.shape[0])):
        return np.linalg.eigvals(-A)
    ab = scipy.linalg.eigvals(-A, B, homogeneous_eigvals=True)
    alpha, beta = ab[0], ab[1]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(np.abs(beta) > 0, alpha / np.where(beta == 0, 1, beta), np.inf)


def companion_eigs_near(problem, sigma, k, tol=1e-13):
    """The k eigenvalues nearest sigma, by shift-invert Arnoldi on the first companion
    pencil (-A) v = lambda B v, i.e. eigenvalues nu = 1/(lambda - sigma) of
    (-A - sigma B)^{-1} B.  The solve with M = -(A + sigma B) reduces to one solve with
    P(sigma) = sum_i sigma^i C_i by eliminating the lower block rows."""
    C = poly_coeffs(problem)
    deg = len(C) - 1
    n = problem.n
    sigma = complex(sigma)
    lu = scipy.linalg.lu_factor(sum(sigma ** i * C[i] for i in range(deg + 1)), check_finite=False)

    # Companion rows 2..k read  -v_{i-1} + ... :  M = -(A + sigma B).  Writing the
    # unknown as blocks u_0..u_{k-1} (u_{k-1} = y-part), rows i >= 1 of M u = b give
    # u_{i-1} = b_i + sigma u_i, so every u_i is u_{k-1} times a power of sigma plus
    # known terms; the first row then gives P(sigma) u_{k-1} = -(b_0 + ...).
    def apply(v):
        v = v.reshape(deg, n)
        b = np.empty_like(v)
        b[0] = C[deg] @ v[0]
        b[1:] = v[1:]
        # u_i = sigma^{k-1-i} u_{k-1} + s_i, with s_{k-1} = 0, s_{i-1} = b_i + sigma s_i
        s = np.zeros_like(v)
        for i in range(deg - 1, 0, -1):
            s[i - 1] = b[i] + sigma * s[i]
        # first row of M u = b: -(sum_i C_{k-1-i} u_i + sigma C_k u_0) = b_0
        rhs = -b[0] - sigma * (C[deg] @ s[0])
        for i in range(deg):
            rhs = rhs - C[deg - 1 - i] @ s[i]
        ylast = scipy.linalg.lu_solve(lu, rhs, check_finite=False)
        u = np.empty_like(v)
        for i in range(deg):
            u[i] = sigma ** (deg - 1 - i) * ylast + s[i]
        return u.ravel()

    N = deg * n
    op = spla.LinearOperator((N, N), matvec=apply, dtype=complex)
    nu = spla.eigs(op, k=k, which="LM", tol=tol, return_eigenvectors=False,
                   ncv=min(N - 1, max(2 * k + 1, 40)))
    lam = sigma + 1.0 / nu
    return lam[np.argsort(np.abs(lam - sigma))]


def taylor_surrogate(problem, sigma, rho, tol=1e-16):
    """The polynomial P(mu) = sum_q mu^q C_q, mu = lambda - sigma, that matches T(sigma + mu)
    to a relative tail below tol on |mu| <= rho (the Taylor expansion of every f_j; exact for
    polynomial terms), as a polynomial Problem in mu."""
    d = taylor_degree(problem.terms, rho, tol)
    C = reduced_coeffs_about(problem.terms, problem.mats, sigma, d)
    return Problem([("pow", q) for q in range(d + 1)], C)


def eigs_near(problem, sigma, k, rho):
    """The k eigenvalues of T nearest sigma: shift-invert Arnoldi on the companion form of the
    Taylor surrogate about sigma (valid on |lambda - sigma| <= rho; the caller checks that the
    k-th distance stays well inside)."""
    if problem.is_polynomial:
        return companion_eigs_near(problem, sigma, k)
    S = taylor_surrogate(problem, sigma, rho)
    return sigma + companion_eigs_near(S, 0.0, k)


def eigen_residual(problem, lam, seed=0, steps=2):
    """Certificate that lam is an eigenvalue of T: ||T(lam) x|| with ||x|| = 1, x taken by
    `steps` inverse-iteration steps x <- T(lam)^{-1} x from a seeded random vector (one LU of
    T(lam)).  Since ||T(lam) x|| >= sigma_min(T(lam)) for every unit x, a small value bounds the
    smallest singular value of T(lam), i.e. T(lam) is within that distance of a singular
    matrix (Sec. 2: the eigenvalues are the points where T is singular)."""
    rng = np.random.default_rng(seed)
    n = problem.n
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    T = problem.T(complex(lam))
    lu = scipy.linalg.lu_factor(T, check_finite=False)
    for _ in range(max(1, steps)):
        x = scipy.linalg.lu_solve(lu, x / np.linalg.norm(x), check_finite=False)
    x /= np.linalg.norm(x)
    return float(np.linalg.norm(T @ x))


def refine_eigenvalue(problem, lam, steps=3, seed=0):
    """Two-sided Rayleigh functional iteration on T itself: with x = T(l)^{-1} b and
    y = T(l)^{-H} c (one LU of T(l) per step), l <- l - (y^H T(l) x) / (y^H T'(l) x).
    Used to sharpen eigenvalues from the companion operator, whose non-normality lets
    Arnoldi's residual test leave errors far above the residual.  Returns (l, res) with
    res = eigen_residual(problem, l): the residual of a unit vector taken at the final l,
    not at the l of the last step."""
    rng = np.random.default_rng(seed)
    n = problem.n
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    l = complex(lam)
    for _ in range(steps):
        T = problem.T(l)
        lu = scipy.linalg.lu_factor(T, check_finite=False)
        x = scipy.linalg.lu_solve(lu, b, check_finite=False)
        x /= np.linalg.norm(x)
        y = scipy.linalg.lu_solve(lu, c, trans=2, check_finite=False)
        y /= np.linalg.norm(y)
        num = np.vdot(y, T @ x)
        den = np.vdot(y, problem.dT(l) @ x)
        if den == 0:
            break
        l = l - num / den
    return l, eigen_residual(problem, l, seed=seed + 1)


def logdet(M):
    """log det M (complex, branch not normalised) from LU with partial pivoting."""
    lu, piv = scipy.linalg.lu_factor(M, check_finite=False)
    d = np.diag(lu)
    sign = (-1.0) ** int(np.sum(piv != np.arange(len(piv))))
    return np.sum(np.log(d.astype(complex))) + (0 if sign > 0 else 1j * np.pi)


def logdet_slope(problem, z):
    """d/dz log det T(z) = trace(T(z)^{-1} T'(z)), from LU factors of T(z)."""
    lu = scipy.linalg.lu_factor(problem.T(z), check_finite=False)
    return complex(np.trace(scipy.linalg.lu_solve(lu, problem.dT(z), check_finite=False)))


def phase_trend(problem, c, h, deflate=None):
    """Coefficients (a1, a2, a3) of the cubic Taylor polynomial of log g about c, g(z) =
    det T(z) / prod_i (z - mu_i): a1 = (log g)'(c) exactly, a2 and a3 from central differences of
    the exact slope at c - h, c, c + h."""
    mu = np.asarray([] if deflate is None else deflate, dtype=complex)

    def s(z):
        return logdet_slope(problem, z) - np.sum(1.0 / (z - mu))

    sm, s0, sp = s(c - h), s(c), s(c + h)
    return (s0, (sp - sm) / (4 * h), (sp - 2 * s0 + sm) / (6 * h * h))


def winding_count(problem, contour, npts=256, max_step=0.5, deflate=None, trend=(), log=None):
    """Number of eigenvalues of T inside C: (1/2 pi) times the total change of
    arg det T(z) around C (argument principle).  The sampling is refined until every step of
    the unwrapped phase is below max_step radians.

    deflate (optional): points mu_i, e.g. eigenvalues found by another method.  The phase
    followed is then that of g(z) = det T(z) / prod_i (z - mu_i), and the count is the winding
    number of g plus the number of mu_i inside C.  This is exact whatever the mu_i are (a
    wrong or missing mu_i changes the winding of g by the same amount); it only makes the
    phase vary slowly where the mu_i sit next to true eigenvalues, so far fewer samples are
    needed when many eigenvalues lie inside.

    trend (optional): coefficients a_1, a_2, ... of a polynomial p(z) = sum_k a_k (z - c)^k, c
    the contour's centre; the phase followed is then that of g(z) exp(-p(z)).  The factor is
    entire and has no zeros, so the count is unchanged for any coefficients; with those of the
    Taylor polynomial of log g (phase_trend) it takes out the smooth part of the phase, which
    for large n (a delay problem's exponential terms give log det T a slope of order n) would
    otherwise change by more than pi between samples and alias.
    log (optional): called with the number of evaluations of det T so far, every 16."""
    mu = np.asarray([] if deflate is None else deflate, dtype=complex)
    theta = np.linspace(0.0, 2 * np.pi, npts + 1)
    vals = {}

    def phase(t):
        if t not in vals:
            z = contour.point(t)
            w = z - contour.c
            ph = logdet(problem.T(z)).imag - np.sum(np.angle(z - mu)) - sum(
                (a * w ** (k + 1)).imag for k, a in enumerate(trend))
            vals[t] = np.angle(np.exp(1j * ph))
            if log is not None and len(vals) % 16 == 0:
                log(len(vals))
        return vals[t]

    pts = list(theta)
    total = 0.0
    i = 0
    while i < len(pts) - 1:
        a, b = pts[i], pts[i + 1]
        d = np.angle(np.exp(1j * (phase(b) - phase(a))))
        if abs(d) > max_step and b - a > 1e-9:
            pts.insert(i + 1, 0.5 * (a + b))
            continue
        total += d
        i += 1
    return int(round(total / (2 * np.pi))) + int(np.sum(contour.inside(mu)))
