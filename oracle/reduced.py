"""Steps 1 and 2 of Algorithm 1 (oracle; test infrastructure only).

Step 1 solves the projected problem Q^H T(lambda) Q y = 0.  For polynomial T the paper
uses "a simple linearization" (Sec. 4.2), the first companion form of Sec. 2:

    L(lambda) = lambda diag(A_k, I, ..., I) + [[A_{k-1}, ..., A_1, A_0],
                                               [-I,  0, ...,  0,  0 ],
                                               [ 0, -I, ...,  0,  0 ], ...]

whose right eigenvectors are [lambda^{k-1} y; ...; lambda y; y] (Sec. 2, quoted for k = 2
and written out here for general k).  Non-polynomial T needs "a Newton- or a
projection-type" method (Sec. 6); the reading taken here is: replace each
non-polynomial f_j by its Taylor polynomial about the contour centre, of the smallest
degree d whose Lagrange remainder on the disk |lambda - c| <= 1.5 max(a, b) is below
1e-16 relative, linearise that polynomial, select, then take up to 3 Newton steps per
selected pair on the exact reduced function.

Second reading for non-polynomial T, required when a term is a caller-supplied function
(no Taylor coefficients to linearise): the projected problem is solved by a contour-integral
method of the kind Sec. 3 reviews, applied to the small m0 x m0 function.  The moments
(1/2 pi i) oint mu^p T_red(z)^{-1} dz (Sec. 3 eq. cauchymoments, with the normalised variable
mu = (z - c)/L, L = 1.5 max(a, b)) are taken on the ellipse of the same shape scaled by 1.5
(the same enlargement as the Taylor disk above), by the trapezoid rule in the ellipse
parameter; the block Hankel matrices of moments 0..2K-1 (K = 2, or 3 when the first has full
rank) reduce the eigenvalues inside that ellipse to a linear eigenproblem (W.-J. Beyn, "An
integral method for solving nonlinear eigenvalue problems", Linear Algebra Appl. 436 (2012),
with the block Hankel form of the Sakurai-Sugiura methods); each pair found then takes
Newton steps on the exact reduced function.  When fewer than m0 pairs are found, the
selection is completed with unit vectors orthogonal to those found, paired with values spread
over the enlarged ellipse: outside C, so never counted, and each one still filtered into the
wanted subspace by Step 4.

Step 2 keeps the m0 pairs "closest to the interior of C" (Sec. 4.2): the reduced
eigenvalues sorted by normalised contour radius, ascending, ties by index, infinite
ones last.
"""
import math

import numpy as np
import scipy.linalg

from .problem import f_eval, f_deriv, taylor_coeffs


def companion_first(coeffs):
    """First companion pencil of P(lambda) = sum_i lambda^i C_i, i = 0..k.
    Returns (A, B) with L(lambda) = lambda B + A, so that eigenpairs solve
    (-A) v = lambda B v."""
    k = len(coeffs) - 1
    if k < 1:
        raise ValueError("degree must be >= 1")
    m = coeffs[0].shape[0]
    N = k * m
    A = np.zeros((N, N), dtype=complex)
    B = np.zeros((N, N), dtype=complex)
    B[:m, :m] = coeffs[k]
    for i in range(1, k):
        B[i * m:(i + 1) * m, i * m:(i + 1) * m] = np.eye(m)
    for i in range(k):                      # block column i holds C_{k-1-i}
        A[:m, i * m:(i + 1) * m] = coeffs[k - 1 - i]
    for i in range(1, k):                   # -I below the first block row
        A[i * m:(i + 1) * m, (i - 1) * m:i * m] = -np.eye(m)
    return A, B


def _poly_eigs(coeffs):
    """All eigenvalues (inf for beta = 0) and the y-part of each eigenvector of the
    matrix polynomial sum_i lambda^i C_i, via the first companion form."""
    k = len(coeffs) - 1
    m = coeffs[0].shape[0]
    A, B = companion_first(coeffs)
    ab, V = scipy.linalg.eig(-A, B, homogeneous_eigvals=True)
    alpha, beta = ab[0], ab[1]
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = np.where(np.abs(beta) > 0, alpha / np.where(beta == 0, 1, beta), np.inf)
    Y = np.zeros((m, V.shape[1]), dtype=complex)
    for col in range(V.shape[1]):
        blocks = V[:, col].reshape(k, m)    # block i = lambda^{k-1-i} y
        b = int(np.argmax(np.linalg.norm(blocks, axis=1)))
        Y[:, col] = blocks[b]
    return lam, Y


def taylor_degree(terms, rho, tol=1e-16):
    """Smallest degree d with (tau rho)^{d+1} e^{tau rho} / (d+1)! <= tol for every
    'exp' term and d >= p for every 'pow' term."""
    d = 1
    for kind, p in terms:
        if kind == "pow":
            d = max(d, int(p))
        else:
            x = abs(float(p)) * rho
            e = 1
            while (x ** (e + 1)) * math.exp(x) / math.factorial(e + 1) > tol:
                e += 1
            d = max(d, e)
    return d


def reduced_coeffs_about(terms, Ahat, centre, degree):
    """Coefficients B_p of sum_j f_j(c + mu) Ahat_j = sum_p mu^p B_p (truncated)."""
    B = [np.zeros_like(Ahat[0]) for _ in range(degree + 1)]
    for (kind, p), Aj in zip(terms, Ahat):
        t = taylor_coeffs(kind, p, centre, degree)
        for q in range(degree + 1):
            if t[q] != 0:
                B[q] = B[q] + t[q] * Aj
    return B


def reduced_T(terms, Ahat, lam):
    return sum(complex(f_eval(k, p, lam)) * Aj for (k, p), Aj in zip(terms, Ahat))


def reduced_dT(terms, Ahat, lam):
    return sum(complex(f_deriv(k, p, lam)) * Aj for (k, p), Aj in zip(terms, Ahat))


def newton_polish(terms, Ahat, lam, y, steps=3):
    """Newton on F(y, lambda) = [T(lambda) y ; v^H y - 1] with v = y / |y|^2 (so that
    v^H y = 1 initially); Jacobian [[T(lambda), T'(lambda) y], [v^H, 0]]."""
    m = y.shape[0]
    v = y / np.vdot(y, y)
    for _ in range(steps):
        Tl = reduced_T(terms, Ahat, lam)
        F = np.concatenate([Tl @ y, [np.vdot(v, y) - 1.0]])
        scale = sum(abs(complex(f_eval(k, p, lam))) * np.linalg.norm(Aj) for (k, p), Aj in zip(terms, Ahat))
        if np.linalg.norm(F[:m]) <= 1e-15 * scale * np.linalg.norm(y) and abs(F[m]) < 1e-15:
            break
        J = np.zeros((m + 1, m + 1), dtype=complex)
        J[:m, :m] = Tl
        J[:m, m] = reduced_dT(terms, Ahat, lam) @ y
        J[m, :m] = v.conj()
        d = np.linalg.solve(J, -F)
        y = y + d[:m]
        lam = lam + d[m]
    return lam, y


def solve_reduced(terms, Ahat, contour):
    """All approximate eigenpairs (lambda, y) of sum_j f_j(lambda) Ahat_j y = 0
    (Algorithm 1, Step 1).  Returns (lam, Y, polished) where polished marks pairs
    that went through Newton (non-polynomial case only)."""
    if all(k == "pow" for k, _ in terms):
        k = max(int(p) for _, p in terms)
        coeffs = [np.zeros_like(Ahat[0]) for _ in range(k + 1)]
        for (_, p), Aj in zip(terms, Ahat):
            coeffs[int(p)] = coeffs[int(p)] + Aj
        lam, Y = _poly_eigs(coeffs)
        return lam, Y
    rho = 1.5 * max(contour.a, contour.b)
    d = taylor_degree(terms, rho)
    B = reduced_coeffs_about(terms, Ahat, contour.c, d)
    mu, Y = _poly_eigs(B)
    return contour.c + mu, Y


def select(lam, contour, m0):
    """Indices of the m0 eigenvalues closest to the interior of C (Algorithm 1 Step 2):
    ascending normalised radius, stable in the index, infinite last."""
    r = contour.radius(lam)
    order = np.argsort(r, kind="stable")
    return order[:m0]


CONTOUR_SCALE = 1.5      # enlargement of C for the reduced contour-integral solve
CONTOUR_POINTS = 96      # trapezoid points on the enlarged ellipse
CONTOUR_RANK_TOL = 1e-10  # singular values below this fraction of the integrand's size are noise


def contour_eigs(terms, Ahat, contour, scale=CONTOUR_SCALE, npts=CONTOUR_POINTS,
                 rank_tol=CONTOUR_RANK_TOL):
    """Eigenpairs of sum_j f_j(lambda) Ahat_j y = 0 inside the ellipse C scaled by `scale`,
    by the moments of the resolvent (Sec. 3 eq. cauchymoments; Beyn's method with block
    Hankel moments).  By Keldysh's theorem T^{-1}(z) = sum_i v_i w_i^H / (z - lambda_i) + an
    analytic part inside the ellipse, so M_p = (1/2 pi i) oint mu(z)^p T^{-1}(z) dz equals
    V mu(Lambda)^p W^H; the Hankel matrices H0 = [M_{i+j}], H1 = [M_{i+j+1}] then factor as
    Vb W^H and Vb mu(Lambda) W^H with Vb = [V; V mu; ...], and the SVD H0 = U S Z^H gives
    U^H H1 Z S^{-1} = (U^H Vb) mu(Lambda) (U^H Vb)^{-1}.  Returns (lam, Y), Y with unit columns
    (the first block of U s_i).  The numerical rank counts the singular values above
    rank_tol times the size of the integrand, sum_q |w_q| ||T^{-1}(z_q)||_F (with no eigenvalue
    inside, the moments are rounding noise of that size times the machine epsilon)."""
    m = Ahat[0].shape[0]
    c = complex(contour.c)
    a, b = contour.a * scale, contour.b * scale
    L = max(a, b)
    K_max = 3
    M = [np.zeros((m, m), dtype=complex) for _ in range(2 * K_max)]
    size = 0.0
    for q in range(npts):
        th = 2.0 * np.pi * (q + 0.5) / npts
        z = c + a * np.cos(th) + 1j * b * np.sin(th)
        dz = -a * np.sin(th) + 1j * b * np.cos(th)
        w = dz / (1j * npts)                 # (1/2 pi i) dz/dtheta (2 pi / npts)
        mu = (z - c) / L
        Tinv = np.linalg.solve(reduced_T(terms, Ahat, z), np.eye(m))
        size += abs(w) * np.linalg.norm(Tinv)
        for p in range(2 * K_max):
            M[p] += (w * mu ** p) * Tinv
    for K in (2, 3):
        H0 = np.block([[M[i + j] for j in range(K)] for i in range(K)])
        H1 = np.block([[M[i + j + 1] for j in range(K)] for i in range(K)])
        U, sv, Zh = np.linalg.svd(H0)
        k = int(np.sum(sv > rank_tol * size))
        if k < K * m:
            break
    else:
        raise RuntimeError("contour_eigs: the enlarged contour holds too many eigenvalues")
    if k == 0:
        return np.zeros(0, dtype=complex), np.zeros((m, 0), dtype=complex)
    Uk = U[:, :k]
    B = Uk.conj().T @ H1 @ Zh[:k].conj().T / sv[:k][None, :]
    mu_e, S = np.linalg.eig(B)
    lam = c + L * mu_e
    Y = (Uk @ S)[:m]
    Y = Y / np.linalg.norm(Y, axis=0)[None, :]
    return lam, Y


def contour_reduced(terms, Ahat, contour, m0, scale=CONTOUR_SCALE):
    """Steps 1-2 with the contour-integral reading: the pairs found inside the enlarged
    ellipse, Newton-polished on the exact reduced function and sorted by normalised radius
    (the m0 closest to the interior), completed to m0 when fewer were found.  Returns
    (lam, Y, found) with found[i] False for the completing pairs."""
    m = Ahat[0].shape[0]
    lam, Y = contour_eigs(terms, Ahat, contour, scale=scale)
    keep = contour.radius(lam) < scale
    lam, Y = lam[keep], Y[:, keep]
    for i in range(len(lam)):
        lam[i], y = newton_polish(terms, Ahat, lam[i], Y[:, i])
        Y[:, i] = y / np.linalg.norm(y)
    order = np.argsort(contour.radius(lam), kind="stable")[:m0]
    lam, Y = lam[order], Y[:, order]
    k = len(lam)
    found = np.ones(m0, dtype=bool)
    if k < m0:
        # unit vectors orthogonal to the pairs found: the trailing columns of a Householder QR
        # of [Y, I]
        Qc, _ = np.linalg.qr(np.concatenate([Y, np.eye(m, dtype=complex)], axis=1))
        pad = m0 - k
        th = 2.0 * np.pi * (np.arange(pad) + 0.5) / pad
        lam_pad = contour.c + scale * (contour.a * np.cos(th) + 1j * contour.b * np.sin(th))
        lam = np.concatenate([lam, lam_pad])
        Y = np.concatenate([Y, Qc[:, k:m0]], axis=1)
        found[k:] = False
    return lam, Y, found
