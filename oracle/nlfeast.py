"""Algorithm 1 (NLFEAST for T(lambda) x = 0), literally, in complex128 (oracle; test
infrastructure only).

    Step 0  Q = X0, orthonormalise its columns.
    Step 1  solve the projected problem Q^H T(lambda) Q y = 0.
    Step 2  keep the m0 pairs closest to the interior of C: Lambda = diag(lambda_i),
            X = [Q y_1, ..., Q y_m0].
    Step 3  stop if ||T(lambda_i) Q y_i|| <= eps for every lambda_i inside C.
    Step 4  Q = sum_j omega_j (X - T(z_j)^{-1} T(X, Lambda)) (z_j I - Lambda)^{-1}.
    Step 5  orthonormalise Q (QR) and go to Step 1.

(Sec. 4.2, Algorithm 1 and the block contour integral eq. nlfeast_int.)

Readings where the paper is silent:
* Ritz vectors are normalised, ||x_i||_2 = 1, so the Step 3 residual is absolute and
  relative at once.
* "inside C" is strictly inside (normalised radius < 1).
* Step 3 is checked only after at least one Step 4 (iterations = number of Step 4
  executions, as in "converges in three iterations" of Example 1); with no Ritz value
  inside after 3 iterations the result is empty; the iteration cap defaults to 50.
* if m0 or more Ritz values lie inside, the precondition of Algorithm 1 (fewer than m0
  eigenvalues inside C) is violated and M0TooSmall is raised.
* spurious Ritz values: with m0 well above the count, a Ritz value of the projected problem
  can sit inside C without approximating any eigenvalue (the projected problem has more
  eigenvalues than the subspace has dimensions); its residual stays large while the true
  pairs converge.  Step 3 then also stops when, at iteration it >= 4, the number of
  converged inside pairs is the same positive number as in each of the three previous
  iterations and the largest residual among the unconverged inside pairs is at least half of
  its value three iterations earlier; the unconverged inside pairs are reported as
  spurious (eigenvalues: the converged inside pairs only).
* Step 4 uses the literal sum of the paper; T(z_j) is factored once per contour
  (the shifts are fixed) by LU with partial pivoting (scipy lu_factor).
* Step 0/5 orthonormalisation is Householder QR (numpy.linalg.qr).
"""
import time

import numpy as np
import scipy.linalg

from .reduced import solve_reduced, select, newton_polish, contour_reduced


class M0TooSmall(RuntimeError):
    pass


class Result:
    def __init__(self, lam, X, res, inside, iters, history, converged, spurious=None):
        self.lam = lam
        self.X = X
        self.res = res
        self.inside = inside
        self.iters = iters
        self.history = history
        self.converged = converged
        self.spurious = np.zeros_like(inside) if spurious is None else spurious

    @property
    def eigenvalues(self):
        return self.lam[self.inside & ~self.spurious]


def stalled(history):
    """The stopping rule for spurious Ritz values (module docstring)."""
    if len(history) < 5:
        return False
    h = history[-4:]
    n = h[-1]["n_conv"]
    return n > 0 and all(x["n_conv"] == n for x in h) and h[-1]["max_unconv"] >= 0.5 * h[0]["max_unconv"]


def orthonormalise(Q):
    """Steps 0 and 5: Householder QR, keep the orthonormal factor."""
    q, _ = np.linalg.qr(Q)
    return q


def step4(factors, X, R, lam, z, omega):
    """Step 4: Q = sum_j omega_j (X - T(z_j)^{-1} T(X, Lambda)) (z_j I - Lambda)^{-1},
    with R = T(X, Lambda) and factors the LU factors of T(z_j)."""
    Q = np.zeros(X.shape, dtype=complex)
    for zj, wj, fac in zip(z, omega, factors):
        Yj = scipy.linalg.lu_solve(fac, R, check_finite=False)
        Q += wj * (X - Yj) / (zj - lam)[None, :]
    return Q


def solve(problem, contour, z, omega, X0, m0, tol, max_iter=50, factors=None,
          verbose=False, reduced="auto"):
    """Run Algorithm 1.  problem: oracle.problem.Problem; contour: quadrature.Contour;
    (z, omega): quadrature; X0: n x m0 initial guess.  Returns a Result whose arrays
    are sorted by Step 2's selection order.  reduced: 'auto' (linearisation, with the
    Taylor reading for 'exp' terms and the contour-integral reading when a term is a
    caller-supplied function) or 'contour' (the contour-integral reading for every
    non-polynomial problem)."""
    use_contour = problem.has_user_terms or (reduced == "contour" and not problem.is_polynomial)
    n = problem.n
    X0 = np.asarray(X0, dtype=complex)
    if X0.shape != (n, m0):
        raise ValueError("X0 must be n x m0")
    # fixed shifts: factor every T(z_j) once
    if factors is None:
        factors = [scipy.linalg.lu_factor(problem.T(zj), check_finite=False) for zj in z]
    Q = orthonormalise(X0)                                   # Step 0
    history = []
    it = 0
    while True:
        Ahat = problem.project(Q)                            # Step 1
        if use_contour:                                      # Steps 1-2, contour reading
            lam, Y, _ = contour_reduced(problem.terms, Ahat, contour, m0)
        else:
            lam_all, Y_all = solve_reduced(problem.terms, Ahat, contour)
            sel = select(lam_all, contour, m0)               # Step 2
            lam = lam_all[sel].astype(complex)
            Y = Y_all[:, sel]
            if not problem.is_polynomial:
                for i in range(m0):
                    if np.isfinite(lam[i]):
                        lam[i], Y[:, i] = newton_polish(problem.terms, Ahat, lam[i], Y[:, i])
        X = Q @ Y
        X = X / np.linalg.norm(X, axis=0)[None, :]
        finite = np.isfinite(lam)
        lam_f = np.where(finite, lam, 0.0)
        R = problem.block_residual(X, lam_f)                 # T(X, Lambda)
        res = np.linalg.norm(R, axis=0)
        res = np.where(finite, res, np.inf)
        inside = contour.inside(lam)
        n_in = int(inside.sum())
        unconv = inside & ~(res <= tol)
        history.append(dict(it=it, n_inside=n_in,
                            max_res=float(res[inside].max()) if n_in else 0.0,
                            n_conv=n_in - int(unconv.sum()),
                            max_unconv=float(res[unconv].max()) if unconv.any() else 0.0))
        if verbose:
            print("it %d inside %d max_res %.3e" % (it, n_in, history[-1]["max_res"]))
        if n_in >= m0:
            raise M0TooSmall("%d Ritz values inside C with m0 = %d" % (n_in, m0))
        if it >= 1 and n_in > 0 and np.all(res[inside] <= tol):   # Step 3
            return Result(lam, X, res, inside, it, history, True)
        if it >= 4 and stalled(history):
            return Result(lam, X, res, inside, it, history, True, spurious=unconv)
        if it >= 3 and n_in == 0:
            return Result(lam, X, res, inside, it, history, True)
        if it >= max_iter:
            return Result(lam, X, res, inside, it, history, False)
        Q = orthonormalise(step4(factors, X, R, lam_f, z, omega))   # Steps 4, 5
        it += 1


def adjoint_problem(problem):
    """S(mu) = T(conj mu)^H = sum_j conj(f_j(conj mu)) A_j^H: y^H T(lambda) = 0 (the left
    eigenvectors of Sec. 2 eq. NLEVP) is S(conj lambda) y = 0.  For 'pow' and 'exp' terms,
    whose parameters are real, conj(f(conj mu)) = f(mu)."""
    from .problem import Problem, ScalarFunction
    terms = []
    for k, p in problem.terms:
        if k == "fn":
            terms.append(("fn", ScalarFunction(lambda mu, F=p: np.conj(F.f(np.conj(mu))),
                                               lambda mu, F=p: np.conj(F.df(np.conj(mu))),
                                               "adjoint of %s" % p.name)))
        else:
            terms.append((k, p))
    return Problem(terms, [A.conj().T for A in problem.mats])


def solve_left(problem, contour, nc, Y0, m0, tol, rule="gauss", max_iter=50, reduced="auto",
               verbose=False):
    """Left eigenpairs of T inside C: Algorithm 1 applied to the adjoint function S on the
    conjugate contour, with that contour's own quadrature, and the eigenvalues conjugated back
    (so they are T's).  Returns a Result whose X holds the left eigenvectors y (unit norm),
    res the values ||T(lambda_i)^H y_i||."""
    from .quadrature import Contour, nodes_weights
    Cc = Contour(np.conj(contour.c), contour.a, contour.b)
    z, w = nodes_weights(Cc, nc, rule)
    r = solve(adjoint_problem(problem), Cc, z, w, Y0, m0, tol, max_iter=max_iter, verbose=verbose,
              reduced=reduced)
    r.lam = np.conj(r.lam)
    return r


def timed_solve(*args, **kw):
    t0 = time.perf_counter()
    r = solve(*args, **kw)
    return r, time.perf_counter() - t0
