"""Algorithm 1 of Sec. 4.2 (NLFEAST for T(lambda) x = 0) in complex128: the oracle, test
infrastructure only.  `solve` runs the algorithm's Steps 0-5 in their order with the block
contour integral of eq. nlfeast_int evaluated by the quadrature sum of Step 4.

Choices where the paper leaves room:
* Ritz vectors are scaled to unit 2-norm, so the Step 3 residual is absolute and relative
  at once.
* A Ritz value counts as inside C when its normalised radius is below 1.
* Step 3 may stop only after Step 4 has run at least once, so the iteration count is the
  number of Step 4 executions (Example 1 converges "in three iterations" in this sense).
  The iteration cap defaults to 50; with no Ritz value inside after 3 iterations the result
  is empty.
* When m0 or more Ritz values are inside, the algorithm's precondition (fewer than m0
  eigenvalues inside C) does not hold and M0TooSmall is raised.
* Spurious Ritz values (Sec. 4.2 calls them Ritz pairs that match no eigenpair of the full
  problem): the projected problem has more eigenvalues than the subspace has dimensions, and
  an extra one can land inside C.  Its residual does not shrink from one iteration to the
  next, whereas the residual of a genuine pair shrinks by about the filter ratio
  |rho(lambda_out)| / |rho(lambda_i)| per iteration, rho(l) = sum_k omega_k / (z_k - l)
  being the rational filter of the quadrature and lambda_out the first eigenvalue the
  subspace leaves out.  From iteration 2 on, every Ritz value is paired with one of the
  previous iteration's (`match_previous`); an unconverged value inside is *stagnant* when its
  residual exceeds theta_i times its partner's (`stagnant`), with
  theta_i = min(0.97, max(0.25, (rho_min / |rho(lambda_i)|)^(1/3))), rho_min the smallest
  |rho| over the selected values (the farthest selected value bounds |rho(lambda_out)| from
  above; the cube root and the bounds leave a margin for a genuine pair).  Step 3 then stops
  when at least one pair inside has converged and every other value inside is stagnant; the
  stagnant ones are returned flagged as spurious.
* Step 4 uses the quadrature sum exactly as the paper writes it; every T(z_j) is factored
  once (the shifts are fixed) by LU with partial pivoting (scipy lu_factor).
* Steps 0 and 5 orthonormalise by Householder QR (numpy.linalg.qr).
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


def match_previous(lam, prev):
    """Pair each current Ritz value with at most one of the previous iteration's: repeatedly
    take the closest unpaired pair (ties: lower current index, then lower previous index).
    Returns, per current value, the index of its partner or -1."""
    lam = np.asarray(lam, dtype=complex)
    prev = np.asarray(prev, dtype=complex)
    with np.errstate(invalid="ignore"):
        d = np.abs(lam[:, None] - prev[None, :])
    d = np.where(np.isfinite(d), d, np.inf)
    partner = -np.ones(len(lam), dtype=np.int64)
    used = np.zeros(len(prev), dtype=bool)
    for f in np.argsort(d, axis=None, kind="stable"):
        i, j = divmod(int(f), len(prev))
        if not np.isfinite(d[i, j]):
            break
        if partner[i] < 0 and not used[j]:
            partner[i] = j
            used[j] = True
    return partner


def stagnant(lam, res, unconv, rho, prev_lam, prev_res):
    """Mask of the unconverged values inside C (`unconv`) whose residual did not shrink by
    the factor a genuine pair reaches (module docstring).  rho: |rho(lambda_i)| of every
    selected value (0 for infinite ones)."""
    finite = np.isfinite(lam)
    rho_min = float(np.min(rho[finite])) if finite.any() else 0.0
    partner = match_previous(lam, prev_lam)
    out = np.zeros(len(lam), dtype=bool)
    for i in np.flatnonzero(unconv):
        theta = min(0.97, max(0.25, (rho_min / max(rho[i], 1e-300)) ** (1.0 / 3.0)))
        before = prev_res[partner[i]] if partner[i] >= 0 else 0.0
        out[i] = not (res[i] <= theta * before)
    return out


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
    prev = None
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
        if it >= 2 and prev is not None and n_in > n_in - int(unconv.sum()) > 0:
            rho = np.array([abs(np.sum(omega / (z - l))) if np.isfinite(l) else 0.0 for l in lam])
            stag = stagnant(lam, res, unconv, rho, prev[0], prev[1])
            history[-1]["n_stagnant"] = int(stag.sum())
            if np.all(stag[unconv]):
                return Result(lam, X, res, inside, it, history, True, spurious=stag)
        prev = (lam.copy(), res.copy())
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
