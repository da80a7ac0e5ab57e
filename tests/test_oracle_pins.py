"""Pins of the CPU oracle to facts fixed by the paper and by mathematics, not by the
oracle itself: closed-form spectra (mass-spring QEPs of Sec. 5), values printed in the
paper (Table 1), closed forms of the quadrature filter, the reduction of Step 4 to the
linear FEAST filter for a linear pencil (Sec. 4.2), brute-force companion eigenvalues,
and a known-spectrum non-polynomial family."""
import json
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import workloads as wl
from oracle import brute, dense, nlfeast, nlfeast as onl, problem as pb, quadrature as qd, reduced

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def mass_spring_closed_form(n, tau, kappa):
    """Eigenvalues of lambda^2 I + lambda tau T3 + kappa T3, T3 = tridiag(-1, 3, -1):
    T3 has eigenvalues mu_j = 3 - 2 cos(j pi / (n + 1)) with the same eigenvectors for
    all three coefficients, so each mu_j gives the scalar quadratic
    lambda^2 + tau mu_j lambda + kappa mu_j = 0."""
    j = np.arange(1, n + 1)
    mu = 3.0 - 2.0 * np.cos(j * np.pi / (n + 1))
    disc = np.sqrt((tau * mu) ** 2 - 4.0 * kappa * mu + 0j)
    return np.concatenate([(-tau * mu + disc) / 2.0, (-tau * mu - disc) / 2.0])


def load_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_ex1.txt")) if l.strip() and not l.startswith("#")]
    return np.array([float(r[1]) for r in rows]), np.array([float(r[2]) for r in rows])


def match_error(a, b, scale):
    """Largest |a_i - b_pi(i)| / scale over the optimal one-to-one matching."""
    from scipy.optimize import linear_sum_assignment
    a = np.asarray(a)
    b = np.asarray(b)
    assert len(a) == len(b)
    if len(a) == 0:
        return 0.0
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return float(np.max(cost[r, c]) / scale)


# ---------------------------------------------------------------- quadrature

@pytest.mark.parametrize("nc", [4, 8, 16, 24])
def test_gauss_filter_is_one_at_centre(nc):
    # on a circle omega_k / (z_k - c) = w_k / 2, and the Legendre weights sum to 2
    C = qd.Contour(0.3 - 0.2j, 0.7)
    z, w = qd.nodes_weights(C, nc)
    assert abs(qd.filter_value(z, w, C.c) - 1.0) < 1e-14


@pytest.mark.parametrize("nc", [4, 8, 16])
def test_trapezoid_filter_closed_form(nc):
    # nodes at the nc-th roots of -1 give rho(lambda) = 1 / (1 + mu^nc), mu = (lambda-c)/r
    C = qd.Contour(1.0 + 1.0j, 2.0)
    z, w = qd.nodes_weights(C, nc, rule="trapezoid")
    rng = np.random.default_rng(5)
    lam = C.c + 2.0 * (rng.uniform(-1.5, 1.5, 20) + 1j * rng.uniform(-1.5, 1.5, 20))
    mu = (lam - C.c) / 2.0
    assert np.max(np.abs(qd.filter_value(z, w, lam) - 1.0 / (1.0 + mu ** nc))) < 1e-12


@pytest.mark.parametrize("shape,nc", [((0.0, 1.0, 1.0), 64), ((-1.55, 0.05, 0.0035), 512),
                                      ((2 + 1j, 0.5, 2.0), 256)])
def test_weights_against_adaptive_integration(shape, nc):
    # sum_k omega_k g(z_k) for g(z) = z^2 / (z - lam) vs adaptive integration of the
    # parametrised contour integral (independent of the Legendre rule)
    c, a, b = shape
    C = qd.Contour(c, a, b)
    lam = C.c + 0.3 * a + 0.2j * b
    z, w = qd.nodes_weights(C, nc)
    g = lambda zz: zz ** 2 / (zz - lam)
    approx = np.sum(w * g(z))

    def integrand(t, part):
        v = g(C.point(t)) * C.dpoint(t) / (2j * np.pi)
        return v.real if part == 0 else v.imag

    ref = sum(s * scipy.integrate.quad(integrand, 0, 2 * np.pi, args=(p,), limit=400, epsabs=1e-14)[0]
              for p, s in ((0, 1), (1, 1j)))
    # residue theorem: the integral equals lam^2 (lam inside)
    assert abs(ref - lam ** 2) < 1e-9 * max(1, abs(lam) ** 2)
    assert abs(approx - ref) < 1e-8 * max(1, abs(ref))


def test_inside_is_strict():
    C = qd.Contour(0.0, 2.0, 1.0)
    assert not C.inside(2.0 + 0j)
    assert C.inside(1.999 + 0j)
    assert not C.inside(np.inf)


# ---------------------------------------------------------------- brute force

def test_companion_matches_mass_spring_closed_form():
    terms, mats = wl.mass_spring(60, 0.6202, 0.4807)
    lam = brute.companion_eigs(pb.Problem(terms, mats))
    ref = mass_spring_closed_form(60, 0.6202, 0.4807)
    assert match_error(lam, ref, 1.0) < 1e-12


def test_table1_is_the_closed_form():
    # the printed Table 1 (10 digits) agrees with the closed form to its rounding
    tab, _ = load_table1()
    ref = mass_spring_closed_form(1000, 0.6202, 0.4807)
    C = qd.Contour(-1.55, 0.05, 0.0035)
    inside = ref[C.inside(ref)]
    assert len(inside) == 20
    assert np.max(np.abs(np.sort(inside.real) - np.sort(tab))) < 6e-11
    assert np.max(np.abs(inside.imag)) == 0.0


def test_shift_invert_near_matches_full_companion():
    terms, mats = wl.random_qep(80, 11)
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)
    sigma = full[17] + 0.01
    near = brute.companion_eigs_near(P, sigma, 12)
    ref = full[np.argsort(np.abs(full - sigma))[:12]]
    assert match_error(near, ref, 1.0) < 1e-11


def test_winding_count_matches_companion():
    terms, mats = wl.random_qep(40, 12)
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)
    C = qd.Contour(full[3], 0.4)
    assert brute.winding_count(P, C) == int(C.inside(full).sum())


# ---------------------------------------------------------------- reduced solve

def test_companion_first_general_degree():
    rng = np.random.default_rng(3)
    coeffs = [wl.cn(rng, (5, 5)) for _ in range(4)]       # cubic
    lam, Y = reduced._poly_eigs(coeffs)
    assert len(lam) == 15
    for l, y in zip(lam, Y.T):
        P = sum(l ** i * c for i, c in enumerate(coeffs))
        s = np.linalg.svd(P, compute_uv=False)
        assert s[-1] < 1e-10 * s[0]
        assert np.linalg.norm(P @ y) < 1e-9 * s[0] * np.linalg.norm(y)


def test_taylor_coeffs_sum_to_function():
    for kind, p in (("pow", 3), ("pow", 0), ("exp", 1.7)):
        t = pb.taylor_coeffs(kind, p, 0.3 + 0.4j, 20)
        mu = 0.05 - 0.02j
        approx = sum(t[q] * mu ** q for q in range(21))
        exact = pb.f_eval(kind, p, 0.3 + 0.4j + mu)
        assert abs(approx - exact) < 1e-15 * max(1, abs(exact))


def test_select_orders_by_normalised_radius():
    C = qd.Contour(0.0, 2.0, 1.0)
    lam = np.array([3.0, 0.5j, np.inf, 1.0, 0.9j, 1.0])
    assert list(reduced.select(lam, C, 6)) == [1, 3, 5, 4, 0, 2]   # radii .5 .5 .5 .9 1.5 inf


# ---------------------------------------------------------------- Step 4

def test_step4_is_linear_feast_filter_for_a_pencil():
    # T(lambda) = lambda I - D: X - T^{-1}(z) T(X, Lambda) = (zI - D)^{-1} X (zI - Lambda),
    # so Step 4 gives Q = rho(D) X for every Lambda off the nodes (Sec. 4.2: the
    # nonlinear integral reduces to the linear FEAST one for a linear pencil)
    rng = np.random.default_rng(4)
    n, m = 30, 6
    d = wl.cn(rng, n)
    P = pb.Problem([("pow", 1), ("pow", 0)], [np.eye(n), -np.diag(d)])
    C = qd.Contour(0.1, 0.9)
    z, w = qd.nodes_weights(C, 12)
    X = wl.cn(rng, (n, m))
    lam = wl.cn(rng, m)
    R = P.block_residual(X, lam)
    facs = [scipy.linalg.lu_factor(P.T(zk)) for zk in z]
    Q = nlfeast.step4(facs, X, R, lam, z, w)
    rho = qd.filter_value(z, w, d)
    assert np.max(np.abs(Q - rho[:, None] * X)) < 1e-12 * np.max(np.abs(X))


def test_step4_fixed_point_at_exact_eigenpairs():
    # exact eigenpairs give T(X, Lambda) = 0 and Q = X rho(Lambda)
    terms, mats = wl.mass_spring(40, 0.6202, 0.4807)
    P = pb.Problem(terms, mats)
    j = np.arange(1, 41)
    V = np.sin(np.outer(j, j) * np.pi / 41)          # eigenvectors of T3
    lam = mass_spring_closed_form(40, 0.6202, 0.4807)[:40]
    X = V / np.linalg.norm(V, axis=0)
    R = P.block_residual(X.astype(complex), lam)
    assert np.max(np.linalg.norm(R, axis=0)) < 1e-13
    C = qd.Contour(-0.5, 1.0)
    z, w = qd.nodes_weights(C, 8)
    facs = [scipy.linalg.lu_factor(P.T(zk)) for zk in z]
    Q = nlfeast.step4(facs, X, R, lam, z, w)
    assert np.max(np.abs(Q - X * qd.filter_value(z, w, lam)[None, :])) < 1e-11


# ---------------------------------------------------------------- dense steps

def test_lu_partial_pivot_definition():
    rng = np.random.default_rng(6)
    A = wl.cn(rng, (40, 40))
    LU, ipiv = dense.lu_partial_pivot(A)
    L = np.tril(LU, -1) + np.eye(40)
    U = np.triu(LU)
    assert np.max(np.abs(dense.apply_pivots(ipiv, A) - L @ U)) < 1e-13
    assert np.max(np.abs(L)) <= np.sqrt(2.0) + 1e-15        # |l| <= sqrt 2 with |Re|+|Im| pivots
    lu2, piv2 = scipy.linalg.lu_factor(A)
    assert np.array_equal(ipiv, piv2)                        # same pivot choices as LAPACK
    assert np.max(np.abs(LU - lu2)) < 1e-12
    B = wl.cn(rng, (40, 3))
    assert np.max(np.abs(dense.lu_solve(LU, ipiv, B) - np.linalg.solve(A, B))) < 1e-11


def test_assemble_hand_checked_2x2():
    # T(z) = z^2 A2 + z A1 + A0 + exp(-z/2) E with each A_j a single unit entry, so T(z) is
    # [[z^2, z], [1, exp(-z/2)]]; at z = 1 + 2i: z^2 = -3 + 4i and
    # exp(-1/2 - i) = e^{-1/2} (cos 1 - i sin 1) = 0.6065306597 (0.5403023059 - 0.8414709848 i)
    # = 0.3277099140 - 0.5103779515 i
    unit = lambda i, j: np.eye(2, dtype=complex)[:, [i]] @ np.eye(2, dtype=complex)[[j], :]
    terms = [("pow", 2), ("pow", 1), ("pow", 0), ("exp", 0.5)]
    mats = [unit(0, 0), unit(0, 1), unit(1, 0), unit(1, 1)]
    T1, T2 = dense.assemble(terms, mats, [1 + 2j, -1.0])
    assert T1[0, 0] == -3 + 4j and T1[0, 1] == 1 + 2j and T1[1, 0] == 1.0
    assert abs(T1[1, 1] - (0.3277099140 - 0.5103779515j)) < 1e-10
    assert T2[0, 0] == 1.0 and T2[0, 1] == -1.0 and T2[1, 0] == 1.0
    assert abs(T2[1, 1] - 1.6487212707) < 1e-10              # e^{1/2}


def test_project_on_the_sine_eigenvectors():
    # the mass-spring coefficients I, tau T3, kappa T3 share T3's orthonormal sine
    # eigenvectors q_j(i) = sqrt(2/(n+1)) sin(i j pi/(n+1)) with T3 q_j = mu_j q_j,
    # mu_j = 3 - 2 cos(j pi/(n+1)): on them the projections are diagonal
    n, tau, kappa = 50, 0.6202, 0.4807
    terms, mats = wl.mass_spring(n, tau, kappa)
    i = np.arange(1, n + 1)
    cols = np.array([1, 4, 9, 30, 50])
    Q = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, cols) * np.pi / (n + 1))
    mu = 3.0 - 2.0 * np.cos(cols * np.pi / (n + 1))
    A2, A1, A0 = dense.project(mats, Q.astype(complex))
    assert np.max(np.abs(A2 - np.eye(5))) < 1e-13
    assert np.max(np.abs(A1 - np.diag(tau * mu))) < 1e-13
    assert np.max(np.abs(A0 - np.diag(kappa * mu))) < 1e-13


def test_block_residual_on_the_sine_eigenvectors():
    # T(l) q_j = p_j(l) q_j with p_j(l) = l^2 + tau mu_j l + kappa mu_j: zero at the roots,
    # and |p_j(l)| (times ||q_j|| = 1) at any other l
    n, tau, kappa = 40, 0.6202, 0.4807
    terms, mats = wl.mass_spring(n, tau, kappa)
    i = np.arange(1, n + 1)
    cols = np.array([2, 7, 19, 33])
    Q = (np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, cols) * np.pi / (n + 1))).astype(complex)
    mu = 3.0 - 2.0 * np.cos(cols * np.pi / (n + 1))
    disc = np.sqrt((tau * mu) ** 2 - 4.0 * kappa * mu + 0j)
    roots = (-tau * mu + disc) / 2.0
    R, norms = dense.block_residual(terms, mats, Q, roots)
    assert np.max(norms) < 1e-14
    shifted = roots + np.array([1e-3, 0.2j, -0.5, 1.0 + 1.0j])
    R, norms = dense.block_residual(terms, mats, Q, shifted)
    p = shifted ** 2 + tau * mu * shifted + kappa * mu
    assert np.max(np.abs(norms - np.abs(p)) / np.abs(p)) < 1e-12
    assert np.max(np.abs(R - Q * p[None, :])) < 1e-14


def test_step4_sum_is_the_trapezoid_filter_on_a_diagonal_pencil():
    # T(l) = l I - diag(d): the solves are Y_k = (z_k - d)^{-1} (l - d) X exactly, and the
    # quadrature sum reduces to Q = diag(rho(d)) X, where for the n_c-point trapezoid rule on a
    # circle rho(mu) = 1 / (1 + ((mu - c)/r)^{n_c}) in closed form
    rng = np.random.default_rng(31)
    n, m, nc = 24, 5, 8
    c, r = 0.3 - 0.2j, 0.7
    d = c + r * rng.uniform(0.2, 1.8, n) * np.exp(2j * np.pi * rng.uniform(size=n))
    X = wl.cn(rng, (n, m))
    lam = c + 0.5 * r * wl.cn(rng, m)
    z, w = qd.nodes_weights(qd.Contour(c, r), nc, "trapezoid")
    solves = [((lam[None, :] - d[:, None]) / (zk - d)[:, None]) * X for zk in z]
    Q = dense.step4_sum(X, solves, lam, z, w)
    rho = 1.0 / (1.0 + ((d - c) / r) ** nc)
    assert np.max(np.abs(Q - rho[:, None] * X)) < 1e-12 * np.max(np.abs(X))


def test_refine_eigenvalue_returns_to_the_closed_form():
    # from 1e-4 away, four steps of two-sided Rayleigh functional iteration (the error roughly
    # squares per step: the x and y of each step are one inverse-iteration step from fixed
    # vectors) land on the exact mass-spring
    # eigenvalue, and the residual it reports is that of a unit vector at the final value
    n, tau, kappa = 60, 0.6202, 0.4807
    terms, mats = wl.mass_spring(n, tau, kappa)
    P = pb.Problem(terms, mats)
    exact = mass_spring_closed_form(n, tau, kappa)
    for lam in exact[[3, 41, 70]]:
        l, res = brute.refine_eigenvalue(P, lam + 1e-4 * (1 + 1j), steps=4)
        assert abs(l - lam) < 1e-13 * max(abs(lam), 1.0)
        assert res < 1e-13
    # the certificate is an upper bound of the smallest singular value, and a tight one
    far = exact[5] + 1e-3
    smin = np.linalg.svd(P.T(far), compute_uv=False)[-1]
    res = brute.eigen_residual(P, far)
    assert smin * (1 - 1e-10) <= res < 1.01 * smin


def test_eigs_near_on_a_known_spectrum_delay_problem():
    # the delay family U diag(p_i(l)) V^H has the scalar roots of p_i as its eigenvalues: the
    # Taylor-surrogate Arnoldi route returns the nearest ones
    c, rad = 0.4 + 0.6j, 0.3
    terms, mats, (b, cc, e) = known_spectrum_delay(40, 21, c, rad, 6)
    big = qd.Contour(c, 4.0 * rad)
    truth = []
    for i in range(40):
        truth += scalar_roots_inside(b[i], cc[i], e[i], big)
    truth = np.array(truth)
    truth = truth[np.argsort(np.abs(truth - c))][:8]
    near = brute.eigs_near(pb.Problem(terms, mats), c, 8, 1.5 * np.max(np.abs(truth - c)))
    assert match_error(near, truth, 1.0) < 1e-10


def test_deflated_winding_count_equals_the_plain_count():
    # the count does not depend on the deflation points: exact, partial and displaced sets
    # all give the companion count
    terms, mats = wl.random_qep(40, 12)
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)
    C = qd.Contour(full[3], 0.5)
    inside = full[C.inside(full)]
    want = len(inside)
    assert want >= 4
    assert brute.winding_count(P, C) == want
    assert brute.winding_count(P, C, npts=64, deflate=inside) == want
    assert brute.winding_count(P, C, npts=64, deflate=inside[:2]) == want
    assert brute.winding_count(P, C, npts=64, deflate=np.append(inside + 0.02, C.c + 0.3j)) == want


def test_winding_trend_keeps_the_count():
    # an entire zero-free factor exp(-p(z)) taken out of the phase changes no winding: any
    # trend coefficients give the companion count; the fitted ones agree with the exact slope
    terms, mats = wl.random_qep(40, 12)
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)
    C = qd.Contour(full[3] + 0.07 - 0.04j, 0.5)    # centre off the spectrum (T(c) regular)
    inside = full[C.inside(full)]
    want = len(inside)
    assert want >= 4
    # a trend whose own phase swings a few radians along C: the samples still resolve it
    assert brute.winding_count(P, C, npts=64, trend=(0.8 - 0.4j, -1.0 + 0.5j, 2.0j)) == want
    assert brute.winding_count(P, C, npts=64, deflate=inside, trend=(3.0, 0.0, -6.0 + 1.0j)) == want
    tr = brute.phase_trend(P, C.c, 0.05 * C.a, deflate=inside)
    # log det T(z) - sum log(z - mu) for the companion eigenvalues is log det C_k (a constant),
    # so with every eigenvalue deflated the slope of log g at the centre is that of the ones
    # outside C: compare with the exact sum over the full companion spectrum
    outside = full[~C.inside(full)]
    assert abs(tr[0] - np.sum(1.0 / (C.c - outside))) < 1e-8 * max(1.0, abs(tr[0]))
    assert brute.winding_count(P, C, npts=8, deflate=inside, trend=tr) == want


def test_winding_trend_removes_aliasing_on_a_delay_problem():
    # the exponential terms of a delay problem give log det T a slope of order n: with the stored
    # delay512 eigenvalues deflated, eight coarse samples along the stored circle still alias
    # unless the fitted trend is taken out; with it, the coarse count equals the stored count
    # (the plain winding number of det T at 256 samples, no deflation)
    terms, mats = wl.make_problem("delay512")
    P = pb.Problem(terms, mats)
    g = json.load(open(os.path.join(GOLDEN, "contours.json")))["delay512"]["regions"][0]
    c, r = complex(*g["centre"]), g["radius"]
    C = qd.Contour(c, r)
    mu = np.array([complex(*v) for v in g["eigenvalues"]])
    tr = brute.phase_trend(P, c, 0.05 * r, deflate=mu)
    assert abs(tr[0]) * r > 5.0                      # the linear trend alone is several turns
    assert brute.winding_count(P, C, npts=8, max_step=0.8, deflate=mu, trend=tr) == g["winding_count"] == 12
    # the same count from a displaced deflation set (exactness does not rest on the stored values)
    assert brute.winding_count(P, C, npts=8, max_step=0.8, deflate=mu[:9] + 1e-3, trend=tr) == 12


def test_lu_pivot_convention_small():
    A = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 10]], dtype=complex)
    _, ipiv = dense.lu_partial_pivot(A)
    assert list(ipiv) == [2, 2, 2]


# ---------------------------------------------------------------- full Algorithm 1

def test_example1_reproduces_table1():
    terms, mats = wl.mass_spring(1000, 0.6202, 0.4807)
    P = pb.Problem(terms, mats)
    C = qd.Contour(-1.55, 0.05, 0.0035)
    z, w = qd.nodes_weights(C, 16)
    r = nlfeast.solve(P, C, z, w, wl.initial_block(1000, 22, 2101), 22, 1e-10)
    tab, _ = load_table1()
    assert r.converged and r.inside.sum() == 20
    assert np.max(np.abs(np.sort(r.eigenvalues.real) - np.sort(tab))) < 6e-11
    assert np.max(r.res[r.inside]) <= 1e-10
    assert r.iters <= 6            # the paper reports 3; the count depends on X0


def test_example2_overdamped():
    # the printed radius r = 19 encloses 34 eigenvalues (> m0 = 25); the half-width of
    # the interval (-30, -11), r = 9.5, encloses the 19 the paper reports
    terms, mats = wl.mass_spring(50, 10.0, 5.0)
    ref = mass_spring_closed_form(50, 10.0, 5.0)
    assert qd.Contour(-20.5, 19.0).inside(ref).sum() == 34
    C = qd.Contour(-20.5, 9.5)
    assert C.inside(ref).sum() == 19
    z, w = qd.nodes_weights(C, 8)
    r = nlfeast.solve(pb.Problem(terms, mats), C, z, w, wl.initial_block(50, 25, 2102), 25, 1e-10)
    assert r.converged and r.inside.sum() == 19
    assert match_error(r.eigenvalues, ref[C.inside(ref)], 20.5) < 1e-12


def test_random_qep_matches_companion():
    terms, mats = wl.random_qep(200, 1001)
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)
    C = qd.Contour(full[0] + 0.05, 0.35)
    k = int(C.inside(full).sum())
    assert 2 <= k < 20
    z, w = qd.nodes_weights(C, 8)
    r = nlfeast.solve(P, C, z, w, wl.initial_block(200, 20, 2001), 20, 1e-12)
    assert r.converged and r.inside.sum() == k
    assert match_error(r.eigenvalues, full[C.inside(full)], 0.35) < 1e-10
    assert np.max(r.res[r.inside]) <= 1e-12


def test_m0_too_small_raises():
    terms, mats = wl.mass_spring(50, 10.0, 5.0)
    C = qd.Contour(-20.5, 19.0)                   # 34 inside
    z, w = qd.nodes_weights(C, 8)
    with pytest.raises(nlfeast.M0TooSmall):
        nlfeast.solve(pb.Problem(terms, mats), C, z, w, wl.initial_block(50, 25, 5), 25, 1e-10, max_iter=8)


def known_spectrum_delay(n, seed, centre, radius, n_in):
    """T(lambda) = U diag(p_i(lambda)) V^H with p_i = lambda^2 + b_i lambda + c_i +
    e_i exp(-lambda), U, V unitary.  det T = det(U V^H) prod p_i, so the eigenvalues are
    the roots of the scalar p_i.  c_i is set so that p_i has a root at a chosen s_i;
    the first n_in roots are placed inside the circle, the rest outside."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(wl.cn(rng, (n, n)))
    V, _ = np.linalg.qr(wl.cn(rng, (n, n)))
    ang = rng.uniform(0, 2 * np.pi, n)
    rad = np.where(np.arange(n) < n_in, rng.uniform(0.0, 0.7, n), rng.uniform(1.4, 4.0, n)) * radius
    s = centre + rad * np.exp(1j * ang)
    b = wl.cn(rng, n) * 0.3
    e = 0.2 * wl.cn(rng, n)
    c = -(s ** 2 + b * s + e * np.exp(-s))
    mk = lambda d: (U * d[None, :]) @ V.conj().T
    mats = [mk(np.ones(n)), mk(b), mk(c), mk(e)]
    terms = [("pow", 2), ("pow", 1), ("pow", 0), ("exp", 1.0)]
    return terms, mats, (b, c, e)


def scalar_roots_inside(b, c, e, contour):
    """Roots of p(l) = l^2 + b l + c + e exp(-l) strictly inside the contour: Newton from
    a grid of starts, deduplicated, with the count checked by the scalar argument
    principle (1/2 pi i) oint p'/p dz."""
    p = lambda l: l ** 2 + b * l + c + e * np.exp(-l)
    dp = lambda l: 2 * l + b - e * np.exp(-l)
    th = np.linspace(0, 2 * np.pi, 4001)
    zz = contour.point(th)
    count = int(round(np.sum(np.diff(np.unwrap(np.angle(p(zz))))) / (2 * np.pi)))
    roots = []
    g = np.linspace(-1, 1, 15)
    for x in g:
        for y in g:
            l = contour.c + contour.a * x + 1j * contour.b * y
            for _ in range(60):
                l = l - p(l) / dp(l)
            if abs(p(l)) < 1e-13 and contour.inside(l) and all(abs(l - r) > 1e-8 for r in roots):
                roots.append(l)
    assert len(roots) == count
    return roots


def test_delay_known_spectrum():
    C = qd.Contour(0.4 + 0.6j, 0.3)
    terms, mats, (b, c, e) = known_spectrum_delay(40, 21, C.c, C.a, 6)
    truth = []
    for i in range(40):
        truth += scalar_roots_inside(b[i], c[i], e[i], C)
    assert len(truth) >= 6
    P = pb.Problem(terms, mats)
    z, w = qd.nodes_weights(C, 16)
    m0 = len(truth) + 6
    r = nlfeast.solve(P, C, z, w, wl.initial_block(40, m0, 22), m0, 1e-12)
    assert r.converged and r.inside.sum() == len(truth)
    assert match_error(r.eigenvalues, np.array(truth), C.a) < 1e-10


def test_match_previous_pairs_nearest_first():
    # greedy one-to-one pairing: 0.0 and 0.1 both prefer 0.05; 0.0 is closer (0.05 < ... ties go
    # to the lower current index) and takes it, 0.1 then takes 0.3; infinite values stay unpaired
    cur = np.array([0.0, 0.1, 5.0, np.inf])
    prev = np.array([0.3, 0.05, 4.0])
    assert list(onl.match_previous(cur, prev)) == [1, 0, 2, -1]
    assert list(onl.match_previous(np.array([1.0, 1.0]), np.array([1.0, 1.0]))) == [0, 1]


def test_stagnation_rule_thresholds():
    lam = np.array([0.0, 0.1, 0.5, 3.0])          # the last one is the farthest selected value
    prev_lam = lam + 1e-6
    rho = np.array([1.0, 1.0, 1.0, 1e-3])       # theta = (1e-3)^(1/3) = 0.1 -> floored to 0.25
    unconv = np.array([False, True, True, False])
    prev_res = np.array([1e-12, 1e-4, 1e-2, 1.0])
    res = np.array([1e-13, 0.2e-4, 0.3e-2, 1.0])  # 0.2 <= 0.25: contracting; 0.3 > 0.25: stagnant
    assert list(onl.stagnant(lam, res, unconv, rho, prev_lam, prev_res)) == [False, False, True, False]
    # a slow filter (rho_min close to rho_i) lets a slowly contracting genuine pair through
    rho_slow = np.array([1.0, 1.0, 1.0, 0.6])   # theta = 0.6^(1/3) = 0.84
    assert list(onl.stagnant(lam, res * np.array([1, 4, 2.5, 1]), unconv, rho_slow, prev_lam, prev_res)) == \
        [False, False, False, False]            # ratios 0.8 and 0.75
    # a value that appears from nowhere is paired with a converged one and counts as stagnant
    far = lam.copy()
    far[2] = 0.101
    assert onl.stagnant(far, res, unconv, rho, prev_lam, np.array([1e-12, 1e-4, 1e-12, 1.0]))[2]


def test_stagnation_rule_spares_slow_genuine_pairs():
    # m0 = 12 for the 10 eigenvalues of the n = 200 quadratic: the filter contracts slowly
    # (the first eigenvalue left out of the subspace sits just outside C), the iteration needs
    # many steps, and no genuine pair may be flagged as spurious on the way
    cfg = wl.CONFIGS["qep200"]
    terms, mats = wl.make_problem("qep200")
    g = json.load(open(os.path.join(GOLDEN, "contours.json")))["qep200"]["regions"][0]
    C = qd.Contour(complex(*g["centre"]), g["radius"])
    z, w = qd.nodes_weights(C, 8)
    r = onl.solve(pb.Problem(terms, mats), C, z, w, wl.initial_block(200, 12, 2001), 12, cfg["tol"],
                  max_iter=40)
    assert r.spurious.sum() == 0
    assert sum(h.get("n_stagnant", 0) > 0 for h in r.history) == 0
    ref = np.array([complex(*v) for v in g["eigenvalues"]])
    conv = r.inside & (r.res <= cfg["tol"])
    assert conv.sum() >= 5
    assert all(np.min(np.abs(ref - l)) < 1e-10 for l in r.lam[conv])


@pytest.mark.slow
def test_spurious_ritz_value_region_matches_brute_force():
    # qep2048x8 region 5 (m0 = 64, 40 eigenvalues inside, 16 trapezoid nodes): one Ritz value
    # of the projected quadratic problem stays inside C without converging; the iteration stops
    # by the stagnation rule in the iteration where the last genuine pair converges, and the
    # converged set is exactly the brute-force set
    from scipy.optimize import linear_sum_assignment
    cfg = wl.CONFIGS["qep2048x8"]
    terms, mats = wl.make_problem("qep2048x8")
    gs = json.load(open(os.path.join(GOLDEN, "contours.json")))["qep2048x8"]["regions"]
    ri = 4
    g = gs[ri]
    M = sum(x["m0"] for x in gs)
    col = sum(x["m0"] for x in gs[:ri])
    X0 = wl.initial_block(cfg["n"], M, 2000 + cfg["id"])[:, col:col + g["m0"]]
    C = qd.Contour(complex(*g["centre"]), g["radius"])
    z, w = qd.nodes_weights(C, cfg["nc"], "trapezoid")
    r = onl.solve(pb.Problem(terms, mats), C, z, w, X0, g["m0"], cfg["tol"], max_iter=30)
    ref = np.array([complex(*v) for v in g["eigenvalues"]])
    assert r.converged and r.spurious.sum() >= 1 and r.iters <= 7
    assert r.history[-2]["n_conv"] < len(g["eigenvalues"])      # stopped as soon as all converged
    ev = r.eigenvalues
    assert len(ev) == len(ref) == 40
    cost = np.abs(ev[:, None] - ref[None, :]) / np.maximum(np.abs(ref)[None, :], g["radius"])
    a, b = linear_sum_assignment(cost)
    assert cost[a, b].max() < 1e-10      # the FP64 parity tolerance; residuals are at 1e-10


# ---- the contour-integral reading of the reduced problem (caller-supplied functions)

def _random_reduced_quadratic(m, seed):
    rng = np.random.default_rng(seed)
    return [np.eye(m, dtype=complex), wl.cn(rng, (m, m)) / np.sqrt(m), wl.cn(rng, (m, m)) / np.sqrt(m)]


@pytest.mark.parametrize("shape", [(0.2 + 0.1j, 0.6, 0.6), (-0.1 + 0.0j, 0.9, 0.35)])
def test_contour_eigs_match_companion_on_a_polynomial(shape):
    """For a polynomial reduced problem the pairs inside the enlarged ellipse are exactly the
    companion eigenvalues there (away from its boundary, where the trapezoid rule loses
    accuracy), and each vector is a null vector of T(lambda)."""
    c, a, b = shape
    C = qd.Contour(c, a, b)
    Ahat = _random_reduced_quadratic(12, 41)
    terms = [("pow", 2), ("pow", 1), ("pow", 0)]
    lam, Y = reduced.contour_eigs(terms, Ahat, C)
    comp = brute.companion_eigs(pb.Problem(terms, Ahat))
    rho_c = C.radius(comp)
    want = comp[rho_c < reduced.CONTOUR_SCALE - 0.08]
    assert len(want) >= 4
    got = lam[C.radius(lam) < reduced.CONTOUR_SCALE - 0.08]
    assert len(got) == len(want)
    assert match_error(got, want, max(a, b)) < 1e-9
    for i in np.flatnonzero(C.radius(lam) < reduced.CONTOUR_SCALE - 0.08):
        T = reduced.reduced_T(terms, Ahat, lam[i])
        assert np.linalg.norm(T @ Y[:, i]) < 1e-8 * np.linalg.norm(T)


def test_contour_reduced_completes_to_m0():
    """T(lambda) = lambda I - diag(d) with three d_i inside the enlarged circle: three pairs
    found (the d_i, unit vectors e_i), the rest completed with vectors orthogonal to them and
    values on the enlarged contour."""
    m, m0 = 10, 10
    C = qd.Contour(0.0, 1.0)
    d = np.array([0.1, -0.5j, 0.9 + 0.3j, 3.0, -4.0, 5j, 2.5 + 2.5j, -3 - 3j, 6.0, 7.0])
    Ahat = [np.eye(m, dtype=complex), -np.diag(d)]
    terms = [("pow", 1), ("pow", 0)]
    lam, Y, found = reduced.contour_reduced(terms, Ahat, C, m0)
    assert found.sum() == 3 and found[:3].all()
    assert match_error(lam[:3], d[:3], 1.0) < 1e-12
    assert np.allclose(C.radius(lam[3:]), reduced.CONTOUR_SCALE)
    assert np.allclose(Y.conj().T @ Y, np.eye(m0), atol=1e-12)


def _as_user_terms(terms):
    """The same problem with every 'exp' term handed over as a caller-supplied function."""
    out = []
    for k, p in terms:
        if k == "exp":
            tau = float(p)
            out.append(("fn", pb.ScalarFunction(lambda z, t=tau: np.exp(-t * z),
                                                lambda z, t=tau: -t * np.exp(-t * z), "exp")))
        else:
            out.append((k, p))
    return out


@pytest.mark.parametrize("route", ["user", "forced"])
def test_contour_reading_delay_known_spectrum(route):
    """The known-spectrum delay problem through the contour-integral reduced solve, with the
    exponential either supplied as a caller function or kept built in and the reading forced."""
    C = qd.Contour(0.4 + 0.6j, 0.3)
    terms, mats, (b, c, e) = known_spectrum_delay(40, 21, C.c, C.a, 6)
    truth = []
    for i in range(40):
        truth += scalar_roots_inside(b[i], c[i], e[i], C)
    P = pb.Problem(_as_user_terms(terms) if route == "user" else terms, mats)
    z, w = qd.nodes_weights(C, 16)
    m0 = len(truth) + 6
    r = nlfeast.solve(P, C, z, w, wl.initial_block(40, m0, 22), m0, 1e-12, reduced="contour")
    assert r.converged and r.inside.sum() == len(truth)
    assert match_error(r.eigenvalues, np.array(truth), C.a) < 1e-10


def test_contour_reading_rational_matches_brute_force():
    """A0 - lambda I + lambda/(lambda - sigma) C: multiplied by (lambda - sigma) it is the
    quadratic -lambda^2 I + lambda (A0 + sigma I + C) - sigma A0, whose companion
    eigenvalues inside the circle are the truth."""
    n = 120
    terms, mats = wl.rational_nep(n, 1008)
    sig = terms[2][1]
    F = pb.ScalarFunction(lambda z: wl.pole_value(z, sig), lambda z: wl.pole_deriv(z, sig), "pole")
    P = pb.Problem([terms[0], terms[1], ("fn", F)], mats)
    A0, _, Cm = mats
    quad = pb.Problem([("pow", 2), ("pow", 1), ("pow", 0)],
                      [-np.eye(n), A0 + sig * np.eye(n) + Cm, -sig * A0])
    lam = brute.companion_eigs(quad)
    c = -0.5 - 0.8j
    d = np.sort(np.abs(lam - c))
    r = 0.5 * (d[9] + d[10])
    assert (d[10] - d[9]) / d[10] > 0.03
    C = qd.Contour(c, r)
    truth = lam[np.abs(lam - c) < r]
    z, w = qd.nodes_weights(C, 16)
    res = nlfeast.solve(P, C, z, w, wl.initial_block(n, 20, 2008), 20, 1e-11)
    assert res.converged and res.inside.sum() == len(truth) == 10
    assert match_error(res.eigenvalues, truth, r) < 1e-11


# ---- left eigenvectors (eigentriples): Algorithm 1 on the adjoint function

def test_left_solve_matches_brute_force_left_null_vectors():
    """Random quadratic problem: the left solve returns the same eigenvalues as the right solve
    and the companion, and each y spans the left null space of T(lambda) (the left singular
    vector of its smallest singular value, by an independent SVD); every simple eigenvalue has
    y^H T'(lambda) x != 0."""
    n, m0 = 60, 14
    terms, mats = wl.random_qep(n, 77)
    P = pb.Problem(terms, mats)
    lam = brute.companion_eigs(P)
    c = lam[np.argmin(np.abs(lam - 0.3j))]
    d = np.sort(np.abs(lam - c))
    r = 0.5 * (d[7] + d[8])
    assert (d[8] - d[7]) / d[8] > 0.02
    C = qd.Contour(c, r)
    z, w = qd.nodes_weights(C, 16)
    right = nlfeast.solve(P, C, z, w, wl.initial_block(n, m0, 78), m0, 1e-12)
    left = nlfeast.solve_left(P, C, 16, wl.initial_block(n, m0, 79), m0, 1e-12)
    truth = lam[np.abs(lam - c) < r]
    # spurious Ritz values inside (reading of the stop rule) occur on both sides here; the
    # converged sets are compared
    good = left.inside & ~left.spurious
    assert left.converged and good.sum() == len(truth) == 8
    assert match_error(left.eigenvalues, truth, r) < 1e-11
    assert match_error(left.eigenvalues, right.eigenvalues, r) < 1e-11
    for l, y in zip(left.lam[good], left.X[:, good].T):
        T = P.T(l)
        U, sv, _ = np.linalg.svd(T)
        assert sv[-1] < 1e-11 * sv[0] and sv[-2] > 1e-6 * sv[0]
        assert abs(abs(np.vdot(U[:, -1], y)) - 1.0) < 1e-10
        assert np.linalg.norm(y.conj() @ T) < 1e-12 * sv[0]
        i = np.argmin(np.abs(right.lam - l))
        assert abs(np.vdot(y, P.dT(l) @ right.X[:, i])) > 1e-6


def test_left_vectors_of_a_real_symmetric_problem_are_conjugate_right_vectors():
    """Example 2's A_j are real symmetric, so T(lambda)^T = T(lambda) and y = conj(x) up to a
    phase (Sec. 5: the right and left eigenvectors coincide for real A_j)."""
    n = 50
    terms, mats = wl.mass_spring(n, 10.0, 5.0)
    P = pb.Problem(terms, mats)
    C = qd.Contour(-20.5, 9.5)
    right = nlfeast.solve(P, C, *qd.nodes_weights(C, 8), wl.initial_block(n, 25, 5), 25, 1e-10)
    left = nlfeast.solve_left(P, C, 8, wl.initial_block(n, 25, 6), 25, 1e-10)
    good = left.inside & ~left.spurious
    assert good.sum() == len(right.eigenvalues) == 19
    for l, y in zip(left.lam[good], left.X[:, good].T):
        i = np.argmin(np.abs(right.lam - l))
        assert abs(right.lam[i] - l) < 1e-10 * abs(l)
        assert abs(abs(np.vdot(right.X[:, i].conj(), y)) - 1.0) < 1e-9


def test_left_solve_of_a_user_function_problem():
    """The adjoint of a caller-supplied term is conj(f(conj mu)): the rational problem's left
    eigenvectors annihilate T(lambda) from the left."""
    n = 80
    terms, mats = wl.rational_nep(n, 1008)
    sig = terms[2][1]
    F = pb.ScalarFunction(lambda z: wl.pole_value(z, sig), lambda z: wl.pole_deriv(z, sig), "pole")
    P = pb.Problem([terms[0], terms[1], ("fn", F)], mats)
    C = qd.Contour(-0.3 + 0.4j, 0.35)
    left = nlfeast.solve_left(P, C, 16, wl.initial_block(n, 16, 7), 16, 1e-12)
    right = nlfeast.solve(P, C, *qd.nodes_weights(C, 16), wl.initial_block(n, 16, 8), 16, 1e-12)
    good = left.inside & ~left.spurious
    assert left.converged and good.sum() == len(right.eigenvalues) >= 3
    assert match_error(left.eigenvalues, right.eigenvalues, C.a) < 1e-11
    for l, y in zip(left.lam[good], left.X[:, good].T):
        assert np.linalg.norm(y.conj() @ P.T(l)) < 1e-11


def test_stored_full_oracle_runs_reproduce_the_reference_sets():
    # the oracle's complete runs of the benchmark workloads (make_oracle_runs.py) against the
    # independent reference sets of contours.json (brute force, certified refinement, winding
    # count): every region's converged eigenvalues inside are exactly that set, to the parity
    # metric's relative error
    runs = json.load(open(os.path.join(GOLDEN, "oracle_runs.json")))
    refs = json.load(open(os.path.join(GOLDEN, "contours.json")))
    assert set(runs) >= {"damped4096", "qep2048x8", "delay8192"}
    for name, run in runs.items():
        cfg = wl.CONFIGS[name]
        for got, g in zip(run["regions"], refs[name]["regions"]):
            lam = np.array([complex(*v) for v in got["eigenvalues"]])
            ref = np.array([complex(*v) for v in g["eigenvalues"]])
            assert len(lam) == len(ref) == got["converged"], (name, len(lam), len(ref))
            assert got["max_residual"] <= cfg["tol"]
            scale = np.maximum(np.abs(ref), g["radius"]) if len(ref) else 1.0
            if len(ref):
                from scipy.optimize import linear_sum_assignment
                cost = np.abs(lam[:, None] - ref[None, :]) / np.asarray(scale)[None, :]
                i, j = linear_sum_assignment(cost)
                assert cost[i, j].max() < 1e-9, (name, cost[i, j].max())
        assert run["converged"] == sum(len(g["eigenvalues"]) for g in refs[name]["regions"])
