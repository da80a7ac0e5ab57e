"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This module only draws random numbers and writes down problem data (the coefficient
matrices A_j with their term kinds, and the initial block X0).  It holds none of the
eigensolver's arithmetic: no quadrature, no factorisation, no projection.

Workloads
  mass_spring(n, tau, kappa)   Sec. 5 Examples 1 and 2: A2 = I, A1 = tau T3,
                               A0 = kappa T3 with T3 = tridiag(-1, 3, -1)
  scattering_1d(npts, V0)      Sec. 5 Example 3: T(k) = k^2 A_h + i k B_h - C_h
  random_qep(n, seed)          A2 = I, A1 and A0 complex Gaussian / sqrt(n)
  damped_qep(n, seed)          mass-spring-damper: A2 = diag(U[1,2]),
                               A1 = 0.05 S / ||S||_2 with S = G G^T / n (G real Gaussian),
                               A0 = tridiag(-1, 2, -1) + 1e-2 CN / sqrt(n)
  delay_problem(n, seed)       lambda^2 M + lambda C + K + exp(-tau lambda) E with M = I,
                               C = 0.1 CN / sqrt(n), K = tridiag(-1, 2, -1),
                               E = 0.5 CN / sqrt(n), tau = 1
  rational_nep(n, seed, sigma) A0 - lambda I + lambda / (lambda - sigma) C with A0 = CN / sqrt(n),
                               C = 0.3 CN / sqrt(n), sigma = 4: a rational problem whose third
                               term is a caller-supplied function ('fn', sigma) evaluated by
                               pole_value / pole_deriv
  initial_block(n, m0, seed)   X0 with i.i.d. CN(0, 1) entries

CN(0, 1) = (N(0,1) + i N(0,1)) / sqrt(2).  Random streams: numpy default_rng(seed).
Every matrix is returned as a complex128 numpy array in C (row-major) order; term kinds
are ('pow', p) for lambda^p, ('exp', tau) for exp(-tau lambda) and ('fn', sigma) for the
pole function lambda / (lambda - sigma).
"""
import numpy as np

QUADRATIC = [("pow", 2), ("pow", 1), ("pow", 0)]
DELAY = [("pow", 2), ("pow", 1), ("pow", 0), ("exp", 1.0)]


def cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def tridiag(n, diag, off):
    T = np.zeros((n, n))
    i = np.arange(n)
    T[i, i] = diag
    T[i[:-1], i[:-1] + 1] = off
    T[i[:-1] + 1, i[:-1]] = off
    return T


def mass_spring(n, tau, kappa):
    T3 = tridiag(n, 3.0, -1.0)
    mats = [np.eye(n), tau * T3, kappa * T3]
    return list(QUADRATIC), [m.astype(complex) for m in mats]


def scattering_1d(npts=302, V0=10.0, width=np.pi * np.sqrt(2.0)):
    """Finite-element matrices of Example 3 on x_j = -L + j h, j = 0..npts+1,
    h = 2L/(npts+1), size npts+2.  Returns terms and [A_h, i B_h, -C_h]."""
    L = width / 2.0
    h = 2.0 * L / (npts + 1)
    m = npts + 2
    Ah = tridiag(m, 4.0, 1.0)
    Ah[0, 0] = Ah[-1, -1] = 2.0
    Ah *= h / 6.0
    Bh = np.zeros((m, m))
    Bh[0, 0] = Bh[-1, -1] = 1.0
    Ch = tridiag(m, 2.0, -1.0)
    Ch[0, 0] = Ch[-1, -1] = 1.0
    Ch = Ch / h + V0 * Ah
    return list(QUADRATIC), [Ah.astype(complex), 1j * Bh, -Ch.astype(complex)]


def random_qep(n, seed):
    rng = np.random.default_rng(seed)
    A1 = cn(rng, (n, n)) / np.sqrt(n)
    A0 = cn(rng, (n, n)) / np.sqrt(n)
    return list(QUADRATIC), [np.eye(n, dtype=complex), A1, A0]


def _spectral_norm_sym(S, iters=200):
    """Largest eigenvalue of a symmetric positive semidefinite S by a fixed number of
    power steps from the all-ones vector (deterministic data normalisation)."""
    v = np.ones(S.shape[0]) / np.sqrt(S.shape[0])
    lam = 0.0
    for _ in range(iters):
        w = S @ v
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def damped_qep(n, seed):
    rng = np.random.default_rng(seed)
    a2 = rng.uniform(1.0, 2.0, n)
    G = rng.standard_normal((n, n))
    S = (G @ G.T) / n
    S = 0.5 * (S + S.T)
    A1 = 0.05 * S / _spectral_norm_sym(S)
    A0 = tridiag(n, 2.0, -1.0) + 1e-2 * cn(rng, (n, n)) / np.sqrt(n)
    return list(QUADRATIC), [np.diag(a2).astype(complex), A1.astype(complex), A0.astype(complex)]


def delay_problem(n, seed, tau=1.0):
    rng = np.random.default_rng(seed)
    C = 0.1 * cn(rng, (n, n)) / np.sqrt(n)
    E = 0.5 * cn(rng, (n, n)) / np.sqrt(n)
    K = tridiag(n, 2.0, -1.0).astype(complex)
    terms = [("pow", 2), ("pow", 1), ("pow", 0), ("exp", float(tau))]
    return terms, [np.eye(n, dtype=complex), C, K, E]


def random_pep(n, seed, degree=4):
    """lambda^d I + sum_{j<d} lambda^j A_j, A_j = CN(0,1)/sqrt(n) (a degree-d polynomial problem
    with the same coefficient statistics as random_qep)."""
    rng = np.random.default_rng(seed)
    mats = [np.eye(n, dtype=complex)] + [cn(rng, (n, n)) / np.sqrt(n) for _ in range(degree)]
    return [("pow", degree - q) for q in range(degree + 1)], mats


def pole_value(z, sigma):
    """The scalar function of a ('fn', sigma) term: lambda / (lambda - sigma)."""
    z = np.asarray(z, dtype=complex)
    return z / (z - sigma)


def pole_deriv(z, sigma):
    """Its derivative, -sigma / (lambda - sigma)^2."""
    z = np.asarray(z, dtype=complex)
    return -sigma / (z - sigma) ** 2


def rational_nep(n, seed, sigma=4.0):
    rng = np.random.default_rng(seed)
    A0 = cn(rng, (n, n)) / np.sqrt(n)
    C = 0.3 * cn(rng, (n, n)) / np.sqrt(n)
    return [("pow", 0), ("pow", 1), ("fn", float(sigma))], [A0, -np.eye(n, dtype=complex), C]


def initial_block(n, m0, seed):
    return cn(np.random.default_rng(seed), (n, m0))


# Named configurations: problem seed 1000 + id, X0 seed 2000 + id, contour seed 3000 + id.
CONFIGS = {
    "qep200": dict(id=1, kind="random_qep", n=200, m0=20, nc=8, tol=1e-12, inside=10),
    "damped4096": dict(id=2, kind="damped_qep", n=4096, m0=64, nc=16, tol=1e-10, inside=40),
    # trapezoid nodes: with 16 Gauss-Legendre nodes on a full circle three of the eight
    # regions keep a spurious Ritz value inside (the oracle behaves the same)
    "qep2048x8": dict(id=4, kind="random_qep", n=2048, nc=16, tol=1e-10, quad="trapezoid",
                      m0s=[16, 24, 32, 48, 64, 80, 96, 128]),
    "delay8192": dict(id=5, kind="delay_problem", n=8192, m0=160, nc=24, tol=1e-10, inside=100),
    # the delay problem at a size the oracle iterates in seconds (parity case)
    "delay512": dict(id=6, kind="delay_problem", n=512, m0=24, nc=16, tol=1e-11, inside=12),
    # a quartic problem for the sweep over the number of quadrature nodes
    "quartic1024": dict(id=7, kind="random_pep", n=1024, m0=24, nc=16, tol=1e-10, inside=14),
    # a rational problem with a caller-supplied term (the contour-integral reduced solve)
    "rational300": dict(id=8, kind="rational_nep", n=300, m0=24, nc=16, tol=1e-11, inside=12),
}


def make_problem(name):
    cfg = CONFIGS[name]
    gen = {"random_qep": random_qep, "damped_qep": damped_qep, "delay_problem": delay_problem,
           "random_pep": random_pep, "rational_nep": rational_nep}[cfg["kind"]]
    return gen(cfg["n"], 1000 + cfg["id"])
