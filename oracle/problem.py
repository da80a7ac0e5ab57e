"""The matrix-valued function T(lambda) (oracle; test infrastructure only).

The paper's problem is T(lambda) x = 0 (Sec. 1 eq. nlevp; Sec. 2 eq. NLEVP).  Its
examples are polynomial, T(lambda) = sum_i lambda^i A_i (Sec. 2 eq. polynomialeig), and
it names non-polynomial T as the general case (Sec. 6).  Here
T(lambda) = sum_j f_j(lambda) A_j with scalar functions

    ('pow', p)    f(lambda) = lambda**p
    ('exp', tau)  f(lambda) = exp(-tau * lambda)
    ('fn', F)     f(lambda) = F.f(lambda), f'(lambda) = F.df(lambda): a scalar function
                  supplied by the caller (a ScalarFunction), analytic in the region of
                  interest; the general T(lambda) of Sec. 6

and the block residual is T(X, Lambda) = sum_j A_j X f_j(Lambda) with
f_j(Lambda) = diag(f_j(lambda_i)), the paper's sum_i A_i X Lambda^i (Sec. 4.2) for
polynomial terms.
"""
import numpy as np


class ScalarFunction:
    """A caller-supplied scalar function for a ('fn', F) term: f and its derivative df,
    each mapping a complex numpy array to a complex numpy array of the same shape."""

    def __init__(self, f, df, name="user"):
        self.f, self.df, self.name = f, df, name

    def __repr__(self):
        return "ScalarFunction(%s)" % self.name


def f_eval(kind, param, lam):
    lam = np.asarray(lam, dtype=complex)
    if kind == "pow":
        return lam ** int(param)
    if kind == "exp":
        return np.exp(-float(param) * lam)
    if kind == "fn":
        return np.asarray(param.f(lam), dtype=complex)
    raise ValueError("unknown term kind %r" % kind)


def f_deriv(kind, param, lam):
    lam = np.asarray(lam, dtype=complex)
    if kind == "pow":
        p = int(param)
        return p * lam ** (p - 1) if p > 0 else np.zeros_like(lam)
    if kind == "exp":
        return -float(param) * np.exp(-float(param) * lam)
    if kind == "fn":
        return np.asarray(param.df(lam), dtype=complex)
    raise ValueError("unknown term kind %r" % kind)


def taylor_coeffs(kind, param, centre, degree):
    """Coefficients t_p of f(centre + mu) = sum_p t_p mu^p, p = 0..degree (exact for
    'pow' once degree >= p)."""
    c = complex(centre)
    t = np.zeros(degree + 1, dtype=complex)
    if kind == "pow":
        q = int(param)
        for p in range(min(q, degree) + 1):
            binom = 1.0
            for i in range(p):
                binom = binom * (q - i) / (i + 1)
            t[p] = binom * c ** (q - p)
        return t
    if kind == "exp":
        tau = float(param)
        e = np.exp(-tau * c)
        fact = 1.0
        for p in range(degree + 1):
            if p > 0:
                fact *= p
            t[p] = e * (-tau) ** p / fact
        return t
    raise ValueError("unknown term kind %r" % kind)


class Problem:
    """T(lambda) = sum_j f_j(lambda) A_j with dense complex A_j (n x n)."""

    def __init__(self, terms, mats):
        if len(terms) != len(mats) or not terms:
            raise ValueError("need one matrix per term")
        self.terms = [(str(k), p if k == "fn" else float(p)) for k, p in terms]
        self.mats = [np.asarray(A, dtype=complex) for A in mats]
        n = self.mats[0].shape[0]
        for A in self.mats:
            if A.shape != (n, n):
                raise ValueError("all A_j must be n x n")
        self.n = n

    @property
    def has_user_terms(self):
        return any(k == "fn" for k, _ in self.terms)

    @property
    def is_polynomial(self):
        return all(k == "pow" for k, _ in self.terms)

    @property
    def degree(self):
        return max(int(p) for k, p in self.terms if k == "pow") if self.is_polynomial else None

    def T(self, z):
        """T(z) = sum_j f_j(z) A_j."""
        out = np.zeros((self.n, self.n), dtype=complex)
        for (k, p), A in zip(self.terms, self.mats):
            out += complex(f_eval(k, p, z)) * A
        return out

    def dT(self, z):
        """T'(z) = sum_j f_j'(z) A_j."""
        out = np.zeros((self.n, self.n), dtype=complex)
        for (k, p), A in zip(self.terms, self.mats):
            out += complex(f_deriv(k, p, z)) * A
        return out

    def block_residual(self, X, lam):
        """T(X, Lambda) = sum_j A_j X f_j(Lambda) (Sec. 4.2)."""
        R = np.zeros(X.shape, dtype=complex)
        for (k, p), A in zip(self.terms, self.mats):
            R += (A @ X) * f_eval(k, p, lam)[None, :]
        return R

    def project(self, Q):
        """Reduced coefficients Q^H A_j Q (Algorithm 1, Step 1)."""
        return [Q.conj().T @ A @ Q for A in self.mats]
