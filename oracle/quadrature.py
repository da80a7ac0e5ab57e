"""Quadrature nodes and weights on a closed contour (oracle; test infrastructure only).

Algorithm 1 takes "a set of n_c quadrature nodes and weights (z_j, omega_j)" over the
contour C (Sec. 4.2, Algorithm 1 inputs) and approximates (1/2 pi i) oint_C g(z) dz by
sum_j omega_j g(z_j) (Sec. 3, eq. feast_sum; Step 4 of Algorithm 1).  The paper does
not name a rule.  Reading taken here:

* Gauss-Legendre with n_c points on the parameter interval [0, 2 pi] of the whole
  contour: theta_k = pi (1 + t_k), with (t_k, w_k) the Legendre points/weights on [-1, 1].
* the trapezoid rule theta_k = 2 pi (k + 1/2) / n_c is the alternative.
* the factor 1/(2 pi i) is folded into omega_k.

Contours: a circle z = c + r e^{i theta} (Sec. 5, Examples 2 and 3) or an axis-aligned
ellipse z = c + a cos(theta) + i b sin(theta) (Sec. 5, Example 1).
"""
import numpy as np


class Contour:
    """Axis-aligned ellipse with centre c and semi-axes a (real) and b (imaginary).
    a == b is a circle (Sec. 5, Examples 1-3)."""

    def __init__(self, centre, a, b=None):
        self.c = complex(centre)
        self.a = float(a)
        self.b = float(a if b is None else b)
        if self.a <= 0 or self.b <= 0:
            raise ValueError("semi-axes must be positive")

    def point(self, theta):
        return self.c + self.a * np.cos(theta) + 1j * self.b * np.sin(theta)

    def dpoint(self, theta):
        """dz/dtheta."""
        return -self.a * np.sin(theta) + 1j * self.b * np.cos(theta)

    def radius(self, lam):
        """Normalised elliptic radius: < 1 strictly inside, 1 on C, > 1 outside.
        Infinite or NaN values map to +inf (they are never inside)."""
        lam = np.asarray(lam, dtype=complex)
        d = lam - self.c
        with np.errstate(invalid="ignore", over="ignore"):
            rho = np.sqrt((d.real / self.a) ** 2 + (d.imag / self.b) ** 2)
        rho = np.where(np.isfinite(rho), rho, np.inf)
        return rho

    def inside(self, lam):
        """Strictly inside C (a value on C counts as outside)."""
        return self.radius(lam) < 1.0


def nodes_weights(contour, nc, rule="gauss"):
    """(z_k, omega_k), k = 0..nc-1, such that sum_k omega_k g(z_k) approximates
    (1/2 pi i) oint_C g(z) dz.

    With z(theta) the parametrisation, (1/2 pi i) int_0^{2pi} g(z(theta)) z'(theta) dtheta
    is approximated by sum_k W_k g(z(theta_k)) z'(theta_k) / (2 pi i) where (theta_k, W_k)
    is the rule on [0, 2 pi]."""
    if nc < 1:
        raise ValueError("nc must be positive")
    if rule == "gauss":
        t, w = np.polynomial.legendre.leggauss(nc)
        theta = np.pi * (1.0 + t)
        W = np.pi * w
    elif rule == "trapezoid":
        theta = 2.0 * np.pi * (np.arange(nc) + 0.5) / nc
        W = np.full(nc, 2.0 * np.pi / nc)
    else:
        raise ValueError("unknown rule %r" % rule)
    z = contour.point(theta)
    omega = W * contour.dpoint(theta) / (2j * np.pi)
    return z.astype(complex), omega.astype(complex)


def filter_value(z, omega, lam):
    """The scalar rational filter rho(lambda) = sum_k omega_k / (z_k - lambda): the
    quadrature approximation of (1/2 pi i) oint dz / (z - lambda), which is 1 inside C
    and 0 outside (Sec. 3, eqs. feast_int and feast_sum for a 1x1 pencil)."""
    lam = np.asarray(lam, dtype=complex)
    return np.sum(omega[:, None] / (z[:, None] - lam.ravel()[None, :]), axis=0).reshape(lam.shape)
