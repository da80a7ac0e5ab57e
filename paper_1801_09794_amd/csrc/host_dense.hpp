// Host-side small dense routines of the nonlinear FEAST library: contour quadrature, the
// Cholesky factor used by the orthonormalisation, and the reduced (projected) eigenproblem of
// Algorithm 1, Steps 1-2.
#pragma once

#include <atomic>
#include <complex>
#include <cstdint>
#include <vector>

namespace nlf {

using cplx = std::complex<double>;

struct Ellipse {
    cplx c;
    double a, b;     // semi-axes: real direction, imaginary direction
    double radius(cplx l) const;   // normalised radius; +inf for non-finite l
};

// (z_k, omega_k) such that sum_k omega_k g(z_k) approximates (1/2 pi i) oint_C g(z) dz.
// rule 0: Gauss-Legendre on the parameter interval [0, 2 pi]; rule 1: trapezoid with
// theta_k = 2 pi (k + 1/2) / nc.
void quadrature(const Ellipse& E, int nc, int rule, std::vector<cplx>& z, std::vector<cplx>& w);

// Upper-triangular R with G = R^H R (G Hermitian positive definite, m x m, column-major).
// Returns false when a pivot is not positive.  Rinv receives R^{-1} (upper triangular);
// min_pivot_ratio (optional) the smallest R_jj^2 / G_jj, a detector of near dependence.
bool cholesky_upper_inverse(int m, const cplx* G, std::vector<cplx>& Rinv,
                            double* min_pivot_ratio = nullptr);

// A caller-supplied scalar function: fn(user, term, param, count, z, f, df) writes f(z_i) and,
// when df is not null, f'(z_i), as interleaved (re, im) pairs for count points; a nonzero
// return marks a failure.  A failure is recorded in `failed` (the evaluation then yields NaN)
// and turned into an error by the caller once the host work that asked has finished.
using UserFnPtr = int32_t (*)(void*, int32_t, double, int64_t, const double*, double*, double*);
struct UserFunction {
    UserFnPtr fn = nullptr;
    void* user = nullptr;
    mutable std::atomic<int> failed{0};
};

// Term of T(lambda): kind 0 = lambda^p, kind 1 = exp(-tau lambda), kind 2 = the caller's
// function fn, called with the term's position `index` and parameter.  conj: the term of the
// adjoint function T(conj mu)^H, i.e. conj(f(conj mu)) (the same function for kinds 0 and 1,
// whose parameters are real).
struct Term {
    int kind;
    double param;
    const UserFunction* fn = nullptr;
    int index = 0;
    bool conj = false;
};
cplx term_value(const Term& t, cplx l);
cplx term_deriv(const Term& t, cplx l);
// f(z_i) for count points (one call of a caller-supplied function).
void term_values(const Term& t, const cplx* z, int64_t count, cplx* f);
// True when a caller-supplied function among the terms has reported a failure.
bool user_failed(const std::vector<Term>& terms);

// Host threads the dense routines below may use from the calling thread (default 16); callers
// that run several reduced solves at once lower it per thread.
int& host_thread_budget();

struct ReducedResult {
    std::vector<cplx> lambda;   // m_keep values, selection order
    std::vector<cplx> Y;        // m x m_keep, unit columns
    std::vector<int> found;     // 1 for an eigenpair of the reduced problem, 0 for a completing pair
    int n_finite = 0;
    bool ok = true;
    // host milliseconds of the parts of the contour-integral solve: resolvent points and moments,
    // rank-revealing QR + small eigenproblem, Newton refinement; and the Newton pairs and steps
    double ms_points = 0, ms_rank_eig = 0, ms_newton = 0;
    int newton_pairs = 0, newton_steps = 0, rank = 0;
};

// Enlargement of the contour, trapezoid points and relative rank threshold of the
// contour-integral reduced solve.
constexpr double CONTOUR_SCALE = 1.5;
constexpr int CONTOUR_POINTS = 96;
constexpr double CONTOUR_RANK_TOL = 1e-10;

// All eigenpairs of sum_j f_j(lambda) Ahat_j y = 0 (Ahat: J matrices m x m, column-major,
// consecutive), then the m_keep closest to the interior of E (ascending normalised radius,
// stable, non-finite last).  Polynomial terms: exact companion linearisation, inverted about
// a shift inside the contour (the centre unless a Ritz value in `avoid` is close to it).
// Non-polynomial terms (method 0 or 1; always with a caller-supplied term): the contour-integral
// solve (contour_pairs), Newton refinement of every pair found, and completion to m_keep pairs
// (requires m_keep <= m) by unit vectors orthogonal to those found, paired with values spread
// over the enlarged ellipse.  Method 2 with exponential terms: Taylor expansion about the shift,
// linearised, followed by Newton refinement on the exact reduced function.
ReducedResult reduced_solve(int m, const std::vector<Term>& terms, const cplx* Ahat,
                            const Ellipse& E, int m_keep, const std::vector<cplx>* avoid = nullptr,
                            int method = 0);

// Eigenpairs of sum_j f_j(lambda) Ahat_j y = 0 inside the ellipse E enlarged CONTOUR_SCALE
// times, from the moments M_p = (1/2 pi i) oint mu^p T(z)^{-1} dz, mu = (z - c)/L (L the larger
// enlarged semi-axis), by the trapezoid rule with CONTOUR_POINTS points: the block Hankel
// matrices H0 = [M_{i+j}], H1 = [M_{i+j+1}] (K x K blocks, K = 2, or 3 when H0 has full rank)
// factor as Vb W^H and Vb mu(Lambda) W^H (Keldysh), and a pivoted QR H0 P = Q R with numerical
// rank k (pivots above CONTOUR_RANK_TOL times the integrand's size sum_q |w_q| ||T(z_q)^{-1}||_F:
// with no eigenvalue inside, the moments are rounding noise of that size) gives the k x k matrix Q_k^H H1 P_k R_11^{-1}, similar to mu(Lambda), whose
// eigenvectors s_i give the eigenvectors as the first block of Q_k s_i.  Returns false when
// T(z) is singular at a point or H0 keeps full rank with K = 3.
bool contour_pairs(int m, const std::vector<Term>& terms, const cplx* Ahat, const Ellipse& E,
                   std::vector<cplx>& lam, std::vector<cplx>& Y, double* ms_points = nullptr,
                   double* ms_rank_eig = nullptr);

// The two stages of contour_pairs, so that the first can run elsewhere (the solver forms the
// moments on the device).  contour_points: the CONTOUR_POINTS trapezoid points z_q of the
// enlarged ellipse, their weights w_q (including 1/(2 pi i)) and mu_q = (z_q - c)/L.
// Moments: M holds CONTOUR_MOMENTS blocks m x m, M_p = sum_q w_q mu_q^p T(z_q)^{-1}, and isize
// the CONTOUR_POINTS values |w_q| ||T(z_q)^{-1}||_F.  contour_pairs_from_moments: the rank
// decision, the reduced k x k eigenproblem and the eigenvectors (as in contour_pairs).
constexpr int CONTOUR_KMAX = 3;
constexpr int CONTOUR_MOMENTS = 2 * CONTOUR_KMAX;
void contour_points(const Ellipse& E, std::vector<cplx>& z, std::vector<cplx>& w, std::vector<cplx>& mu);
bool contour_pairs_from_moments(int m, const Ellipse& E, const std::vector<cplx>& M,
                                const std::vector<double>& isize, std::vector<cplx>& lam,
                                std::vector<cplx>& Y);
// Steps 1-2 by the contour-integral route from moments formed elsewhere: contour_pairs_from_moments,
// then the Newton refinement and completion of reduced_solve.
ReducedResult contour_reduced_from_moments(int m, const std::vector<Term>& terms, const cplx* Ahat,
                                           const Ellipse& E, int m_keep, const std::vector<cplx>& M,
                                           const std::vector<double>& isize);
// Whether reduced_solve takes the contour-integral route for these terms and method.
bool takes_contour_route(const std::vector<Term>& terms, int method);

// Complex Schur decomposition A = Z T Z^H of a dense N x N matrix (column-major) by
// Householder reduction to Hessenberg form and the shifted QR algorithm (Givens rotations,
// Wilkinson shifts); eigenvectors of selected eigenvalues by back substitution on T.
struct Schur {
    int N = 0;
    std::vector<cplx> T, Z, evals;
    double norm = 0.0;
    bool compute(int N, std::vector<cplx>& A, bool with_vectors);   // A is overwritten
    void vectors(const std::vector<int>& want, std::vector<cplx>& out) const;   // unit columns
};

// Eigenvalues of a dense N x N matrix by Householder reduction to Hessenberg form and the
// shifted QR algorithm confined to the active window; eigenvectors of selected eigenvalues by
// inverse iteration on the Hessenberg matrix and the reflectors' back-transformation.
struct HessEig {
    int N = 0;
    std::vector<cplx> H, H0, V, evals;
    std::vector<double> beta;
    double norm = 0.0;
    bool compute(int N, std::vector<cplx>& A);                               // A is consumed
    void vectors(const std::vector<int>& want, std::vector<cplx>& out) const;   // unit columns
};

// Dense complex eigen-decomposition of an N x N matrix (column-major): eigenvalues and the
// eigenvectors of the indices in `want` (unit 2-norm), via Householder Hessenberg reduction
// and the shifted QR algorithm with Givens rotations.  Returns false if QR fails to converge.
bool eig_dense(int N, std::vector<cplx>& A, std::vector<cplx>& evals,
               const std::vector<int>* want, std::vector<cplx>* evecs);

}  // namespace nlf
