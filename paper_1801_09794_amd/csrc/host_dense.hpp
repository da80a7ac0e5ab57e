// Host-side small dense routines of the nonlinear FEAST library: contour quadrature, the
// Cholesky factor used by the orthonormalisation, and the reduced (projected) eigenproblem of
// Algorithm 1, Steps 1-2.
#pragma once

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

// Term of T(lambda): kind 0 = lambda^p, kind 1 = exp(-tau lambda).
struct Term {
    int kind;
    double param;
};
cplx term_value(const Term& t, cplx l);
cplx term_deriv(const Term& t, cplx l);

// Host threads the dense routines below may use from the calling thread (default 16); callers
// that run several reduced solves at once lower it per thread.
int& host_thread_budget();

struct ReducedResult {
    std::vector<cplx> lambda;   // m_keep values, selection order
    std::vector<cplx> Y;        // m x m_keep, unit columns
    int n_finite = 0;
    bool ok = true;
};

// All eigenpairs of sum_j f_j(lambda) Ahat_j y = 0 (Ahat: J matrices m x m, column-major,
// consecutive), then the m_keep closest to the interior of E (ascending normalised radius,
// stable, non-finite last).  Polynomial terms: exact companion linearisation, inverted about
// a shift inside the contour (the centre unless a Ritz value in `avoid` is close to it);
// exponential terms: Taylor expansion about that shift followed by Newton refinement on the
// exact reduced function.
ReducedResult reduced_solve(int m, const std::vector<Term>& terms, const cplx* Ahat,
                            const Ellipse& E, int m_keep, const std::vector<cplx>* avoid = nullptr);

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
