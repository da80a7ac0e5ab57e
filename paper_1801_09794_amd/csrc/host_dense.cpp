// Host-side small dense routines (see host_dense.hpp).
#include "host_dense.hpp"

#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <limits>
#include <numeric>
#include <thread>

namespace nlf {

static const double kEps = 2.220446049250313e-16;
static const double kPi = 3.14159265358979323846;

// Complex dot products with independent partial sums in AVX2 registers (two complex values per
// register, two registers per sum), so consecutive multiply-adds do not wait on each other as
// they would in one running complex sum.  With x = [ar, ai, ...] and y = [br, bi, ...]:
// x*y = [ar br, ai bi], x*swap(y) = [ar bi, ai br], from which conj(a) b and a b follow.
template <bool CONJ>
static inline cplx cdot(int64_t n, const cplx* a, const cplx* b) {
    const double* x = reinterpret_cast<const double*>(a);
    const double* y = reinterpret_cast<const double*>(b);
    __m256d p0 = _mm256_setzero_pd(), q0 = _mm256_setzero_pd();
    __m256d p1 = _mm256_setzero_pd(), q1 = _mm256_setzero_pd();
    int64_t i = 0;
    for (; i + 4 <= n; i += 4) {
        const __m256d xa = _mm256_loadu_pd(x + 2 * i), ya = _mm256_loadu_pd(y + 2 * i);
        const __m256d xb = _mm256_loadu_pd(x + 2 * i + 4), yb = _mm256_loadu_pd(y + 2 * i + 4);
        p0 = _mm256_fmadd_pd(xa, ya, p0);
        q0 = _mm256_fmadd_pd(xa, _mm256_permute_pd(ya, 0x5), q0);
        p1 = _mm256_fmadd_pd(xb, yb, p1);
        q1 = _mm256_fmadd_pd(xb, _mm256_permute_pd(yb, 0x5), q1);
    }
    for (; i + 2 <= n; i += 2) {
        const __m256d xa = _mm256_loadu_pd(x + 2 * i), ya = _mm256_loadu_pd(y + 2 * i);
        p0 = _mm256_fmadd_pd(xa, ya, p0);
        q0 = _mm256_fmadd_pd(xa, _mm256_permute_pd(ya, 0x5), q0);
    }
    alignas(32) double P[4], Q[4];
    _mm256_store_pd(P, _mm256_add_pd(p0, p1));
    _mm256_store_pd(Q, _mm256_add_pd(q0, q1));
    // P = [ar br, ai bi] summed over both lanes pairs; Q = [ar bi, ai br]
    double rr = P[0] + P[2], ii = P[1] + P[3], ri = Q[0] + Q[2], ir = Q[1] + Q[3];
    if (i < n) {
        rr += x[2 * i] * y[2 * i];
        ii += x[2 * i + 1] * y[2 * i + 1];
        ri += x[2 * i] * y[2 * i + 1];
        ir += x[2 * i + 1] * y[2 * i];
    }
    return CONJ ? cplx(rr + ii, ri - ir) : cplx(rr - ii, ri + ir);
}
static inline cplx cdotc(int64_t n, const cplx* a, const cplx* b) { return cdot<true>(n, a, b); }
static inline cplx cdotu(int64_t n, const cplx* a, const cplx* b) { return cdot<false>(n, a, b); }
// y_i += alpha x_i (two complex values per register: x alpha = fmaddsub(x, re(alpha),
// swap(x) im(alpha)))
static inline void caxpy(int64_t n, cplx alpha, const cplx* x, cplx* y) {
    const double* xs = reinterpret_cast<const double*>(x);
    double* ys = reinterpret_cast<double*>(y);
    const __m256d ar = _mm256_set1_pd(alpha.real()), ai = _mm256_set1_pd(alpha.imag());
    int64_t i = 0;
    for (; i + 2 <= n; i += 2) {
        const __m256d xv = _mm256_loadu_pd(xs + 2 * i);
        const __m256d prod = _mm256_fmaddsub_pd(xv, ar, _mm256_mul_pd(_mm256_permute_pd(xv, 0x5), ai));
        _mm256_storeu_pd(ys + 2 * i, _mm256_add_pd(_mm256_loadu_pd(ys + 2 * i), prod));
    }
    for (; i < n; ++i) y[i] += alpha * x[i];
}
// sum_i |a_i|^2 with independent partial sums
static inline double csumsq(int64_t n, const cplx* a) {
    const double* x = reinterpret_cast<const double*>(a);
    __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
    int64_t i = 0;
    for (; i + 4 <= n; i += 4) {
        const __m256d xa = _mm256_loadu_pd(x + 2 * i), xb = _mm256_loadu_pd(x + 2 * i + 4);
        s0 = _mm256_fmadd_pd(xa, xa, s0);
        s1 = _mm256_fmadd_pd(xb, xb, s1);
    }
    alignas(32) double S[4];
    _mm256_store_pd(S, _mm256_add_pd(s0, s1));
    double t = (S[0] + S[1]) + (S[2] + S[3]);
    for (; i < n; ++i) t += std::norm(a[i]);
    return t;
}

double Ellipse::radius(cplx l) const {
    if (!std::isfinite(l.real()) || !std::isfinite(l.imag())) return std::numeric_limits<double>::infinity();
    const cplx d = l - c;
    return std::sqrt((d.real() / a) * (d.real() / a) + (d.imag() / b) * (d.imag() / b));
}

// Legendre points/weights on [-1, 1], ascending: Newton's method on P_n from the
// asymptotic first guesses cos(pi (i + 3/4) / (n + 1/2)); weight 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) {
                // one more evaluation for the derivative at the converged point
                p0 = 1.0; p1 = t;
                for (int k = 1; k < n; ++k) {
                    const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p1 = t; p0 = 1.0; }
                dp = n * (t * p1 - p0) / (t * t - 1.0);
                break;
            }
        }
        x[n - 1 - i] = t;                      // the guesses descend; store ascending
        w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

void quadrature(const Ellipse& E, int nc, int rule, std::vector<cplx>& z, std::vector<cplx>& w) {
    std::vector<double> theta(nc), W(nc);
    if (rule == 0) {
        std::vector<double> t, wt;
        gauss_legendre(nc, t, wt);
        for (int k = 0; k < nc; ++k) {
            theta[k] = kPi * (1.0 + t[k]);
            W[k] = kPi * wt[k];
        }
    } else {
        for (int k = 0; k < nc; ++k) {
            theta[k] = 2.0 * kPi * (k + 0.5) / nc;
            W[k] = 2.0 * kPi / nc;
        }
    }
    z.resize(nc);
    w.resize(nc);
    for (int k = 0; k < nc; ++k) {
        const double ct = std::cos(theta[k]), st = std::sin(theta[k]);
        z[k] = E.c + cplx(E.a * ct, E.b * st);
        const cplx dz(-E.a * st, E.b * ct);              // dz / dtheta
        w[k] = W[k] * dz / cplx(0.0, 2.0 * kPi);          // includes 1 / (2 pi i)
    }
}

bool cholesky_upper_inverse(int m, const cplx* G, std::vector<cplx>& Rinv, double* min_pivot_ratio) {
    std::vector<cplx> R(m * m, 0.0);
    double ratio = 1.0;
    for (int j = 0; j < m; ++j) {
        double d = G[j + j * m].real();
        for (int k = 0; k < j; ++k) d -= std::norm(R[k + j * m]);
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        ratio = std::min(ratio, d / G[j + j * m].real());
        const double rjj = std::sqrt(d);
        R[j + j * m] = rjj;
        for (int i = j + 1; i < m; ++i) {
            cplx s = G[j + i * m];
            for (int k = 0; k < j; ++k) s -= std::conj(R[k + j * m]) * R[k + i * m];
            R[j + i * m] = s / rjj;
        }
    }
    Rinv.assign(m * m, 0.0);
    for (int c = 0; c < m; ++c) {           // solve R x = e_c by back substitution
        Rinv[c + (size_t)c * m] = 1.0 / R[c + (size_t)c * m];
        for (int i = c - 1; i >= 0; --i) {
            cplx s = 0.0;
            for (int k = i + 1; k <= c; ++k) s += R[i + (size_t)k * m] * Rinv[k + (size_t)c * m];
            Rinv[i + (size_t)c * m] = -s / R[i + (size_t)i * m];
        }
    }
    if (min_pivot_ratio) *min_pivot_ratio = ratio;
    return true;
}

// One call of the caller's function at count points; NaN and a recorded failure when it
// reports one (or none is set).
static void user_call(const Term& t, const cplx* z, int64_t count, cplx* f, cplx* df) {
    static_assert(sizeof(cplx) == 2 * sizeof(double), "complex layout");
    for (int64_t i = 0; i < count; ++i) {
        f[i] = cplx(NAN, NAN);
        if (df) df[i] = cplx(NAN, NAN);
    }
    if (!t.fn || !t.fn->fn) {
        if (t.fn) t.fn->failed.store(1);
        return;
    }
    std::vector<cplx> zc;
    if (t.conj) {   // conj(f(conj z)) and its derivative conj(f'(conj z))
        zc.assign(z, z + count);
        for (cplx& v : zc) v = std::conj(v);
        z = zc.data();
    }
    if (t.fn->fn(t.fn->user, t.index, t.param, count, reinterpret_cast<const double*>(z),
                 reinterpret_cast<double*>(f), reinterpret_cast<double*>(df)) != 0)
        t.fn->failed.store(1);
    if (t.conj)
        for (int64_t i = 0; i < count; ++i) {
            f[i] = std::conj(f[i]);
            if (df) df[i] = std::conj(df[i]);
        }
}

void term_values(const Term& t, const cplx* z, int64_t count, cplx* f) {
    if (t.kind == 2) {
        user_call(t, z, count, f, nullptr);
        return;
    }
    for (int64_t i = 0; i < count; ++i) f[i] = term_value(t, z[i]);
}

bool user_failed(const std::vector<Term>& terms) {
    for (const Term& t : terms)
        if (t.kind == 2 && (!t.fn || t.fn->failed.load())) return true;
    return false;
}

cplx term_value(const Term& t, cplx l) {
    if (t.kind == 2) {
        cplx f;
        user_call(t, &l, 1, &f, nullptr);
        return f;
    }
    if (t.kind == 0) {
        const int p = (int)t.param;
        cplx r = 1.0;
        for (int i = 0; i < p; ++i) r *= l;
        return r;
    }
    return std::exp(-t.param * l);
}

cplx term_deriv(const Term& t, cplx l) {
    if (t.kind == 2) {
        cplx f, d;
        user_call(t, &l, 1, &f, &d);
        return d;
    }
    if (t.kind == 0) {
        const int p = (int)t.param;
        if (p == 0) return 0.0;
        cplx r = (double)p;
        for (int i = 0; i < p - 1; ++i) r *= l;
        return r;
    }
    return -t.param * std::exp(-t.param * l);
}

static inline double abs1(cplx a) { return std::fabs(a.real()) + std::fabs(a.imag()); }

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G [x; y] = [rho; 0].
static inline void givens(cplx x, cplx y, double& c, cplx& s, cplx& rho) {
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) { c = 1.0; s = 0.0; rho = x; return; }
    if (ax == 0.0) { c = 0.0; s = std::conj(y) / ay; rho = ay; return; }
    const double r = std::hypot(ax, ay);
    c = ax / r;
    const cplx ph = x / ax;
    s = ph * std::conj(y) / r;
    rho = ph * r;
}

bool Schur::compute(int N_, std::vector<cplx>& A, bool vecs) {
    N = N_;
    std::vector<cplx>& H = A;
    Z.clear();
    if (vecs) {
        Z.assign((size_t)N * N, 0.0);
        for (int i = 0; i < N; ++i) Z[i + (size_t)i * N] = 1.0;
    }
    std::vector<cplx> v(N), s(N);
    // Householder reduction to upper Hessenberg form, H <- P H P, Z <- Z P
    for (int k = 0; k + 2 < N; ++k) {
        double xn2 = 0.0;
        for (int i = k + 1; i < N; ++i) xn2 += std::norm(H[i + (size_t)k * N]);
        if (xn2 == 0.0) continue;
        const double xn = std::sqrt(xn2);
        const cplx x0 = H[k + 1 + (size_t)k * N];
        const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0);
        const cplx alpha = -ph * xn;
        for (int i = k + 1; i < N; ++i) v[i] = H[i + (size_t)k * N];
        v[k + 1] -= alpha;
        double vn2 = 0.0;
        for (int i = k + 1; i < N; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double beta = 2.0 / vn2;
        for (int j = k + 1; j < N; ++j) {                  // rows k+1.., columns k+1..
            cplx t = cdotc(N - k - 1, &v[k + 1], &H[k + 1 + (size_t)j * N]);
            t *= beta;
            caxpy(N - k - 1, -t, &v[k + 1], &H[k + 1 + (size_t)j * N]);
        }
        std::fill(s.begin(), s.end(), cplx(0.0));          // columns k+1.., all rows
        for (int j = k + 1; j < N; ++j)
            for (int i = 0; i < N; ++i) s[i] += H[i + (size_t)j * N] * v[j];
        for (int j = k + 1; j < N; ++j) {
            const cplx cv = beta * std::conj(v[j]);
            for (int i = 0; i < N; ++i) H[i + (size_t)j * N] -= s[i] * cv;
        }
        if (vecs) {
            std::fill(s.begin(), s.end(), cplx(0.0));
            for (int j = k + 1; j < N; ++j)
                for (int i = 0; i < N; ++i) s[i] += Z[i + (size_t)j * N] * v[j];
            for (int j = k + 1; j < N; ++j) {
                const cplx cv = beta * std::conj(v[j]);
                for (int i = 0; i < N; ++i) Z[i + (size_t)j * N] -= s[i] * cv;
            }
        }
        H[k + 1 + (size_t)k * N] = alpha;
        for (int i = k + 2; i < N; ++i) H[i + (size_t)k * N] = 0.0;
    }
    double hnorm = 0.0;
    for (size_t e = 0; e < (size_t)N * N; ++e) hnorm = std::max(hnorm, abs1(H[e]));
    if (hnorm == 0.0) hnorm = 1.0;
    // shifted QR iterations (Wilkinson shift, exceptional shifts at 10 and 20 stalled steps)
    int ihi = N - 1, its = 0, total = 0;
    while (ihi >= 0) {
        int l = ihi;
        while (l > 0) {
            double sc = abs1(H[l - 1 + (size_t)(l - 1) * N]) + abs1(H[l + (size_t)l * N]);
            if (sc == 0.0) sc = hnorm;
            if (abs1(H[l + (size_t)(l - 1) * N]) <= kEps * sc) {
                H[l + (size_t)(l - 1) * N] = 0.0;
                break;
            }
            --l;
        }
        if (l == ihi) {
            --ihi;
            its = 0;
            continue;
        }
        if (++its > 80 || ++total > 100 * N) return false;
        cplx mu;
        const cplx a = H[ihi - 1 + (size_t)(ihi - 1) * N], b = H[ihi - 1 + (size_t)ihi * N];
        const cplx c = H[ihi + (size_t)(ihi - 1) * N], d = H[ihi + (size_t)ihi * N];
        if (its == 10 || its == 20 || its == 40) {
            mu = d + std::abs(c.real()) * 0.75;
        } else {
            const cplx tr2 = 0.5 * (a + d);
            const cplx disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
            const cplx m1 = tr2 + disc, m2 = tr2 - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        cplx x = H[l + (size_t)l * N] - mu, y = H[l + 1 + (size_t)l * N];
        for (int k = l; k < ihi; ++k) {
            if (k > l) {
                x = H[k + (size_t)(k - 1) * N];
                y = H[k + 1 + (size_t)(k - 1) * N];
            }
            double cs;
            cplx sn, rho;
            givens(x, y, cs, sn, rho);
            if (k > l) {
                H[k + (size_t)(k - 1) * N] = rho;
                H[k + 1 + (size_t)(k - 1) * N] = 0.0;
            }
            const cplx csn = std::conj(sn);
            for (int j = k; j < N; ++j) {
                const cplx p = H[k + (size_t)j * N], q = H[k + 1 + (size_t)j * N];
                H[k + (size_t)j * N] = cs * p + sn * q;
                H[k + 1 + (size_t)j * N] = -csn * p + cs * q;
            }
            const int iend = std::min(k + 2, ihi);
            cplx* ck = &H[(size_t)k * N];
            cplx* ck1 = &H[(size_t)(k + 1) * N];
            for (int i = 0; i <= iend; ++i) {
                const cplx p = ck[i], q = ck1[i];
                ck[i] = cs * p + csn * q;
                ck1[i] = -sn * p + cs * q;
            }
            if (vecs) {
                cplx* zk = &Z[(size_t)k * N];
                cplx* zk1 = &Z[(size_t)(k + 1) * N];
                for (int i = 0; i < N; ++i) {
                    const cplx p = zk[i], q = zk1[i];
                    zk[i] = cs * p + csn * q;
                    zk1[i] = -sn * p + cs * q;
                }
            }
        }
    }
    evals.resize(N);
    for (int i = 0; i < N; ++i) evals[i] = H[i + (size_t)i * N];
    T.swap(H);
    norm = hnorm;
    return true;
}

void Schur::vectors(const std::vector<int>& want, std::vector<cplx>& out_vecs) const {
    const std::vector<cplx>& H = T;
    // eigenvectors of the triangular Schur factor by back substitution, then x = Z v
    const double smin = std::max(kEps * norm, std::numeric_limits<double>::min() * N);
    out_vecs.assign((size_t)N * want.size(), 0.0);
    std::vector<cplx> w(N);
    for (size_t q = 0; q < want.size(); ++q) {
        const int k = want[q];
        std::fill(w.begin(), w.end(), cplx(0.0));
        w[k] = 1.0;
        const cplx lk = H[k + (size_t)k * N];
        for (int i = k - 1; i >= 0; --i) {
            cplx t = 0.0;
            for (int j = i + 1; j <= k; ++j) t += H[i + (size_t)j * N] * w[j];
            cplx dd = H[i + (size_t)i * N] - lk;
            if (std::abs(dd) < smin) dd = smin;
            w[i] = -t / dd;
            if (std::abs(w[i]) > 1e100) {
                for (int j = i; j <= k; ++j) w[j] *= 1e-100;
            }
        }
        cplx* out = &out_vecs[(size_t)q * N];
        for (int j = 0; j <= k; ++j) {
            const cplx wj = w[j];
            if (wj == 0.0) continue;
            const cplx* zj = &Z[(size_t)j * N];
            for (int i = 0; i < N; ++i) out[i] += zj[i] * wj;
        }
        double nr = 0.0;
        for (int i = 0; i < N; ++i) nr += std::norm(out[i]);
        nr = std::sqrt(nr);
        if (nr > 0.0)
            for (int i = 0; i < N; ++i) out[i] /= nr;
    }
}

bool eig_dense(int N, std::vector<cplx>& A, std::vector<cplx>& evals, const std::vector<int>* want,
               std::vector<cplx>* evecs) {
    Schur S;
    const bool vecs = want && evecs;
    if (!S.compute(N, A, vecs)) return false;
    evals = S.evals;
    if (vecs) S.vectors(*want, *evecs);
    return true;
}


// ------------------------------------------------------------------------------------------
// Eigenvalues by the QR algorithm restricted to the active window (no Schur vectors), and
// eigenvectors of selected eigenvalues by inverse iteration on the Hessenberg matrix followed
// by the Householder back-transformation.  Work ~ (10/3 + ~4) N^3 real-complex operations
// instead of the ~25 N^3 of the full Schur form with vectors.
// A team of host threads that run one function together and meet at barriers (spinning:
// the phases between barriers are short).
namespace {
struct Team {
    int P;
    std::atomic<int> count{0}, gen{0};
    explicit Team(int p) : P(p) {}
    void barrier() {
        const int g = gen.load(std::memory_order_acquire);
        if (count.fetch_add(1, std::memory_order_acq_rel) == P - 1) {
            count.store(0, std::memory_order_relaxed);
            gen.store(g + 1, std::memory_order_release);
        } else {
            while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
    }
    template <typename F>
    void run(F f) {   // f(thread index) on P threads, the caller being thread 0
        std::vector<std::thread> ts;
        for (int t = 1; t < P; ++t) ts.emplace_back([&, t] { f(t); });
        f(0);
        for (auto& t : ts) t.join();
    }
};

int host_threads(int64_t work, int64_t per_thread) {
    const int hw = std::min((int)std::max(1u, std::thread::hardware_concurrency()), host_thread_budget());
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)hw, 16, work / std::max<int64_t>(per_thread, 1)}));
}
}  // namespace

int& host_thread_budget() {
    static thread_local int b = 16;
    return b;
}

// The two rotation updates of a QR sweep with G = [[c, s], [-conj(s), c]], in AVX2.
// Rows k, k+1 (p = row k, q = row k+1) over cnt columns with stride ld:
//   p <- c p + s q,  q <- -conj(s) p + c q.
// The pair (p, q) of one column is 32 contiguous bytes: one 256-bit register
// [p.re, p.im, q.re, q.im]; with w = its halves swapped and w' = w with re/im swapped,
//   v <- c v + [s.re, s.re, -s.re, -s.re] w + [-s.im, s.im, -s.im, s.im] w'.
static void rotate_rows(cplx* h, int ld, int cnt, double c, cplx s) {
    double* d = reinterpret_cast<double*>(h);
    const __m256d vc = _mm256_set1_pd(c);
    const __m256d vr = _mm256_setr_pd(s.real(), s.real(), -s.real(), -s.real());
    const __m256d vi = _mm256_setr_pd(-s.imag(), s.imag(), -s.imag(), s.imag());
    for (int j = 0; j < cnt; ++j) {
        double* e = d + 2 * (size_t)j * ld;
        const __m256d v = _mm256_loadu_pd(e);
        const __m256d w = _mm256_permute4x64_pd(v, 0x4E);
        const __m256d w2 = _mm256_permute_pd(w, 0x5);
        _mm256_storeu_pd(e, _mm256_fmadd_pd(vc, v, _mm256_fmadd_pd(vr, w, _mm256_mul_pd(vi, w2))));
    }
}

// Columns a (k) and b (k+1) over cnt contiguous rows:  a <- c a + conj(s) b,  b <- -s a + c b;
// two complex numbers per register, complex products by fmaddsub.
static void rotate_cols(cplx* a, cplx* b, int cnt, double c, cplx s) {
    double* pa = reinterpret_cast<double*>(a);
    double* pb = reinterpret_cast<double*>(b);
    const __m256d vc = _mm256_set1_pd(c);
    const __m256d sr = _mm256_set1_pd(s.real()), si = _mm256_set1_pd(s.imag());
    int i = 0;
    for (; i + 2 <= cnt; i += 2) {
        const __m256d va = _mm256_loadu_pd(pa + 2 * i), vb = _mm256_loadu_pd(pb + 2 * i);
        const __m256d sa = _mm256_permute_pd(va, 0x5), sb = _mm256_permute_pd(vb, 0x5);
        // conj(s) b = (sr b.re + si b.im, sr b.im - si b.re): fmsubadd subtracts in odd lanes
        const __m256d cb = _mm256_fmsubadd_pd(sr, vb, _mm256_mul_pd(si, sb));
        // s a = (sr a.re - si a.im, sr a.im + si a.re)
        const __m256d sa2 = _mm256_fmaddsub_pd(sr, va, _mm256_mul_pd(si, sa));
        _mm256_storeu_pd(pa + 2 * i, _mm256_fmadd_pd(vc, va, cb));
        _mm256_storeu_pd(pb + 2 * i, _mm256_fmsub_pd(vc, vb, sa2));
    }
    for (; i < cnt; ++i) {
        const cplx p = a[i], q = b[i];
        a[i] = c * p + std::conj(s) * q;
        b[i] = -s * p + c * q;
    }
}

// Householder reduction to Hessenberg form (the reflectors kept for the eigenvectors), then the
// shifted QR algorithm on the active window for the eigenvalues only; the window is stored with
// an odd leading dimension so that the row rotations do not fall into a few cache sets.  The
// reduction's three O(N^2) updates per column are split over host threads above N = 128.
bool HessEig::compute(int N_, std::vector<cplx>& A) {
    N = N_;
    H.swap(A);
    V.assign((size_t)N * N, 0.0);
    beta.assign(N, 0.0);
    std::vector<cplx> s(N);
    // each reduction step ends in barriers: one thread up to N = 200 (measured on the MI355X machine's host CPU,
    // reduction and QR sweeps together: N = 162, 6.2 ms on one thread against 7.5-10 ms on six;
    // N = 132, 3.8 ms against 4.8-6.7 ms on four), the thread budget above (whole solves of the
    // batched eight-region workload with companion matrices of N = 256: 322-333 ms with it,
    // 352-392 ms with two threads)
    const int P = N <= 200 ? 1 : host_threads((int64_t)N * N, 4096);
    Team team(P);
    cplx alpha_k = 0.0;
    std::vector<char> skip(N, 0);
    team.run([&](int t) {
        for (int k = 0; k + 2 < N; ++k) {
            if (t == 0) {   // reflector for column k
                double xn2 = 0.0;
                for (int i = k + 1; i < N; ++i) xn2 += std::norm(H[i + (size_t)k * N]);
                cplx* v = &V[(size_t)k * N];
                if (xn2 == 0.0) {
                    skip[k] = 1;
                } else {
                    const double xn = std::sqrt(xn2);
                    const cplx x0 = H[k + 1 + (size_t)k * N];
                    const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0);
                    alpha_k = -ph * xn;
                    for (int i = k + 1; i < N; ++i) v[i] = H[i + (size_t)k * N];
                    v[k + 1] -= alpha_k;
                    double vn2 = 0.0;
                    for (int i = k + 1; i < N; ++i) vn2 += std::norm(v[i]);
                    if (vn2 == 0.0) skip[k] = 1;
                    else beta[k] = 2.0 / vn2;
                }
            }
            if (P > 1) team.barrier();
            if (skip[k]) continue;
            const cplx* v = &V[(size_t)k * N];
            const double bt = beta[k];
            const int cols = N - (k + 1);
            const int j0 = k + 1 + (int)((int64_t)cols * t / P), j1 = k + 1 + (int)((int64_t)cols * (t + 1) / P);
            // H <- (I - bt v v^H) H on rows k+1.., columns k+1..
            for (int j = j0; j < j1; ++j) {
                cplx* hj = &H[(size_t)j * N];
                cplx tt = cdotc(N - k - 1, v + k + 1, hj + k + 1);
                tt *= bt;
                caxpy(N - k - 1, -tt, v + k + 1, hj + k + 1);
            }
            if (P > 1) team.barrier();
            // s = H v over all rows (this thread's row range)
            const int i0 = (int)((int64_t)N * t / P), i1 = (int)((int64_t)N * (t + 1) / P);
            for (int i = i0; i < i1; ++i) s[i] = 0.0;
            for (int j = k + 1; j < N; ++j) {
                const cplx vj = v[j];
                const cplx* hj = &H[(size_t)j * N];
                caxpy(i1 - i0, vj, hj + i0, &s[i0]);
            }
            if (P > 1) team.barrier();
            // H <- H (I - bt v v^H) on columns k+1..
            for (int j = j0; j < j1; ++j) {
                const cplx cv = bt * std::conj(v[j]);
                cplx* hj = &H[(size_t)j * N];
                caxpy(N, -cv, s.data(), hj);
            }
            if (P > 1) team.barrier();
            if (t == 0) {
                H[k + 1 + (size_t)k * N] = alpha_k;
                for (int i = k + 2; i < N; ++i) H[i + (size_t)k * N] = 0.0;
            }
        }
    });
    H0 = H;   // Hessenberg matrix before the QR sweeps (for inverse iteration)
    norm = 0.0;
    for (size_t e = 0; e < (size_t)N * N; ++e) norm = std::max(norm, abs1(H0[e]));
    if (norm == 0.0) norm = 1.0;
    const int LD = N + ((N % 2 == 0) ? 1 : 0);
    {
        std::vector<cplx> Hp((size_t)LD * N);
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) Hp[i + (size_t)j * LD] = H0[i + (size_t)j * N];
        H.swap(Hp);
    }
    int ihi = N - 1, its = 0, total = 0;
    while (ihi >= 0) {
        int l = ihi;
        while (l > 0) {
            double sc = abs1(H[l - 1 + (size_t)(l - 1) * LD]) + abs1(H[l + (size_t)l * LD]);
            if (sc == 0.0) sc = norm;
            if (abs1(H[l + (size_t)(l - 1) * LD]) <= kEps * sc) {
                H[l + (size_t)(l - 1) * LD] = 0.0;
                break;
            }
            --l;
        }
        if (l == ihi) {
            --ihi;
            its = 0;
            continue;
        }
        if (++its > 80 || ++total > 100 * N) return false;
        cplx mu;
        const cplx a = H[ihi - 1 + (size_t)(ihi - 1) * LD], b = H[ihi - 1 + (size_t)ihi * LD];
        const cplx c = H[ihi + (size_t)(ihi - 1) * LD], d = H[ihi + (size_t)ihi * LD];
        if (its == 10 || its == 20 || its == 40) {
            mu = d + std::abs(c.real()) * 0.75;
        } else {
            const cplx tr2 = 0.5 * (a + d);
            const cplx disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
            const cplx m1 = tr2 + disc, m2 = tr2 - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        cplx x = H[l + (size_t)l * LD] - mu, y = H[l + 1 + (size_t)l * LD];
        for (int k = l; k < ihi; ++k) {
            if (k > l) {
                x = H[k + (size_t)(k - 1) * LD];
                y = H[k + 1 + (size_t)(k - 1) * LD];
            }
            double cs;
            cplx sn, rho;
            givens(x, y, cs, sn, rho);
            if (k > l) {
                H[k + (size_t)(k - 1) * LD] = rho;
                H[k + 1 + (size_t)(k - 1) * LD] = 0.0;
            }
            rotate_rows(&H[k + (size_t)k * LD], LD, ihi - k + 1, cs, sn);   // rows k, k+1 in the window
            const int iend = std::min(k + 2, ihi);
            rotate_cols(&H[l + (size_t)k * LD], &H[l + (size_t)(k + 1) * LD], iend - l + 1, cs, sn);
        }
    }
    evals.resize(N);
    for (int i = 0; i < N; ++i) evals[i] = H[i + (size_t)i * LD];
    H.clear();
    return true;
}

void HessEig::vectors(const std::vector<int>& want, std::vector<cplx>& out) const {
    out.assign((size_t)N * want.size(), 0.0);
    // row-major copy of the Hessenberg matrix: the elimination below works on rows
    std::vector<cplx> Hr((size_t)N * N);
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) Hr[(size_t)i * N + j] = H0[i + (size_t)j * N];
    const double smin = std::max(kEps * norm, std::numeric_limits<double>::min() * N);
    // the wanted vectors are independent: spread them over host threads
    const int P = host_threads((int64_t)want.size() * N * N, (int64_t)4 * N * N);
    auto one = [&](size_t q, std::vector<cplx>& M, std::vector<cplx>& x, std::vector<int>& piv) {
        const cplx lam = evals[want[q]];
        // LU of H0 - lam I with row exchanges between neighbours only (row i of M at M + i N)
        M = Hr;
        for (int i = 0; i < N; ++i) M[(size_t)i * N + i] -= lam;
        for (int k = 0; k + 1 < N; ++k) {
            cplx* rk = &M[(size_t)k * N];
            cplx* rk1 = &M[(size_t)(k + 1) * N];
            piv[k] = k;
            if (abs1(rk1[k]) > abs1(rk[k])) {
                piv[k] = k + 1;
                for (int j = k; j < N; ++j) std::swap(rk[j], rk1[j]);
            }
            if (rk[k] == 0.0) rk[k] = smin;
            const cplx lk = rk1[k] / rk[k];
            rk1[k] = lk;
            if (lk != 0.0) caxpy(N - k - 1, -lk, rk + k + 1, rk1 + k + 1);
        }
        if (M[(size_t)(N - 1) * N + N - 1] == 0.0) M[(size_t)(N - 1) * N + N - 1] = smin;
        for (int i = 0; i < N; ++i) x[i] = 1.0 / std::sqrt((double)N);
        for (int it = 0; it < 2; ++it) {
            for (int k = 0; k + 1 < N; ++k) {          // forward: L^{-1} P x
                if (piv[k] != k) std::swap(x[k], x[k + 1]);
                x[k + 1] -= M[(size_t)(k + 1) * N + k] * x[k];
            }
            for (int i = N - 1; i >= 0; --i) {         // back: U^{-1}
                const cplx* ri = &M[(size_t)i * N];
                const cplx t = x[i] - cdotu(N - i - 1, ri + i + 1, &x[i + 1]);
                cplx d = ri[i];
                if (std::abs(d) < smin) d = smin;
                x[i] = t / d;
            }
            double nr = 0.0;
            for (int i = 0; i < N; ++i) nr += std::norm(x[i]);
            nr = std::sqrt(nr);
            for (int i = 0; i < N; ++i) x[i] /= nr;
        }
        // back-transform with the reflectors: x <- P_0 P_1 ... P_{N-3} x
        for (int k = N - 3; k >= 0; --k) {
            if (beta[k] == 0.0) continue;
            const cplx* v = &V[(size_t)k * N];
            cplx t = cdotc(N - k - 1, v + k + 1, &x[k + 1]);
            t *= beta[k];
            caxpy(N - k - 1, -t, v + k + 1, &x[k + 1]);
        }
        double nr = 0.0;
        for (int i = 0; i < N; ++i) nr += std::norm(x[i]);
        nr = std::sqrt(nr);
        cplx* o = &out[(size_t)q * N];
        for (int i = 0; i < N; ++i) o[i] = x[i] / nr;
    };
    std::atomic<size_t> next{0};
    auto worker = [&] {
        std::vector<cplx> M((size_t)N * N), x(N);
        std::vector<int> piv(N);
        for (size_t q; (q = next.fetch_add(1)) < want.size();) one(q, M, x, piv);
    };
    if (P <= 1) {
        worker();
    } else {
        std::vector<std::thread> ts;
        for (int t = 0; t < P; ++t) ts.emplace_back(worker);
        for (auto& t : ts) t.join();
    }
}

// LU with partial pivoting (|Re| + |Im| pivots) of an m x m matrix; solves M X = B in place.
// pivot_ratio (optional) receives min |u_kk| / max |u_kk|.
static bool lu_solve_small(int m, std::vector<cplx> M, cplx* B, int nrhs, double* pivot_ratio = nullptr) {
    std::vector<int> piv(m);
    double umin = INFINITY, umax = 0.0;
    for (int k = 0; k < m; ++k) {
        int p = k;
        double best = abs1(M[k + (size_t)k * m]);
        for (int i = k + 1; i < m; ++i) {
            const double v = abs1(M[i + (size_t)k * m]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return false;
        umin = std::min(umin, best);
        umax = std::max(umax, best);
        if (p != k)
            for (int j = 0; j < m; ++j) std::swap(M[k + (size_t)j * m], M[p + (size_t)j * m]);
        const cplx inv = 1.0 / M[k + (size_t)k * m];
        for (int i = k + 1; i < m; ++i) M[i + (size_t)k * m] *= inv;
        for (int j = k + 1; j < m; ++j) {
            const cplx u = M[k + (size_t)j * m];
            if (u == 0.0) continue;
            for (int i = k + 1; i < m; ++i) M[i + (size_t)j * m] -= M[i + (size_t)k * m] * u;
        }
    }
    if (pivot_ratio) *pivot_ratio = umin / umax;
    for (int c = 0; c < nrhs; ++c) {
        cplx* b = B + (size_t)c * m;
        for (int k = 0; k < m; ++k)
            if (piv[k] != k) std::swap(b[k], b[piv[k]]);
        for (int k = 0; k < m; ++k)
            for (int i = k + 1; i < m; ++i) b[i] -= M[i + (size_t)k * m] * b[k];
        for (int k = m - 1; k >= 0; --k) {
            b[k] /= M[k + (size_t)k * m];
            for (int i = 0; i < k; ++i) b[i] -= M[i + (size_t)k * m] * b[k];
        }
    }
    return true;
}

// Taylor coefficients of f(c + mu) up to degree d.
static std::vector<cplx> taylor(const Term& t, cplx c, int d) {
    std::vector<cplx> out(d + 1, 0.0);
    if (t.kind == 0) {
        const int p = (int)t.param;
        double binom = 1.0;
        for (int q = 0; q <= std::min(p, d); ++q) {
            cplx cp = 1.0;
            for (int i = 0; i < p - q; ++i) cp *= c;
            out[q] = binom * cp;
            binom = binom * (p - q) / (q + 1);
        }
    } else {
        const cplx e = std::exp(-t.param * c);
        double f = 1.0;
        for (int q = 0; q <= d; ++q) {
            if (q > 0) f *= q;
            out[q] = e * std::pow(-t.param, q) / f;
        }
    }
    return out;
}

// Shift for the inverted linearisation: the contour centre unless a previous Ritz value lies
// within 0.2 rho of it (rho = smaller semi-axis), else the candidate on the circle of radius
// rho / 2 farthest from every previous Ritz value.  An eigenvalue at the shift makes
// T_red(shift) singular and the inverted companion matrix huge, which costs every other Ritz
// value its accuracy.
static std::vector<cplx> shift_candidates(const Ellipse& E, const std::vector<cplx>* avoid) {
    const double rho = std::min(E.a, E.b);
    std::vector<cplx> cand;
    cand.push_back(E.c);
    for (int k = 0; k < 7; ++k) {
        const double th = 2.0 * kPi * k / 7.0 + 0.3;
        cand.push_back(E.c + 0.5 * rho * cplx(std::cos(th), std::sin(th)));
    }
    if (!avoid || avoid->empty()) return cand;
    auto dist = [&](cplx s) {
        double d = INFINITY;
        for (cplx l : *avoid)
            if (std::isfinite(l.real()) && std::isfinite(l.imag())) d = std::min(d, std::abs(l - s));
        return d / rho;
    };
    std::vector<std::pair<double, int>> score;
    for (size_t i = 0; i < cand.size(); ++i) {
        double d = dist(cand[i]);
        if (i == 0 && d >= 0.2) d = INFINITY;        // keep the centre when it is clear
        score.push_back({-d, (int)i});
    }
    std::stable_sort(score.begin(), score.end());
    std::vector<cplx> out;
    for (auto& sc : score) out.push_back(cand[sc.second]);
    return out;
}

// Newton on F(y, l) = [T(l) y; v^H y - 1], Jacobian [[T(l), T'(l) y], [v^H, 0]] (v the
// starting vector), on the exact reduced function, for the pairs (lam[q], Y[:, q]) with q in
// todo (Y: m rows, ld m); the pairs are independent and are spread over host threads.  Each
// refined vector is returned with unit norm.
static int newton_polish(int m, const std::vector<Term>& terms, const cplx* Ahat, std::vector<cplx>& lam,
                         std::vector<cplx>& Yv, const std::vector<int>& todo) {
    const int J = (int)terms.size();
    const size_t mm = (size_t)m * m;
    std::atomic<int> steps{0};
    std::vector<double> anorm(J);   // ||Ahat_j||_F, for the scale of the residual test
    for (int j = 0; j < J; ++j) anorm[j] = std::sqrt(csumsq((int64_t)mm, Ahat + (size_t)j * mm));
    auto polish = [&](int q) {
        std::vector<cplx> Jm((size_t)(m + 1) * (m + 1)), rhs(m + 1), Tl(mm), dT(mm);
        cplx l = lam[q];
        std::vector<cplx> y(Yv.begin() + (size_t)q * m, Yv.begin() + (size_t)(q + 1) * m);
        const std::vector<cplx> v0 = y;   // unit norm, so v0^H y = 1 initially
        for (int it = 0; it < 8; ++it) {
            std::fill(Tl.begin(), Tl.end(), cplx(0.0));
            double scale = 0.0;
            for (int j = 0; j < J; ++j) {
                const cplx f = term_value(terms[j], l);
                const cplx* A = Ahat + (size_t)j * mm;
                caxpy((int64_t)mm, f, A, Tl.data());
                scale += std::abs(f) * anorm[j];
            }
            if (!std::isfinite(scale)) break;
            double rn = 0.0;
            for (int r = 0; r < m; ++r) rhs[r] = 0.0;
            for (int c = 0; c < m; ++c) caxpy(m, -y[c], &Tl[(size_t)c * m], rhs.data());
            for (int r = 0; r < m; ++r) rn += std::norm(rhs[r]);
            cplx vy = 0.0;
            for (int i = 0; i < m; ++i) vy += std::conj(v0[i]) * y[i];
            rhs[m] = -(vy - 1.0);
            if (std::sqrt(rn) <= 1e-15 * scale && std::abs(rhs[m]) < 1e-15) break;
            // T'(l) only when a step is taken
            std::fill(dT.begin(), dT.end(), cplx(0.0));
            for (int j = 0; j < J; ++j) caxpy((int64_t)mm, term_deriv(terms[j], l), Ahat + (size_t)j * mm, dT.data());
            for (int c = 0; c < m; ++c)
                for (int r = 0; r < m; ++r) Jm[r + (size_t)c * (m + 1)] = Tl[r + (size_t)c * m];
            for (int r = 0; r < m; ++r) Jm[r + (size_t)m * (m + 1)] = 0.0;
            for (int c = 0; c < m; ++c)
                for (int r = 0; r < m; ++r) Jm[r + (size_t)m * (m + 1)] += dT[r + (size_t)c * m] * y[c];
            for (int c = 0; c < m; ++c) Jm[m + (size_t)c * (m + 1)] = std::conj(v0[c]);
            Jm[m + (size_t)m * (m + 1)] = 0.0;
            if (!lu_solve_small(m + 1, Jm, rhs.data(), 1)) break;
            steps.fetch_add(1);
            for (int i = 0; i < m; ++i) y[i] += rhs[i];
            l += rhs[m];
        }
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += std::norm(y[i]);
        s = std::sqrt(s);
        for (int i = 0; i < m; ++i) Yv[(size_t)q * m + i] = y[i] / s;
        lam[q] = l;
    };
    const int hw = std::min((int)std::max(1u, std::thread::hardware_concurrency()), host_thread_budget());
    const int nth = std::max(1, std::min({hw, 16, (int)todo.size() / 2}));
    if (nth <= 1 || (size_t)m * m * todo.size() < 200000) {
        for (int q : todo) polish(q);
    } else {
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&] {
                for (size_t i; (i = next.fetch_add(1)) < todo.size();) polish(todo[i]);
            });
        for (auto& t : pool) t.join();
    }
    return steps.load();
}

// Householder QR with column pivoting of the N x N matrix A (column-major, overwritten: R on
// and above the diagonal, the reflectors' tails below, LAPACK's convention H = I - tau v v^H,
// v(0) = 1).  Column j is the remaining column of largest norm; the factorisation stops at the
// first step whose pivot norm is at most `thresh`.  Returns that numerical rank.
static int pivoted_qr(int N, std::vector<cplx>& A, std::vector<cplx>& tau, std::vector<int>& perm, double thresh) {
    perm.resize(N);
    std::iota(perm.begin(), perm.end(), 0);
    tau.assign(N, 0.0);
    // squared norms of the remaining parts of the columns, downdated after every step and
    // recomputed when the downdate has cancelled most of the value
    std::vector<double> nrm2(N), ref(N);
    auto colnorm = [&](int c, int from) {
        return csumsq(N - from, &A[(size_t)c * N + from]);
    };
    const int nth = host_threads((int64_t)N * N, 1 << 14);
    std::atomic<int> rank{N};
    Team team(nth);
    team.run([&](int t) {
        for (int c = t; c < N; c += nth) nrm2[c] = ref[c] = colnorm(c, 0);
        team.barrier();
        for (int j = 0; j < N; ++j) {
            if (t == 0) {
                int p = j;
                for (int c = j + 1; c < N; ++c)
                    if (nrm2[c] > nrm2[p]) p = c;
                if (p != j) {
                    std::swap_ranges(A.begin() + (size_t)j * N, A.begin() + (size_t)(j + 1) * N,
                                     A.begin() + (size_t)p * N);
                    std::swap(perm[j], perm[p]);
                    std::swap(nrm2[j], nrm2[p]);
                    std::swap(ref[j], ref[p]);
                }
                const double nrm = std::sqrt(colnorm(j, j));
                if (nrm == 0.0 || nrm <= thresh) {
                    rank.store(j);
                } else {
                    cplx* a = &A[(size_t)j * N];
                    const cplx alpha = a[j];
                    const double beta = alpha.real() >= 0.0 ? -nrm : nrm;
                    const cplx tj = cplx((beta - alpha.real()) / beta, -alpha.imag() / beta);
                    const cplx scl = 1.0 / (alpha - beta);
                    for (int i = j + 1; i < N; ++i) a[i] *= scl;
                    a[j] = beta;
                    tau[j] = tj;
                }
            }
            team.barrier();
            if (rank.load() <= j) return;
            const cplx* a = &A[(size_t)j * N];
            const cplx ct = std::conj(tau[j]);
            for (int c = j + 1 + t; c < N; c += nth) {   // column c <- (I - conj(tau) v v^H) column c
                cplx* b = &A[(size_t)c * N];
                cplx w = b[j] + cdotc(N - j - 1, a + j + 1, b + j + 1);
                w *= ct;
                b[j] -= w;
                caxpy(N - j - 1, -w, a + j + 1, b + j + 1);
                const double d = nrm2[c] - std::norm(b[j]);
                if (d <= 1e-6 * ref[c]) {
                    nrm2[c] = ref[c] = colnorm(c, j + 1);
                } else {
                    nrm2[c] = d;
                }
            }
            team.barrier();
        }
    });
    return rank.load();
}

void contour_points(const Ellipse& E, std::vector<cplx>& z, std::vector<cplx>& w, std::vector<cplx>& mu) {
    const int NP = CONTOUR_POINTS;
    const double a = CONTOUR_SCALE * E.a, b = CONTOUR_SCALE * E.b, L = std::max(a, b);
    z.resize(NP);
    w.resize(NP);
    mu.resize(NP);
    for (int q = 0; q < NP; ++q) {
        const double th = 2.0 * kPi * (q + 0.5) / NP;
        z[q] = E.c + cplx(a * std::cos(th), b * std::sin(th));
        // (1/2 pi i) dz/dtheta (2 pi / NP)
        w[q] = cplx(-a * std::sin(th), b * std::cos(th)) / cplx(0.0, (double)NP);
        mu[q] = (z[q] - E.c) / L;
    }
}

// The moments on the host: T(z_q) assembled, inverted by LU (points dealt to threads in a fixed
// pattern q = t, t + nth, ..., each thread with its own partial sums, added in thread order, so
// the sums do not depend on timing).
static bool contour_moments_host(int m, const std::vector<Term>& terms, const cplx* Ahat, const Ellipse& E,
                                 std::vector<cplx>& M, std::vector<double>& isize) {
    const int J = (int)terms.size(), NP = CONTOUR_POINTS, NM = CONTOUR_MOMENTS;
    const size_t mm = (size_t)m * m;
    std::vector<cplx> z, w, mu;
    contour_points(E, z, w, mu);
    std::vector<cplx> fz((size_t)J * NP);   // the functions at every point, one call per term
    for (int j = 0; j < J; ++j) term_values(terms[j], z.data(), NP, &fz[(size_t)j * NP]);
    const int hw = std::min((int)std::max(1u, std::thread::hardware_concurrency()), host_thread_budget());
    const int nth = std::max(1, std::min({hw, 16, NP / 4, (int)(mm * NP / 20000) + 1}));
    std::vector<std::vector<cplx>> part(nth, std::vector<cplx>(NM * mm, 0.0));
    isize.assign(NP, 0.0);   // |w_q| ||T(z_q)^{-1}||_F, the integrand's size
    std::atomic<int> bad{0};
    auto work = [&](int t) {
        std::vector<cplx> Tz(mm), Inv(mm);
        for (int q = t; q < NP; q += nth) {
            std::fill(Tz.begin(), Tz.end(), cplx(0.0));
            for (int j = 0; j < J; ++j) {
                const cplx f = fz[(size_t)j * NP + q];
                const cplx* A = Ahat + (size_t)j * mm;
                for (size_t e = 0; e < mm; ++e) Tz[e] += f * A[e];
            }
            std::fill(Inv.begin(), Inv.end(), cplx(0.0));
            for (int i = 0; i < m; ++i) Inv[i + (size_t)i * m] = 1.0;
            if (!lu_solve_small(m, Tz, Inv.data(), m)) {
                bad.store(1);
                continue;
            }
            double fro = 0.0;
            for (size_t e = 0; e < mm; ++e) fro += std::norm(Inv[e]);
            isize[q] = std::abs(w[q]) * std::sqrt(fro);
            cplx wp = w[q];
            for (int p = 0; p < NM; ++p, wp *= mu[q]) {
                cplx* Mp = &part[t][(size_t)p * mm];
                for (size_t e = 0; e < mm; ++e) Mp[e] += wp * Inv[e];
            }
        }
    };
    if (nth == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t) pool.emplace_back(work, t);
        for (auto& th : pool) th.join();
    }
    if (bad.load()) return false;
    M.assign(NM * mm, 0.0);
    for (int t = 0; t < nth; ++t)
        for (size_t e = 0; e < M.size(); ++e) M[e] += part[t][e];
    return true;
}

bool contour_pairs_from_moments(int m, const Ellipse& E, const std::vector<cplx>& M,
                                const std::vector<double>& isize, std::vector<cplx>& lam,
                                std::vector<cplx>& Y) {
    const size_t mm = (size_t)m * m;
    const double L = CONTOUR_SCALE * std::max(E.a, E.b);
    int K = 2, N = 0, k = 0;
    std::vector<cplx> H0, tau;
    std::vector<int> perm;
    for (; K <= CONTOUR_KMAX; ++K) {
        N = K * m;
        H0.assign((size_t)N * N, 0.0);
        for (int bi = 0; bi < K; ++bi)
            for (int bj = 0; bj < K; ++bj) {
                const cplx* Mp = &M[(size_t)(bi + bj) * mm];
                for (int c = 0; c < m; ++c)
                    for (int r = 0; r < m; ++r)
                        H0[(size_t)(bi * m + r) + (size_t)(bj * m + c) * N] = Mp[r + (size_t)c * m];
            }
        k = pivoted_qr(N, H0, tau, perm, CONTOUR_RANK_TOL * std::accumulate(isize.begin(), isize.end(), 0.0));
        if (k < N) break;
    }
    if (K > CONTOUR_KMAX) return false;
    lam.clear();
    Y.clear();
    if (k == 0) return true;
    const int nth = host_threads((int64_t)N * k * k, 1 << 18);
    // Q_k = H_0 ... H_{k-1} [I_k; 0], column by column (columns are independent)
    std::vector<cplx> Qk((size_t)N * k, 0.0);
    for (int i = 0; i < k; ++i) Qk[i + (size_t)i * N] = 1.0;
    // G = Q_k^H H1 P_k (k x k), with column c of H1 P_k = block column of H1 for perm[c]
    std::vector<cplx> G((size_t)k * k, 0.0);
    Team(nth).run([&](int t) {
        for (int c = t; c < k; c += nth) {
            cplx* q = &Qk[(size_t)c * N];
            for (int j = std::min(c, k - 1); j >= 0; --j) {   // H_j leaves e_c alone for j > c
                const cplx* v = &H0[(size_t)j * N];
                cplx s = q[j] + cdotc(N - j - 1, v + j + 1, q + j + 1);
                s *= tau[j];
                q[j] -= s;
                caxpy(N - j - 1, -s, v + j + 1, q + j + 1);
            }
        }
    });
    Team(nth).run([&](int t) {
        std::vector<cplx> h1(N);
        for (int c = t; c < k; c += nth) {
            const int col = perm[c], bj = col / m, cc = col % m;
            for (int bi = 0; bi < K; ++bi) {
                const cplx* Mp = &M[(size_t)(bi + bj + 1) * mm];
                for (int r = 0; r < m; ++r) h1[bi * m + r] = Mp[r + (size_t)cc * m];
            }
            for (int i = 0; i < k; ++i) {
                const cplx* q = &Qk[(size_t)i * N];
                G[i + (size_t)c * k] = cdotc(N, q, h1.data());
            }
        }
    });
    // B = G R_11^{-1}: row i of B from B R_11 = G, left to right (rows are independent)
    std::vector<cplx> B((size_t)k * k);
    Team(nth).run([&](int t) {
        for (int i = t; i < k; i += nth)
            for (int c = 0; c < k; ++c) {
                cplx s = G[i + (size_t)c * k];
                for (int p = 0; p < c; ++p) s -= B[i + (size_t)p * k] * H0[p + (size_t)c * N];
                B[i + (size_t)c * k] = s / H0[c + (size_t)c * N];
            }
    });
    std::vector<cplx> ev, S;
    if (k == 1) {
        ev.assign(1, B[0]);
        S.assign(1, 1.0);
    } else {
        HessEig he;
        if (!he.compute(k, B)) return false;
        ev = he.evals;
        std::vector<int> all(k);
        std::iota(all.begin(), all.end(), 0);
        he.vectors(all, S);
    }
    lam.resize(k);
    Y.assign((size_t)m * k, 0.0);
    for (int i = 0; i < k; ++i) lam[i] = E.c + L * ev[i];
    // y_i = the first block of Q_k s_i, normalised (the vectors are independent)
    Team(nth).run([&](int t) {
        for (int i = t; i < k; i += nth) {
            cplx* y = &Y[(size_t)i * m];
            for (int p = 0; p < k; ++p) {
                const cplx sp = S[p + (size_t)i * k];
                const cplx* q = &Qk[(size_t)p * N];
                caxpy(m, sp, q, y);
            }
            const double nn = std::sqrt(csumsq(m, y));
            if (nn > 0.0)
                for (int r = 0; r < m; ++r) y[r] /= nn;
        }
    });
    return true;
}

bool contour_pairs(int m, const std::vector<Term>& terms, const cplx* Ahat, const Ellipse& E,
                   std::vector<cplx>& lam, std::vector<cplx>& Y, double* ms_points, double* ms_rank_eig) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<cplx> M;
    std::vector<double> isize;
    if (!contour_moments_host(m, terms, Ahat, E, M, isize)) return false;
    const auto t1 = std::chrono::steady_clock::now();
    const bool ok = contour_pairs_from_moments(m, E, M, isize, lam, Y);
    if (ms_points) *ms_points = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (ms_rank_eig)
        *ms_rank_eig = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
    return ok;
}

// Steps 1-2 by the contour-integral solve: the pairs inside the enlarged ellipse, refined by
// Newton, sorted by normalised radius and completed to m_keep (see reduced_solve).
// The pairs found (lam, Y), refined by Newton, sorted by normalised radius and completed to m_keep.
static ReducedResult contour_finish(int m, const std::vector<Term>& terms, const cplx* Ahat, const Ellipse& E,
                                    int m_keep, std::vector<cplx>& lam, std::vector<cplx>& Y, ReducedResult res) {
    res.rank = (int)lam.size();
    std::vector<int> todo;
    for (int q = 0; q < (int)lam.size(); ++q)
        if (std::isfinite(lam[q].real()) && E.radius(lam[q]) < CONTOUR_SCALE) todo.push_back(q);
    const auto t0 = std::chrono::steady_clock::now();
    res.newton_steps = newton_polish(m, terms, Ahat, lam, Y, todo);
    res.newton_pairs = (int)todo.size();
    res.ms_newton = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::vector<double> rad(todo.size());
    for (size_t i = 0; i < todo.size(); ++i) rad[i] = E.radius(lam[todo[i]]);
    std::vector<int> order(todo.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return rad[p] < rad[q]; });
    const int kf = std::min((int)order.size(), m_keep);
    res.lambda.resize(m_keep);
    res.Y.assign((size_t)m * m_keep, 0.0);
    res.found.assign(m_keep, 0);
    for (int i = 0; i < kf; ++i) {
        const int q = todo[order[i]];
        res.lambda[i] = lam[q];
        std::copy(Y.begin() + (size_t)q * m, Y.begin() + (size_t)(q + 1) * m, res.Y.begin() + (size_t)i * m);
        res.found[i] = 1;
    }
    // completion: an orthonormal basis B of the found vectors' span (Gram-Schmidt, twice), then
    // unit vectors e_r orthogonalised (twice) against B and the completions so far, kept when a
    // part of norm >= 0.5/sqrt(m) survives (the projections of all e_r onto a complement of
    // dimension d have squared norms summing to d, so enough e_r always pass), with values spread
    // over the enlarged ellipse
    std::vector<cplx> B((size_t)m * m, 0.0), v(m);
    int nb = 0;
    auto orthogonalise = [&](std::vector<cplx>& x) {
        for (int pass = 0; pass < 2; ++pass)
            for (int c = 0; c < nb; ++c) {
                const cplx* u = &B[(size_t)c * m];
                caxpy(m, -cdotc(m, u, x.data()), u, x.data());
            }
        return std::sqrt(csumsq(m, x.data()));
    };
    // (the basis only serves the completion: with m_keep vectors found there is nothing to add)
    for (int c = 0; c < kf && kf < m_keep; ++c) {
        std::copy(res.Y.begin() + (size_t)c * m, res.Y.begin() + (size_t)(c + 1) * m, v.begin());
        const double nn = orthogonalise(v);
        if (nn < 1e-8) continue;   // numerically inside the span already
        for (int i = 0; i < m; ++i) B[(size_t)nb * m + i] = v[i] / nn;
        ++nb;
    }
    int col = kf;
    for (int r = 0; r < m && col < m_keep; ++r) {
        std::fill(v.begin(), v.end(), cplx(0.0));
        v[r] = 1.0;
        const double nn = orthogonalise(v);
        if (nn < 0.5 / std::sqrt((double)m)) continue;
        for (int i = 0; i < m; ++i) {
            B[(size_t)nb * m + i] = v[i] / nn;
            res.Y[(size_t)col * m + i] = v[i] / nn;
        }
        ++nb;
        ++col;
    }
    if (col < m_keep) {   // not reached for m_keep <= m (see above); kept as a guard
        res.ok = false;
        return res;
    }
    const int pad = m_keep - kf;
    for (int i = 0; i < pad; ++i) {
        const double th = 2.0 * kPi * (i + 0.5) / pad;
        res.lambda[kf + i] = E.c + CONTOUR_SCALE * cplx(E.a * std::cos(th), E.b * std::sin(th));
    }
    res.n_finite = m_keep;
    return res;
}

static ReducedResult contour_reduced(int m, const std::vector<Term>& terms, const cplx* Ahat, const Ellipse& E,
                                     int m_keep) {
    ReducedResult res;
    std::vector<cplx> lam, Y;
    if (m_keep > m || !contour_pairs(m, terms, Ahat, E, lam, Y, &res.ms_points, &res.ms_rank_eig)) {
        res.ok = false;
        return res;
    }
    return contour_finish(m, terms, Ahat, E, m_keep, lam, Y, res);
}

ReducedResult contour_reduced_from_moments(int m, const std::vector<Term>& terms, const cplx* Ahat,
                                           const Ellipse& E, int m_keep, const std::vector<cplx>& M,
                                           const std::vector<double>& isize) {
    ReducedResult res;
    std::vector<cplx> lam, Y;
    const auto t0 = std::chrono::steady_clock::now();
    if (m_keep > m || !contour_pairs_from_moments(m, E, M, isize, lam, Y)) {
        res.ok = false;
        return res;
    }
    res.ms_rank_eig = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return contour_finish(m, terms, Ahat, E, m_keep, lam, Y, res);
}

bool takes_contour_route(const std::vector<Term>& terms, int method) {
    bool poly = true, user = false;
    for (const Term& t : terms) {
        if (t.kind != 0) poly = false;
        if (t.kind == 2) user = true;
    }
    return user || (!poly && method != 2) || method == 3;
}

ReducedResult reduced_solve(int m, const std::vector<Term>& terms, const cplx* Ahat,
                            const Ellipse& E, int m_keep, const std::vector<cplx>* avoid, int method) {
    ReducedResult res;
    const int J = (int)terms.size();
    bool poly = true, user = false;
    int maxpow = 1;
    for (const Term& t : terms) {
        if (t.kind == 0) maxpow = std::max(maxpow, (int)t.param);
        else poly = false;
        if (t.kind == 2) user = true;
    }
    if (user || (!poly && method != 2) || method == 3) return contour_reduced(m, terms, Ahat, E, m_keep);
    const size_t mm = (size_t)m * m;
    const std::vector<cplx> shifts = shift_candidates(E, avoid);
    int deg = maxpow, N = 0;
    cplx sigma = E.c;
    std::vector<cplx> D;
    bool have = false;
    for (cplx sg : shifts) {
        deg = maxpow;
        if (!poly) {
            // smallest d with (tau R)^{d+1} e^{tau R} / (d+1)! <= 1e-4 on the disk about the
            // shift that covers |lambda - c| <= 1.5 max(a, b): the truncated expansion only has
            // to place each Ritz value in the basin of Newton's method on the exact function
            const double R = 1.5 * std::max(E.a, E.b) + std::abs(sg - E.c);
            for (const Term& t : terms) {
                if (t.kind != 1) continue;
                const double x = std::fabs(t.param) * R;
                int e = 1;
                double term = x * x / 2.0;
                while (term * std::exp(x) > 1e-4) {
                    ++e;
                    term *= x / (e + 1);
                }
                deg = std::max(deg, e);
            }
        }
        std::vector<std::vector<cplx>> B(deg + 1, std::vector<cplx>(mm, 0.0));
        for (int j = 0; j < J; ++j) {
            const std::vector<cplx> tc = taylor(terms[j], sg, deg);
            const cplx* A = Ahat + (size_t)j * mm;
            for (int q = 0; q <= deg; ++q) {
                if (tc[q] == 0.0) continue;
                for (size_t e = 0; e < mm; ++e) B[q][e] += tc[q] * A[e];
            }
        }
        // monic polynomial in nu = 1/(lambda - sigma): nu^deg I + sum_{q>=1} nu^{deg-q} D_q,
        // D_q = B_0^{-1} B_q
        D.assign(mm * deg, 0.0);
        for (int q = 1; q <= deg; ++q) std::copy(B[q].begin(), B[q].end(), D.begin() + (size_t)(q - 1) * mm);
        double ratio = 0.0;
        if (lu_solve_small(m, B[0], D.data(), m * deg, &ratio) && ratio > 1e-12) {
            sigma = sg;
            have = true;
            break;
        }
    }
    if (!have) {
        res.ok = false;
        return res;
    }
    N = deg * m;
    std::vector<cplx> M((size_t)N * N, 0.0);
    for (int q = 1; q <= deg; ++q)
        for (int c = 0; c < m; ++c)
            for (int r = 0; r < m; ++r)
                M[r + (size_t)((q - 1) * m + c) * N] = -D[(size_t)(q - 1) * mm + r + (size_t)c * m];
    for (int bI = 1; bI < deg; ++bI)
        for (int i = 0; i < m; ++i) M[(size_t)bI * m + i + (size_t)((bI - 1) * m + i) * N] = 1.0;
    HessEig S;
    if (!S.compute(N, M)) {
        res.ok = false;
        return res;
    }
    const std::vector<cplx>& nu = S.evals;
    std::vector<cplx> lam(N);
    std::vector<double> rad(N);
    for (int i = 0; i < N; ++i) {
        lam[i] = (nu[i] == 0.0) ? cplx(INFINITY, 0.0) : sigma + 1.0 / nu[i];
        rad[i] = E.radius(lam[i]);
    }
    std::vector<int> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return rad[p] < rad[q]; });
    const int keep = std::min(m_keep, N);
    std::vector<int> want(order.begin(), order.begin() + keep);
    std::vector<cplx> V;
    S.vectors(want, V);
    const std::vector<cplx>& nu2 = nu;
    res.lambda.resize(keep);
    res.Y.assign((size_t)m * keep, 0.0);
    for (int q = 0; q < keep; ++q) {
        const int k = want[q];
        res.lambda[q] = (nu2[k] == 0.0) ? cplx(INFINITY, 0.0) : sigma + 1.0 / nu2[k];
        const cplx* v = &V[(size_t)q * N];
        int bb = 0;
        double bn = -1.0;
        for (int bI = 0; bI < deg; ++bI) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += std::norm(v[(size_t)bI * m + i]);
            if (s > bn) { bn = s; bb = bI; }
        }
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += std::norm(v[(size_t)bb * m + i]);
        s = std::sqrt(s);
        for (int i = 0; i < m; ++i) res.Y[(size_t)q * m + i] = v[(size_t)bb * m + i] / s;
    }
    if (!poly) {
        // Newton refinement of the pairs near the contour (normalised radius < 2)
        std::vector<int> todo;
        for (int q = 0; q < keep; ++q)
            if (std::isfinite(res.lambda[q].real()) && E.radius(res.lambda[q]) < 2.0) todo.push_back(q);
        newton_polish(m, terms, Ahat, res.lambda, res.Y, todo);
    }
    res.found.assign(keep, 1);
    res.n_finite = 0;
    for (int q = 0; q < keep; ++q)
        if (std::isfinite(res.lambda[q].real())) ++res.n_finite;
    return res;
}

}  // namespace nlf
