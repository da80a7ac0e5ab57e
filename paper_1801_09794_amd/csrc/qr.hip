// Householder QR of a tall n x m complex block (Step 5 "orthonormalise Q", Algorithm 1), the
// path taken when the block is too ill-conditioned for Cholesky QR: the filtered subspace of
// Step 4 damps the components of eigenvectors far outside the contour to rounding level, and
// the Gram matrix of such a block is numerically singular, while Householder reflections stay
// orthogonal to working precision whatever the rank.
//
// Blocked right-looking factorisation with panels of HB columns: one 1024-thread workgroup
// factors a panel (reflectors written explicitly with unit diagonal into V, and the triangular
// factor T of the block reflector I - V T V^H), complex GEMMs apply it to the trailing columns,
// and the explicit Q = H_1 ... H_p [I; 0] is built by applying the block reflectors in reverse
// order to the first m columns of the identity.  Reflector convention as in LAPACK's zgeqrf:
// H = I - tau v v^H with v(0) = 1 and H^H [alpha; x] = [beta; 0], beta real.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>

namespace nlf {

namespace {

constexpr int QR_NT = 1024;
constexpr int QR_NW = QR_NT / 64;

// Sum of cnt doubles over the workgroup; every thread receives the totals in out (LDS).
__device__ void block_sum(double* v, int cnt, double (*red)[4 * QR_HB], double* out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q = 0; q < cnt; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[wave][q] = x;
    }
    __syncthreads();
    if (tid < cnt) {
        double x = 0.0;
        for (int w = 0; w < QR_NW; ++w) x += red[w][tid];
        out[tid] = x;
    }
    __syncthreads();
}

// Householder factorisation of the panel A[j0:n, j0:j0+b] (b <= QR_HB) in place; writes the
// reflectors to V[:, j0:j0+b] (zero above the diagonal, one on it) and T (ld QR_HB).
__global__ __launch_bounds__(QR_NT) void house_panel_kernel(int64_t n, int64_t j0, int b, z128* A,
                                                             z128* V, z128* T) {
    __shared__ double red[QR_NW][4 * QR_HB];
    __shared__ double tot[4 * QR_HB];
    const int tid = threadIdx.x;
    for (int k = 0; k < b; ++k) {
        const int64_t j = j0 + k;
        z128* a = A + j * n;
        // (1) squared norm below the diagonal
        double s = 0.0;
        for (int64_t r = j + 1 + tid; r < n; r += QR_NT) s += norm2(a[r]);
        block_sum(&s, 1, red, tot);
        const double xn2 = tot[0];
        const z128 alpha = a[j];
        z128 tau(0.0, 0.0), scl(0.0, 0.0);
        double beta = alpha.re;
        if (xn2 > 0.0 || alpha.im != 0.0) {
            const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
            beta = alpha.re >= 0.0 ? -nrm : nrm;
            tau = z128((beta - alpha.re) / beta, -alpha.im / beta);
            scl = cdiv(z128(1.0, 0.0), z128(alpha.re - beta, alpha.im));
        }
        // (2) the reflector, explicitly
        z128* v = V + j * n;
        for (int64_t r = tid; r < n; r += QR_NT)
            v[r] = r < j ? z128(0.0, 0.0) : (r == j ? z128(1.0, 0.0) : a[r] * scl);
        __syncthreads();
        // (3) w_c = v^H A[:, j0+c] for the panel's later columns, d_p = V[:, j0+p]^H v for T
        double part[4 * QR_HB];
        const int nw = b - 1 - k, nd = k;
        for (int q = 0; q < 2 * (nw + nd); ++q) part[q] = 0.0;
        for (int64_t r = j + tid; r < n; r += QR_NT) {
            const z128 cv = conj(v[r]);
            for (int c = 0; c < nw; ++c) {
                const z128 p = cv * A[r + (j + 1 + c) * n];
                part[2 * c] += p.re;
                part[2 * c + 1] += p.im;
            }
            for (int q = 0; q < nd; ++q) {
                const z128 p = conj(V[r + (j0 + q) * n]) * v[r];
                part[2 * (nw + q)] += p.re;
                part[2 * (nw + q) + 1] += p.im;
            }
        }
        block_sum(part, 2 * (nw + nd), red, tot);
        // (4) A[:, j0+c] <- A[:, j0+c] - conj(tau) v w_c (rows >= j)
        const z128 ct = conj(tau);
        for (int64_t r = j + tid; r < n; r += QR_NT) {
            const z128 tv = ct * v[r];
            for (int c = 0; c < nw; ++c) cfms(A[r + (j + 1 + c) * n], tv, z128(tot[2 * c], tot[2 * c + 1]));
        }
        // (5) column k of T: T[k,k] = tau, T[0:k,k] = -tau T[0:k,0:k] d
        if (tid == 0) {
            for (int i = 0; i < k; ++i) {
                z128 acc(0.0, 0.0);
                for (int q = i; q < k; ++q)
                    cfma(acc, T[i + q * QR_HB], z128(tot[2 * (nw + q)], tot[2 * (nw + q) + 1]));
                T[i + k * QR_HB] = z128(0.0, 0.0) - tau * acc;
            }
            T[k + k * QR_HB] = tau;
            for (int i = k + 1; i < QR_HB; ++i) T[i + k * QR_HB] = z128(0.0, 0.0);
            a[j] = z128(beta, 0.0);
        }
        __syncthreads();
    }
}

// E = first m columns of the n x n identity (ld n).
__global__ __launch_bounds__(256) void eye_kernel(int64_t n, int64_t m, z128* E) {
    const int64_t total = n * m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, c = e / n;
        E[e] = z128(i == c ? 1.0 : 0.0, 0.0);
    }
}

}  // namespace

int64_t householder_scratch_elems(int64_t m) {
    return ceil_div(m, (int64_t)QR_HB) * QR_HB * QR_HB + 2 * QR_HB * m;
}

void householder_orthonormalize(hipStream_t s, int64_t n, int64_t m, z128* Q, z128* E, z128* V, z128* small,
                                z128* ws, int64_t ws_elems) {
    const int64_t np = ceil_div(m, (int64_t)QR_HB);
    z128* Tall = small;
    z128* W = Tall + np * QR_HB * QR_HB;
    z128* W2 = W + QR_HB * m;
    const z128 one(1.0, 0.0), zero(0.0, 0.0), mone(-1.0, 0.0);
    for (int64_t p = 0; p < np; ++p) {
        const int64_t j0 = p * QR_HB;
        const int b = (int)std::min<int64_t>(QR_HB, m - j0);
        z128* Tp = Tall + p * QR_HB * QR_HB;
        hipLaunchKernelGGL(house_panel_kernel, dim3(1), dim3(QR_NT), 0, s, n, j0, b, Q, V, Tp);
        NLF_HIP(hipGetLastError());
        const int64_t mc = m - j0 - b;
        if (mc > 0) {   // trailing columns <- (I - V T V^H)^H trailing columns
            const z128* Vp = V + j0 + j0 * n;
            z128* C = Q + j0 + (j0 + b) * n;
            gemm<double>(s, true, b, mc, n - j0, one, Vp, n, 0, C, n, 0, zero, W, QR_HB, 0, 1, ws, ws_elems);
            gemm<double>(s, true, b, mc, b, one, Tp, QR_HB, 0, W, QR_HB, 0, zero, W2, QR_HB, 0, 1);
            gemm<double>(s, false, n - j0, mc, b, mone, Vp, n, 0, W2, QR_HB, 0, one, C, n, 0, 1);
        }
    }
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n * m, 256), 8192))),
                       dim3(256), 0, s, n, m, E);
    NLF_HIP(hipGetLastError());
    for (int64_t p = np - 1; p >= 0; --p) {   // E <- (I - V T V^H) E on rows and columns j0..
        const int64_t j0 = p * QR_HB;
        const int b = (int)std::min<int64_t>(QR_HB, m - j0);
        const z128* Tp = Tall + p * QR_HB * QR_HB;
        const z128* Vp = V + j0 + j0 * n;
        z128* Ep = E + j0 + j0 * n;
        const int64_t ec = m - j0;
        gemm<double>(s, true, b, ec, n - j0, one, Vp, n, 0, Ep, n, 0, zero, W, QR_HB, 0, 1, ws, ws_elems);
        gemm<double>(s, false, b, ec, b, one, Tp, QR_HB, 0, W, QR_HB, 0, zero, W2, QR_HB, 0, 1);
        gemm<double>(s, false, n - j0, ec, b, mone, Vp, n, 0, W2, QR_HB, 0, one, Ep, n, 0, 1);
    }
}

}  // namespace nlf
