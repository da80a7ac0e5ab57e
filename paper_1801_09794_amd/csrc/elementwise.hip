// HBM-bound kernels of the nonlinear FEAST hot path: assembly of T(z_k) for every node,
// Step 4 accumulation, column norms (Step 3 residuals), precision casts of the refinement,
// and the counter-based initial block.  Grid-stride loops over interleaved complex elements,
// consecutive threads on consecutive rows of column-major blocks (coalesced).
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace nlf {

constexpr int MAXJ = 8;

struct APtrs {
    const z128* p[MAXJ];
};

static inline unsigned grid_for(int64_t total, int64_t cap = 8192) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), cap));
}

// Rows per thread and rows per workgroup of the two-dimensional launches below: workgroup
// (x, y) covers rows [x EW_ROWS, (x + 1) EW_ROWS) of column y; thread t handles rows
// x EW_ROWS + t + 256 r, r < EW_RPT, so each load or store instruction of a wavefront touches
// 64 consecutive elements (1 KB of complex128) and every thread has EW_RPT independent
// accesses in flight per stream.
constexpr int EW_RPT = 4;
constexpr int EW_ROWS = 256 * EW_RPT;

// Streaming accesses: the node matrices are written once here and read again only by the LU,
// long after they have left the caches; the A_j are read once per assembly.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ z128 ld_stream(const z128* p) {
    const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
    return z128(v.x, v.y);
}
__device__ __forceinline__ void st_stream(z128* p, z128 v) {
    const v2d w = {v.re, v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<v2d*>(p));
}
__device__ __forceinline__ void st_stream(z64* p, z128 v) {
    const v2f w = {(float)v.re, (float)v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<v2f*>(p));
}

// T_k(i, c) = sum_j coef[k J + j] A_j(i, c): each A_j element is read once and all nz
// outputs are written from registers (one FP64 sum, rounded once for the complex64 copy).
__global__ __launch_bounds__(256) void assemble_kernel(int64_t n, int J, APtrs A, int64_t lda,
                                                       int nz, const z128* __restrict__ coef,
                                                       z128* T64, z64* T32, int64_t ldt,
                                                       int64_t sT) {
    const int64_t c = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * EW_ROWS + threadIdx.x;
    z128 a[EW_RPT][MAXJ];
#pragma unroll
    for (int r = 0; r < EW_RPT; ++r) {
        const int64_t i = r0 + 256 * r;
#pragma unroll
        for (int j = 0; j < MAXJ; ++j)
            if (j < J && i < n) a[r][j] = ld_stream(A.p[j] + i + c * lda);
    }
    const int64_t off = r0 + c * ldt;
    for (int k = 0; k < nz; ++k) {
        z128 w[MAXJ];
#pragma unroll
        for (int j = 0; j < MAXJ; ++j)
            if (j < J) w[j] = coef[k * J + j];
#pragma unroll
        for (int r = 0; r < EW_RPT; ++r) {
            if (r0 + 256 * r >= n) continue;
            z128 acc(0, 0);
#pragma unroll
            for (int j = 0; j < MAXJ; ++j)
                if (j < J) cfma(acc, w[j], a[r][j]);
            if (T64) st_stream(T64 + k * sT + off + 256 * r, acc);
            if (T32) st_stream(T32 + k * sT + off + 256 * r, acc);
        }
    }
}

void assemble(hipStream_t s, int64_t n, int J, const z128* const* A, int64_t lda, int nz,
              const z128* coef_dev, z128* T64, z64* T32, int64_t ldt, int64_t sT) {
    NLF_REQUIRE(J >= 1 && J <= MAXJ, 1, "assemble: 1 <= J <= 8 terms");
    NLF_REQUIRE(n <= 65535, 1, "assemble: n <= 65535");
    APtrs ap{};
    for (int j = 0; j < J; ++j) ap.p[j] = A[j];
    const double bytes = (double)n * n * (16.0 * J + nz * ((T64 ? 16.0 : 0) + (T32 ? 8.0 : 0)));
    ProfScope ps(NLF_PROF_ASSEMBLE, s, 8.0 * n * n * J * nz, bytes);
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)ceil_div(n, EW_ROWS), (unsigned)n), dim3(256), 0, s, n, J,
                       ap, lda, nz, coef_dev, T64, T32, ldt, sT);
    NLF_HIP(hipGetLastError());
}

// one workgroup per column: sqrt(sum |x|^2)
__global__ __launch_bounds__(256) void col_norms_kernel(int64_t n, const z128* X, int64_t ld,
                                                        double* out) {
    __shared__ double red[4];
    const int64_t c = blockIdx.x;
    double s = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += norm2(X[i + c * ld]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

void col_norms(hipStream_t s, int64_t n, int m, const z128* X, int64_t ld, double* out) {
    if (m <= 0) return;
    hipLaunchKernelGGL(col_norms_kernel, dim3(m), dim3(256), 0, s, n, X, ld, out);
    NLF_HIP(hipGetLastError());
}

// Q = X diag(rho) - sum_k Y_k diag(c_k): column c of Q from column c of X and of every Y_k
// (the coefficients of the column are uniform across the workgroup).  Thread t of workgroup
// (x, c) handles rows x 256 RPT + t + 256 r, r < RPT.  The nodes are taken KU at a time with all
// their loads issued before the multiply-adds, so KU RPT loads per thread are in flight; the
// sum still runs over k in ascending order.  Large blocks take four rows and one node at a time
// (enough workgroups to cover the latency), smaller ones fewer rows per thread and more nodes
// per load batch: more workgroups, and fewer round trips to memory per thread.
template <int RPT, int KU>
__global__ __launch_bounds__(256) void accumulate_kernel(int64_t n, int m, int nz,
                                                         const z128* __restrict__ X,
                                                         const z128* __restrict__ Y, int64_t sY,
                                                         const z128* __restrict__ rho,
                                                         const z128* __restrict__ coef, z128* Q) {
    const int64_t c = blockIdx.y;
    const int64_t e0 = (int64_t)blockIdx.x * (256 * RPT) + threadIdx.x + c * n;
    const int64_t end = (c + 1) * n;
    const z128 rc = rho[c];
    z128 q[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) q[r] = e0 + 256 * r < end ? rc * ld_stream(X + e0 + 256 * r) : z128(0, 0);
    int k = 0;
    for (; k + KU <= nz; k += KU) {
        z128 w[KU], y[KU][RPT];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            w[u] = coef[(int64_t)(k + u) * m + c];
            const z128* Yk = Y + (k + u) * sY;
#pragma unroll
            for (int r = 0; r < RPT; ++r) y[u][r] = e0 + 256 * r < end ? ld_stream(Yk + e0 + 256 * r) : z128(0, 0);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
            for (int r = 0; r < RPT; ++r) cfms(q[r], w[u], y[u][r]);
    }
    for (; k < nz; ++k) {
        const z128 w = coef[(int64_t)k * m + c];
        const z128* Yk = Y + k * sY;
        z128 y[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) y[r] = e0 + 256 * r < end ? ld_stream(Yk + e0 + 256 * r) : z128(0, 0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) cfms(q[r], w, y[r]);
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
        if (e0 + 256 * r < end) Q[e0 + 256 * r] = q[r];
}

void accumulate(hipStream_t s, int64_t n, int m, int nz, const z128* X, const z128* Y,
                int64_t sY, const z128* rho, const z128* c, z128* Q) {
    if (n <= 0 || m <= 0) return;
    ProfScope ps(NLF_PROF_ACCUMULATE, s, 8.0 * n * m * nz, 16.0 * n * m * (nz + 2));
    // measured on MI355X (complex128, 16-24 nodes): four-row threads, one node at a time, are
    // fastest from about 1024 such workgroups (n = 8192, m = 160: 6.7 TB/s); two rows and four
    // nodes from 128 (n = 4096, m = 64: 12.9 us against 17.8); one row and eight nodes below
    // (n = 2048, m = 16: 6.2 us against 12.9)
    const int64_t w4 = ceil_div(n, 1024) * m;
    if (w4 >= 1024)
        hipLaunchKernelGGL((accumulate_kernel<4, 1>), dim3((unsigned)ceil_div(n, 1024), (unsigned)m), dim3(256), 0,
                           s, n, m, nz, X, Y, sY, rho, c, Q);
    else if (w4 >= 128)
        hipLaunchKernelGGL((accumulate_kernel<2, 4>), dim3((unsigned)ceil_div(n, 512), (unsigned)m), dim3(256), 0,
                           s, n, m, nz, X, Y, sY, rho, c, Q);
    else
        hipLaunchKernelGGL((accumulate_kernel<1, 8>), dim3((unsigned)ceil_div(n, 256), (unsigned)m), dim3(256), 0,
                           s, n, m, nz, X, Y, sY, rho, c, Q);
    NLF_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void cast_128_64_kernel(int64_t rows, int64_t cols,
                                                          const z128* in, int64_t ldi, int64_t si,
                                                          z64* out, int64_t ldo, int64_t so) {
    const int64_t b = blockIdx.y, total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % rows, c = e / rows;
        const z128 v = in[b * si + i + c * ldi];
        out[b * so + i + c * ldo] = z64((float)v.re, (float)v.im);
    }
}

__global__ __launch_bounds__(256) void cast_64_128_kernel(int64_t rows, int64_t cols,
                                                          const z64* in, int64_t ldi, int64_t si,
                                                          z128* out, int64_t ldo, int64_t so,
                                                          int acc) {
    const int64_t b = blockIdx.y, total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % rows, c = e / rows;
        const z64 v = in[b * si + i + c * ldi];
        z128* o = out + b * so + i + c * ldo;
        const z128 w((double)v.re, (double)v.im);
        *o = acc ? (*o + w) : w;
    }
}

void cast_128_to_64(hipStream_t s, int64_t rows, int64_t cols, int batch, const z128* in,
                    int64_t ldi, int64_t si, z64* out, int64_t ldo, int64_t so) {
    hipLaunchKernelGGL(cast_128_64_kernel, dim3(grid_for(rows * cols, 2048), batch), dim3(256), 0,
                       s, rows, cols, in, ldi, si, out, ldo, so);
    NLF_HIP(hipGetLastError());
}

void cast_64_to_128(hipStream_t s, int64_t rows, int64_t cols, int batch, const z64* in,
                    int64_t ldi, int64_t si, z128* out, int64_t ldo, int64_t so, bool acc) {
    hipLaunchKernelGGL(cast_64_128_kernel, dim3(grid_for(rows * cols, 2048), batch), dim3(256), 0,
                       s, rows, cols, in, ldi, si, out, ldo, so, acc ? 1 : 0);
    NLF_HIP(hipGetLastError());
}

// ||X_b||_F^2 per block in two deterministic stages: BLOCK_SQ_PARTS workgroups per block each
// sum a strided set of columns, then one wavefront per block adds the partial sums.
constexpr int BLOCK_SQ_PARTS = 64;

__global__ __launch_bounds__(256) void block_sqnorm_part_kernel(int64_t rows, int64_t cols,
                                                                const z128* X, int64_t ld,
                                                                int64_t sX, double* part) {
    __shared__ double red[4];
    const int64_t b = blockIdx.y;
    double s = 0;
    for (int64_t c = blockIdx.x; c < cols; c += BLOCK_SQ_PARTS) {
        const z128* col = X + b * sX + c * ld;
        for (int64_t i = threadIdx.x; i < rows; i += 256) s += norm2(col[i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[b * BLOCK_SQ_PARTS + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(64) void block_sqnorm_sum_kernel(const double* part, double* out) {
    double s = part[blockIdx.x * BLOCK_SQ_PARTS + threadIdx.x];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

int64_t block_sqnorms_scratch(int batch) { return (int64_t)batch * BLOCK_SQ_PARTS; }

void block_sqnorms(hipStream_t s, int64_t rows, int64_t cols, int batch, const z128* X,
                   int64_t ld, int64_t sX, double* out, double* part) {
    static_assert(BLOCK_SQ_PARTS == 64, "one wavefront sums the partials");
    hipLaunchKernelGGL(block_sqnorm_part_kernel, dim3(BLOCK_SQ_PARTS, batch), dim3(256), 0, s, rows, cols,
                       X, ld, sX, part);
    NLF_HIP(hipGetLastError());
    hipLaunchKernelGGL(block_sqnorm_sum_kernel, dim3(batch), dim3(64), 0, s, (const double*)part, out);
    NLF_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void copy_block_kernel(int64_t rows, int64_t cols, const z128* in,
                                                         int64_t ldi, z128* out, int64_t ldo) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % rows, c = e / rows;
        out[i + c * ldo] = in[i + c * ldi];
    }
}

void copy_block(hipStream_t s, int64_t rows, int64_t cols, const z128* in, int64_t ldi, z128* out,
                int64_t ldo) {
    hipLaunchKernelGGL(copy_block_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, rows, cols,
                       in, ldi, out, ldo);
    NLF_HIP(hipGetLastError());
}

// splitmix64 finaliser (Steele, Lea, Flood 2014) as a counter-based generator; two 53-bit
// uniforms per element feed the Box-Muller transform.  CN(0,1) = (N + iN)/sqrt 2.
__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void random_normal_kernel(int64_t rows, int64_t cols,
                                                            uint64_t seed, z128* out, int64_t ld) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const uint64_t h1 = splitmix(seed ^ splitmix(2 * (uint64_t)e));
        const uint64_t h2 = splitmix(seed ^ splitmix(2 * (uint64_t)e + 1));
        const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);   // (0, 1]
        const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);           // [0, 1)
        const double r = sqrt(-2.0 * log(u1)), t = 6.283185307179586 * u2;
        const int64_t i = e % rows, c = e / rows;
        out[i + c * ld] = z128(r * cos(t) * 0.7071067811865476, r * sin(t) * 0.7071067811865476);
    }
}

void random_normal(hipStream_t s, int64_t rows, int64_t cols, uint64_t seed, z128* out, int64_t ld) {
    hipLaunchKernelGGL(random_normal_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, rows,
                       cols, seed, out, ld);
    NLF_HIP(hipGetLastError());
}

// flags[j] = 1 when the n x n matrix A_j (ld lda) differs anywhere from the identity; every
// thread that finds a difference writes the same value, so plain stores suffice (the flags are
// cleared beforehand)
__global__ __launch_bounds__(256) void identity_check_kernel(int64_t n, APtrs A, int64_t lda, int32_t* flags) {
    const int j = blockIdx.y;
    const z128* a = A.p[j];
    const int64_t total = n * n;
    bool diff = false;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, c = e / n;
        const z128 v = a[i + c * lda];
        diff = diff || v.im != 0.0 || v.re != (i == c ? 1.0 : 0.0);
    }
    if (diff) flags[j] = 1;
}

void identity_flags(hipStream_t s, int64_t n, int J, const z128* const* A, int64_t lda, int32_t* flags) {
    NLF_REQUIRE(J >= 1 && J <= MAXJ, 1, "identity_flags: 1 <= J <= 8 terms");
    fill_i32(s, flags, J, 0);
    APtrs ap{};
    for (int j = 0; j < J; ++j) ap.p[j] = A[j];
    hipLaunchKernelGGL(identity_check_kernel, dim3(grid_for(n * n, 2048), J), dim3(256), 0, s, n, ap, lda, flags);
    NLF_HIP(hipGetLastError());
}

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t v) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        p[e] = v;
}

void fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t v) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
    NLF_HIP(hipGetLastError());
}

}  // namespace nlf
