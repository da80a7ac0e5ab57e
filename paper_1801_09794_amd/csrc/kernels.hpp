// Internal launch interfaces of the HIP kernels (not part of the C ABI).
#pragma once

#include "common.hpp"

#include <functional>

namespace nlf {

struct GemmConfig {
    int tm = 2, tn = 2;   // MFMA tiles per wave in m and n (workgroup tile 32tm x 32tn)
};

// C_b = alpha op(A_b) B_b + beta C_b, op(A) = A^H when conjA.  ws (optional) enables split-K
// for small outputs with long reductions.  force overrides the tile choice.  lu_update launches
// the same tile program under the lu_update_kernel symbol (LU trailing updates; no split-K).
template <typename R>
void gemm(hipStream_t s, bool conjA, int64_t M, int64_t N, int64_t K, Cx<R> alpha,
          const Cx<R>* A, int64_t lda, int64_t sA, const Cx<R>* B, int64_t ldb, int64_t sB,
          Cx<R> beta, Cx<R>* C, int64_t ldc, int64_t sC, int batch, Cx<R>* ws = nullptr,
          int64_t ws_elems = 0, const GemmConfig* force = nullptr, bool lu_update = false);

// LU with partial pivoting (in place), batched over strided matrices.  With dinv and tmp
// (getrf_tmp_elems per matrix) it runs right-looking with 512-column panels and leaves the
// explicit inverses of the diagonal blocks of L and U in dinv (as lu_block_inverses does);
// without them it is the plain column-halving recursion.
int64_t getrf_tmp_elems(int64_t n);
// Width of the panels factored by one workgroup (4..32, default 32); set per calling thread.
int& lu_panel_width();
// Per-thread override of the LU trailing-update GEMM tile ({0, 0} = default choice).
GemmConfig& lu_update_tile();
// A trailing update of the blocked LU handed to a capture hook instead of being launched:
// launch(stream) issues it (the arguments are bound), flops and bytes are its algorithmic work.
struct LuUpdateLaunch {
    std::function<void(hipStream_t)> launch;
    double flops = 0, bytes = 0;
};
// Per-thread hook (null: launch directly).  While a factorisation is captured into a graph,
// the hook receives each trailing update, so the capture can be split around them and the
// updates launched eagerly (and timed) between the graph segments.
std::function<void(LuUpdateLaunch&&)>*& lu_update_hook();
// Look-ahead resources for the blocked LU: a second stream for the panel factorisations and
// two events owned by the caller (all null: one stream).
struct LuAux {
    hipStream_t s = nullptr;
    hipEvent_t panel_done = nullptr, next_ready = nullptr;
};
template <typename R>
void getrf(hipStream_t s, int64_t n, int batch, Cx<R>* A, int64_t lda, int64_t sA,
           int32_t* ipiv, int32_t* perm, int32_t* info, int32_t* scratch,
           Cx<R>* dinv = nullptr, Cx<R>* tmp = nullptr, const LuAux* aux = nullptr);
// Scratch (int32 elements) that getrf needs for its row-exchange lists.
int64_t getrf_scratch_ints(int64_t n, int batch);

// X_b = A_b^{-1} B_b from getrf factors; B may be shared (sB = 0).  X must not alias B.
template <typename R>
void getrs(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
           int64_t sA, const int32_t* perm, const Cx<R>* B, int64_t ldb, int64_t sB, Cx<R>* X,
           int64_t ldx, int64_t sX);

// Explicit inverses of the 256 x 256 diagonal blocks of the L and U factors (once per
// factorisation), and the triangular solves built on them (one batched GEMM per block step).
int64_t lu_inverse_elems(int64_t n);     // per matrix
template <typename R>
void lu_block_inverses(hipStream_t s, int64_t n, int batch, const Cx<R>* LU, int64_t lda,
                       int64_t sA, Cx<R>* dinv);
template <typename R>
void getrs_inv(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
               int64_t sA, const int32_t* perm, const Cx<R>* dinv, const Cx<R>* B, int64_t ldb,
               int64_t sB, Cx<R>* X, int64_t ldx, int64_t sX, Cx<R>* tmp);   // tmp: 256 x nrhs per matrix
// X = A^{-H} B with the same factors (the solves of the adjoint problem): Z is n x nrhs scratch
// per matrix (ld n, stride n * nrhs; may equal B with those strides), X must not overlap Z.
template <typename R>
void getrs_inv_adjoint(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
                       int64_t sA, const int32_t* perm, const Cx<R>* dinv, const Cx<R>* B, int64_t ldb,
                       int64_t sB, Cx<R>* Z, Cx<R>* X, int64_t ldx, int64_t sX, Cx<R>* tmp);

// In-place triangular solves B <- L^{-1} B (unit lower) and B <- U^{-1} B (upper).
template <typename R>
void trsm_lower_unit(hipStream_t s, int64_t n, int64_t N, int batch, const Cx<R>* L,
                     int64_t ldl, int64_t sL, Cx<R>* B, int64_t ldb, int64_t sB);
template <typename R>
void trsm_upper(hipStream_t s, int64_t n, int64_t N, int batch, const Cx<R>* U, int64_t ldu,
                int64_t sU, Cx<R>* B, int64_t ldb, int64_t sB);

// ---- elementwise / reduction kernels (elementwise.hip)

// T_k = sum_j coef[k*J + j] A_j for k < nz; outputs in c128 (T64) and/or c64 (T32).
void assemble(hipStream_t s, int64_t n, int J, const z128* const* A, int64_t lda,
              int nz, const z128* coef_dev, z128* T64, z64* T32, int64_t ldt, int64_t sT);
// column 2-norms of a c128 n x m block (ld) into out (device doubles)
void col_norms(hipStream_t s, int64_t n, int m, const z128* X, int64_t ld, double* out);
// Q = X diag(rho) - sum_k Y_k diag(c_k) with rho (m) and c (nz x m) on the device
void accumulate(hipStream_t s, int64_t n, int m, int nz, const z128* X, const z128* Y,
                int64_t sY, const z128* rho, const z128* c, z128* Q);
// precision casts of an n x m block (ld in, ld out), batched
void cast_128_to_64(hipStream_t s, int64_t rows, int64_t cols, int batch, const z128* in,
                    int64_t ldi, int64_t si, z64* out, int64_t ldo, int64_t so);
void cast_64_to_128(hipStream_t s, int64_t rows, int64_t cols, int batch, const z64* in,
                    int64_t ldi, int64_t si, z128* out, int64_t ldo, int64_t so, bool accumulate);
// sum of squared magnitudes of each of `batch` n x m blocks into out[b] (device doubles);
// part: block_sqnorms_scratch(batch) doubles for the partial sums
int64_t block_sqnorms_scratch(int batch);
void block_sqnorms(hipStream_t s, int64_t rows, int64_t cols, int batch, const z128* X,
                   int64_t ld, int64_t sX, double* out, double* part);
// copy an n x m c128 block (ld in, ld out)
void copy_block(hipStream_t s, int64_t rows, int64_t cols, const z128* in, int64_t ldi,
                z128* out, int64_t ldo);
// p[0..count) = v (a kernel, so that the sequence stays capturable in a HIP graph)
void fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t v);
// flags[j] = 0 when the n x n matrix A[j] (ld lda) is exactly the identity, else 1
void identity_flags(hipStream_t s, int64_t n, int J, const z128* const* A, int64_t lda, int32_t* flags);
// counter-based standard complex normal draws CN(0,1) for an n x m block
void random_normal(hipStream_t s, int64_t rows, int64_t cols, uint64_t seed, z128* out, int64_t ld);

// Householder QR of Q (n x m, ld n, m <= n), for blocks too ill-conditioned for Cholesky QR:
// the first m columns of the orthogonal factor are written to E (n x m, ld n); Q is
// overwritten.  V: n x m scratch (the reflectors); small: householder_scratch_elems(m)
// elements; ws, ws_elems: split-K scratch of the GEMMs (as for the Gram matrix).
constexpr int QR_HB = 8;   // panel width
int64_t householder_scratch_elems(int64_t m);
void householder_orthonormalize(hipStream_t s, int64_t n, int64_t m, z128* Q, z128* E, z128* V, z128* small,
                                z128* ws, int64_t ws_elems);

}  // namespace nlf
