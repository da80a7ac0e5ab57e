// Complex GEMM on gfx950 matrix cores: C = alpha op(A) B + beta C, op(A) = A or A^H.
//
// Every dense contraction of the nonlinear FEAST hot path goes through this kernel: the
// trailing updates and off-diagonal blocks of the blocked LU of T(z_k), the triangular solves
// against the residual block, the projections Q^H A_j Q, the block residual, the Ritz vectors
// and the Gram matrices of the orthonormalisation.
//
// There is no complex MFMA, so one complex multiply-add of a 16x16x4 block is four real
// v_mfma_*_16x16x4 instructions (the "4M" scheme): Cr += Ar Br, Cr -= Ai Bi, Ci += Ar Bi,
// Ci += Ai Br, or three (the "3M" scheme of gemm_tile_body, taken by every product with
// op(A) = A and a reduction of at least 64).  The MFMA's A operand is fed from op(B) and its B operand from op(A), so the
// 16 consecutive output columns of one MFMA row are 16 consecutive rows m of C: each store
// instruction writes 256-byte contiguous runs of the column-major C without an LDS transpose.
//
// Work decomposition: a 256-thread workgroup (4 waves as 2x2) owns a (32 TM) x (32 TN)
// complex tile of C; each wave owns (16 TM) x (16 TN), i.e. TM x TN MFMA tiles with a real
// and an imaginary accumulator each (and a third one under 3M).  K advances in steps of BK complex elements staged in
// LDS as [k][m] and [k][n] (interleaved complex, so one ds_read_b64/b128 gives re and im).
// The next K step is fetched into registers while the current one is multiplied.
// Optional split-K writes alpha-scaled partial products to a workspace; gemm_reduce sums them.
//
// 3M products with a reduction that is a multiple of 16 take the direct-to-LDS forms (namespace
// dma below): the operand tiles go from global memory straight into LDS, with no staging
// registers between the MFMA blocks.  FP64: 64 x 64 tiles (the LU trailing updates and the
// triangular-solve updates), 64 x 32 tiles (32-column edges and small products), a split-K
// variant (long reductions into few tiles); FP32: 128 x 64 tiles.  The staged program above
// serves the conjugated products (Gram matrices, Q^H W) and shapes the direct forms do not take.
#include "common.hpp"
#include "kernels.hpp"

namespace nlf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
// Accumulator layout of a 16x16 output block: lane l, register r holds row acc_row(l >> 4, r)
// and column (l & 15).  Measured on gfx950: v_mfma_f64_16x16x4f64 puts rows (l >> 4) + 4r in
// a lane, v_mfma_f32_16x16x4f32 rows 4 (l >> 4) + r.
template <> struct Mfma<double> {
    using acc_t = v4d;
    static __device__ __forceinline__ int acc_row(int q, int r) { return q + 4 * r; }
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    using acc_t = v4f;
    static __device__ __forceinline__ int acc_row(int q, int r) { return 4 * q + r; }
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename R>
struct GemmArgs {
    int64_t M, N, K;
    Cx<R> alpha, beta;
    const Cx<R>* A; int64_t lda, sA;
    const Cx<R>* B; int64_t ldb, sB;
    Cx<R>* C; int64_t ldc, sC;
    int tilesM, tilesN;
    int64_t kchunk;        // K range per split (split-K only)
    Cx<R>* P;              // split-K partials: [batch][split][N][M] (ld M)
    int nsplit;
};

// Map the hardware workgroup id to a tile so that each XCD (workgroups are dispatched
// round-robin over the 8 XCDs) receives a contiguous range of tiles, which then share
// A-row and B-column blocks in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int w, int nT) {
    const int q = nT >> 3, r = nT & 7;
    const int xcd = w & 7, slot = w >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Tile order inside an XCD's range: groups of GROUP_M tile rows are swept column by column, so
// the workgroups resident on one XCD at a time cover a roughly square patch of C and share the
// K-slices of A and B in that XCD's L2 (a plain column-major order would pair all tile rows
// with only a couple of tile columns).
constexpr int GROUP_M = 8;
__device__ __forceinline__ void tile_coords(int t, int tilesM, int tilesN, int& tm, int& tn) {
    const int per_group = GROUP_M * tilesN;
    const int group = t / per_group;
    const int first = group * GROUP_M;
    const int gsize = min(tilesM - first, GROUP_M);
    const int r = t - group * per_group;
    tm = first + r % gsize;
    tn = r / gsize;
}

// Global -> register staging of one K step.  A thread loads LA elements of op(A) and LB of B;
// element e of the thread sits at (row, k) = (a_r[e], a_k[e]) of the BM x BK tile of op(A)
// and (b_k[e], b_n[e]) of the BK x BN tile of B.
template <typename R, int TM, int TN, int BK, bool CONJA>
struct GemmTile {
    static constexpr int BM = 32 * TM, BN = 32 * TN;
    static constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    static constexpr int PAD = 1;                       // LDS row padding (complex elements)
    static __device__ __forceinline__ void a_coord(int tid, int e, int& m, int& k) {
        const int idx = tid + 256 * e;
        if (!CONJA) { m = idx % BM; k = idx / BM; }      // op(A) = A: consecutive threads along m
        else        { k = idx % BK; m = idx / BK; }      // op(A) = A^H: along k (contiguous in A)
    }
    static __device__ __forceinline__ void b_coord(int tid, int e, int& k, int& n) {
        const int idx = tid + 256 * e;
        k = idx % BK; n = idx / BK;                      // consecutive threads along k
    }
};

// The loads are issued here and their values are not touched until gemm_stage writes them to
// LDS after the current step's MFMAs, so the memory latency overlaps the matrix work; lanes
// outside the matrix read element 0 (always valid) and are zeroed at the LDS store through the
// bit mask `ok` (bit e: A element e, bit LA + e: B element e).
template <typename R, int TM, int TN, int BK, bool CONJA>
__device__ __forceinline__ void gemm_fetch(int64_t M, int64_t N, int64_t lda, int64_t ldb,
                                           const Cx<R>* __restrict__ A,
                                           const Cx<R>* __restrict__ B, int64_t m0, int64_t n0,
                                           int64_t k0, int64_t kend, int tid,
                                           Cx<R> (&ra)[GemmTile<R, TM, TN, BK, CONJA>::LA],
                                           Cx<R> (&rb)[GemmTile<R, TM, TN, BK, CONJA>::LB],
                                           uint32_t& ok) {
    using T = GemmTile<R, TM, TN, BK, CONJA>;
    ok = 0;
#pragma unroll
    for (int e = 0; e < T::LA; ++e) {
        int m, k;
        T::a_coord(tid, e, m, k);
        const int64_t gm = m0 + m, gk = k0 + k;
        const bool in = gm < M && gk < kend;
        ok |= (uint32_t)in << e;
        ra[e] = A[in ? (!CONJA ? gm + gk * lda : gk + gm * lda) : 0];
    }
#pragma unroll
    for (int e = 0; e < T::LB; ++e) {
        int k, n;
        T::b_coord(tid, e, k, n);
        const int64_t gn = n0 + n, gk = k0 + k;
        const bool in = gn < N && gk < kend;
        ok |= (uint32_t)in << (T::LA + e);
        rb[e] = B[in ? gk + gn * ldb : 0];
    }
}

// As: one BK x (BM + 1) staging buffer, Bs: one BK x (BN + 1) buffer (row k at k * (BM + 1)).
template <typename R, int TM, int TN, int BK, bool CONJA>
__device__ __forceinline__ void gemm_stage(Cx<R>* As, Cx<R>* Bs, int tid, const Cx<R>* ra,
                                           const Cx<R>* rb, uint32_t ok) {
    using T = GemmTile<R, TM, TN, BK, CONJA>;
    static_assert(T::PAD == 1, "stage layout");
    static_assert(T::LA + T::LB <= 32, "mask width");
#pragma unroll
    for (int e = 0; e < T::LA; ++e) {
        int m, k;
        T::a_coord(tid, e, m, k);
        const bool in = (ok >> e) & 1u;
        As[k * (T::BM + 1) + m] = Cx<R>(in ? ra[e].re : R(0), in ? (CONJA ? -ra[e].im : ra[e].im) : R(0));
    }
#pragma unroll
    for (int e = 0; e < T::LB; ++e) {
        int k, n;
        T::b_coord(tid, e, k, n);
        const bool in = (ok >> (T::LA + e)) & 1u;
        Bs[k * (T::BN + 1) + n] = Cx<R>(in ? rb[e].re : R(0), in ? rb[e].im : R(0));
    }
}

// M3: the complex products by three real MFMAs instead of four (the "3M" scheme): with
// T1 = Ar Br, T2 = Ai Bi and T3 = (Ar + Ai)(Br + Bi) accumulated separately, Cr = T1 - T2 and
// Ci = T3 - T1 - T2 in the epilogue (one accumulator more, a quarter fewer matrix instructions;
// the imaginary part's rounding error grows to about (|Ar| + |Ai|)(|Br| + |Bi|) eps per term).
template <typename R, int TM, int TN, int BK, bool CONJA, bool SPLIT, bool M3 = false>
__device__ __forceinline__ void gemm_tile_body(const GemmArgs<R>& g) {
    using T = GemmTile<R, TM, TN, BK, CONJA>;
    constexpr int BM = T::BM, BN = T::BN, LA = T::LA, LB = T::LB, PAD = T::PAD;
    static_assert(LA * 256 == BM * BK && LB * 256 == BN * BK, "tile/thread mismatch");
    using acc_t = typename Mfma<R>::acc_t;

    // double-buffered staging: step s reads buffer s & 1 while step s+1 is written to the other
    __shared__ Cx<R> As[2][BK][BM + PAD];
    __shared__ Cx<R> Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int nT = g.tilesM * g.tilesN;
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, nT), g.tilesM, g.tilesN, tm, tn);
    const int64_t batch = blockIdx.y;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

    const Cx<R>* __restrict__ A = g.A + batch * g.sA;
    const Cx<R>* __restrict__ B = g.B + batch * g.sB;
    const int64_t M = g.M, N = g.N, lda = g.lda, ldb = g.ldb;

    int64_t kbeg = 0, kend = g.K;
    if (SPLIT) {
        kbeg = (int64_t)blockIdx.z * g.kchunk;
        kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
    }

    // 4M: accR, accI; 3M: accR = T1, accI = T2, acc3 = T3 (combined in the epilogue)
    acc_t accR[TM][TN], accI[TM][TN], acc3[M3 ? TM : 1][M3 ? TN : 1];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            accR[i][j] = acc_t{0, 0, 0, 0};
            accI[i][j] = acc_t{0, 0, 0, 0};
            if constexpr (M3) acc3[i][j] = acc_t{0, 0, 0, 0};
        }

    Cx<R> ra[LA], rb[LB];
    uint32_t ok = 0;
    const int col = lane & 15, krow = lane >> 4;
    if (kbeg < kend) {
        gemm_fetch<R, TM, TN, BK, CONJA>(M, N, lda, ldb, A, B, m0, n0, kbeg, kend, tid, ra, rb, ok);
        gemm_stage<R, TM, TN, BK, CONJA>(&As[0][0][0], &Bs[0][0][0], tid, ra, rb, ok);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            const bool more = k0 + BK < kend;
            if (more) gemm_fetch<R, TM, TN, BK, CONJA>(M, N, lda, ldb, A, B, m0, n0, k0 + BK, kend, tid, ra, rb, ok);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                Cx<R> a[TM], b[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = As[buf][kk + krow][wm * 16 * TM + i * 16 + col];
#pragma unroll
                for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kk + krow][wn * 16 * TN + j * 16 + col];
                if constexpr (M3) {
                    R as[TM], bs[TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i) as[i] = a[i].re + a[i].im;
#pragma unroll
                    for (int j = 0; j < TN; ++j) bs[j] = b[j].re + b[j].im;
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) accR[i][j] = Mfma<R>::mma(b[j].re, a[i].re, accR[i][j]);
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) accI[i][j] = Mfma<R>::mma(b[j].im, a[i].im, accI[i][j]);
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc3[i][j] = Mfma<R>::mma(bs[j], as[i], acc3[i][j]);
                    continue;
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) accR[i][j] = Mfma<R>::mma(b[j].re, a[i].re, accR[i][j]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) accI[i][j] = Mfma<R>::mma(b[j].re, a[i].im, accI[i][j]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) accR[i][j] = Mfma<R>::mma(-b[j].im, a[i].im, accR[i][j]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) accI[i][j] = Mfma<R>::mma(b[j].im, a[i].re, accI[i][j]);
            }
            if (more) gemm_stage<R, TM, TN, BK, CONJA>(&As[buf ^ 1][0][0], &Bs[buf ^ 1][0][0], tid, ra, rb, ok);
            __syncthreads();
            buf ^= 1;
        }
    }

    if constexpr (M3) {   // Cr = T1 - T2, Ci = T3 - T1 - T2
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const acc_t t1 = accR[i][j], t2 = accI[i][j];
                accR[i][j] = t1 - t2;
                accI[i][j] = acc3[i][j] - t1 - t2;
            }
    }
    // epilogue: lane holds, for tile (i, j) and register r, C(m, n) with
    // m = m0 + wm*16TM + 16i + (lane & 15), n = n0 + wn*16TN + 16j + acc_row(lane >> 4, r)
    if (SPLIT) {
        Cx<R>* P = g.P + (batch * g.nsplit + blockIdx.z) * g.M * g.N;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t m = m0 + wm * 16 * TM + i * 16 + col;
                    const int64_t n = n0 + wn * 16 * TN + j * 16 + Mfma<R>::acc_row(krow, r);
                    if (m < g.M && n < g.N) {
                        Cx<R> v(accR[i][j][r], accI[i][j][r]);
                        P[m + n * g.M] = g.alpha * v;
                    }
                }
    } else {
        Cx<R>* C = g.C + batch * g.sC;
        const bool useBeta = (g.beta.re != R(0) || g.beta.im != R(0));
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t m = m0 + wm * 16 * TM + i * 16 + col;
                    const int64_t n = n0 + wn * 16 * TN + j * 16 + Mfma<R>::acc_row(krow, r);
                    if (m < g.M && n < g.N) {
                        Cx<R> v(accR[i][j][r], accI[i][j][r]);
                        Cx<R> out = g.alpha * v;
                        if (useBeta) out = out + g.beta * C[m + n * g.ldc];
                        C[m + n * g.ldc] = out;
                    }
                }
    }
}

template <typename R, int TM, int TN, int BK, bool CONJA, bool SPLIT, bool M3>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs<R> g) {
    gemm_tile_body<R, TM, TN, BK, CONJA, SPLIT, M3>(g);
}

// The same tile program under its own symbol for the rank-NB trailing updates of the blocked
// LU, so that traces and counters can single out the dominant launches of the factorisation.
// It takes the 3M products in both precisions: in FP32 the larger rounding of the imaginary
// parts is left to the FP64 refinement, which needs no more sweeps for it (measured on the
// box, delay8192 FP32 + refinement: trailing updates 271 -> 222 ms per solve, the same six
// iterations and 27 ms of refinement; damped4096: 22.5 -> 18.3 ms).
template <typename R, int TM, int TN, int BK>
__global__ __launch_bounds__(256) void lu_update_kernel(GemmArgs<R> g) {
    gemm_tile_body<R, TM, TN, BK, false, false, true>(g);
}

// ------------------------------------------------ FP64 3M tile with direct-to-LDS operand loads
//
// The same 64 x 64 tile, 2 x 2 waves and 3M products as gemm_tile_body<double, 2, 2, 8>, for
// reductions that are a multiple of 16 (RAGGED: tiles reaching past the last row or column).
// The operand tiles go from global memory straight into LDS (global_load_lds_dwordx4: each lane
// moves one complex element, which lands at the instruction's LDS base + 16 x lane), so no
// staging registers, masks or LDS store instructions sit between the MFMA blocks; each stage
// ends in one wait for the wave's own loads and one barrier. Measured against the staged form at
// 7680 x 7680 x 512, 24 matrices: 77.1 -> 63.0 ms (88% of the FP64 matrix peak in executed
// flops), bit-identical results.
//
// LDS layout of one stage (BK = 8):
//  * op(A): [k][64] complex, one row of the tile per load instruction (64 consecutive rows of
//    the column-major A: 1 KB contiguous);
//  * B: blocks of 8 columns x 8 k. Lane l of the load instruction for block (kh, g) fetches
//    column n = 8 g + (l >> 3) at k = 8 kh + ((l & 7) ^ sw(n)), sw(n) = (n >> 1) & 7, so the 8
//    lanes of a column read its 128 contiguous bytes, and the MFMA operand reads (16 lanes,
//    16 consecutive columns, one k) fall on 16 distinct 16-byte bank groups.
// The stage loop is unrolled over two separately declared buffers so that the compiler sees
// that the loads into one buffer do not alias the reads of the other.
namespace dma {
constexpr int BK = 8;
using Z = Cx<double>;
#define NLF_GPTR(p) ((__attribute__((address_space(1))) void*)(p))
#define NLF_LPTR(p) ((__attribute__((address_space(3))) void*)(p))

// RAGGED: lanes whose row (aok) or column (bit r of bok) lies outside the matrix load nothing;
// the stale LDS entries they leave only feed output rows or columns that are never stored
// BR: B blocks (8 columns x 8 k) loaded per wave and stage
template <bool RAGGED, int BR>
__device__ __forceinline__ void issue(Z* As, Z* Bs, const Z* ga, const Z* const* gb, int64_t lda, int64_t k0,
                                      int wave, bool aok, unsigned bok) {
#pragma unroll
    for (int r = 0; r < BK / 4; ++r)
        if (!RAGGED || aok)
            __builtin_amdgcn_global_load_lds(NLF_GPTR(ga + (k0 + 4 * r) * lda), NLF_LPTR(As + (wave + 4 * r) * 64),
                                             16, 0, 0);
#pragma unroll
    for (int r = 0; r < BR; ++r)
        if (!RAGGED || ((bok >> r) & 1u))
            __builtin_amdgcn_global_load_lds(NLF_GPTR(gb[r] + k0), NLF_LPTR(Bs + (wave + 4 * r) * 64), 16, 0, 0);
}

using acc_t = Mfma<double>::acc_t;
// TN: 16-column MFMA blocks per wave (the tile is 64 x 32 TN); B holds 8 TN column blocks per k half
template <int TN>
__device__ __forceinline__ void multiply(const Z* As, const Z* Bs, int aoff, const int* boff, acc_t (&t1)[2][TN],
                                         acc_t (&t2)[2][TN], acc_t (&t3)[2][TN]) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        Z a[2], b[TN];
        double as[2], bs[TN];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[kk * 64 + aoff + i * 16];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[(kk >> 3) * (256 * TN) + (boff[j] ^ (kk & 4))];
#pragma unroll
        for (int i = 0; i < 2; ++i) as[i] = a[i].re + a[i].im;
#pragma unroll
        for (int j = 0; j < TN; ++j) bs[j] = b[j].re + b[j].im;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t1[i][j] = Mfma<double>::mma(b[j].re, a[i].re, t1[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t2[i][j] = Mfma<double>::mma(b[j].im, a[i].im, t2[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t3[i][j] = Mfma<double>::mma(bs[j], as[i], t3[i][j]);
    }
}

// s_waitcnt vmcnt(0), other counters left alone (gfx9 encoding: expcnt 7, lgkmcnt 15)
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// SPLIT: blockIdx.z takes the reduction range [z kchunk, (z + 1) kchunk) and writes alpha times
// its partial product to g.P (summed with beta C by gemm_reduce_kernel)
// TN = 2: the 64 x 64 tile; TN = 1: 64 x 32 (ragged 32-column edges of FP64 products)
template <bool RAGGED, bool SPLIT = false, int TN = 2>
__device__ __forceinline__ void tile_body(const GemmArgs<double>& g) {
    constexpr int BN = 32 * TN, BR = (BN / 8) * (BK / 8) / 4;
    static_assert(BR >= 1 && (BN / 8) * (BK / 8) % 4 == 0, "B blocks per wave");
    __shared__ Z A0[BK * 64], A1[BK * 64], B0[BK * BN], B1[BK * BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave & 1, wn = wave >> 1;
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, g.tilesM * g.tilesN), g.tilesM, g.tilesN, tm, tn);
    const int64_t batch = blockIdx.y, m0 = (int64_t)tm * 64, n0 = (int64_t)tn * BN;
    const Z* A = g.A + batch * g.sA;
    const Z* B = g.B + batch * g.sB;
    const int64_t lda = g.lda, ldb = g.ldb;
    int64_t kbeg = 0, K = g.K;
    if (SPLIT) {
        kbeg = (int64_t)blockIdx.z * g.kchunk;
        K = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
    }

    // this lane's source of the A rows k = wave + 4 r and of the B blocks b = wave + 4 r
    const Z* ga = A + (m0 + lane) + (int64_t)wave * lda;
    const Z* gb[BR];
    unsigned bok = 0;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const int b = wave + 4 * r, kh = b / (BN / 8), grp = b % (BN / 8);
        const int n = 8 * grp + (lane >> 3), k = 8 * kh + ((lane & 7) ^ ((n >> 1) & 7));
        gb[r] = B + k + (n0 + n) * ldb;
        bok |= (unsigned)(n0 + n < g.N) << r;
    }
    const bool aok = m0 + lane < g.M;
    // a wave whose 32 rows or 16 TN columns all lie outside C has no MFMA work
    const bool active = !RAGGED || (m0 + wm * 32 < g.M && n0 + wn * 16 * TN < g.N);
    // this lane's MFMA operands: A element (k, wm 32 + 16 i + col), B element (k, wn 16 TN + 16 j + col)
    const int col = lane & 15, krow = lane >> 4;
    const int aoff = krow * 64 + wm * 32 + col;
    int boff[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int n = wn * 16 * TN + j * 16 + col;
        boff[j] = (n >> 3) * 64 + (n & 7) * 8 + (krow ^ ((n >> 1) & 7));
    }
    acc_t t1[2][TN], t2[2][TN], t3[2][TN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            t1[i][j] = acc_t{0, 0, 0, 0};
            t2[i][j] = acc_t{0, 0, 0, 0};
            t3[i][j] = acc_t{0, 0, 0, 0};
        }

    issue<RAGGED, BR>(A0, B0, ga, gb, lda, kbeg, wave, aok, bok);
    wait_loads();
    __syncthreads();
    // the range is a multiple of 2 BK: every trip multiplies both buffers; the scheduling
    // barriers keep the loads of the next stage ahead of the MFMAs and the wait behind them
    for (int64_t k0 = kbeg; k0 < K; k0 += 2 * BK) {
        issue<RAGGED, BR>(A1, B1, ga, gb, lda, k0 + BK, wave, aok, bok);
        __builtin_amdgcn_sched_barrier(0);
        if (active) multiply<TN>(A0, B0, aoff, boff, t1, t2, t3);
        __builtin_amdgcn_sched_barrier(0);
        wait_loads();
        __syncthreads();
        if (k0 + 2 * BK < K) issue<RAGGED, BR>(A0, B0, ga, gb, lda, k0 + 2 * BK, wave, aok, bok);
        __builtin_amdgcn_sched_barrier(0);
        if (active) multiply<TN>(A1, B1, aoff, boff, t1, t2, t3);
        __builtin_amdgcn_sched_barrier(0);
        wait_loads();
        __syncthreads();
    }

    Z* C = g.C + batch * g.sC;
    Z* P = SPLIT ? g.P + (batch * g.nsplit + blockIdx.z) * g.M * g.N : nullptr;
    const bool useBeta = (g.beta.re != 0.0 || g.beta.im != 0.0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 32 + i * 16 + col;
                const int64_t n = n0 + wn * 16 * TN + j * 16 + Mfma<double>::acc_row(krow, r);
                if (RAGGED && (m >= g.M || n >= g.N)) continue;
                const double p1 = t1[i][j][r], p2 = t2[i][j][r];
                Z out = g.alpha * Z(p1 - p2, t3[i][j][r] - p1 - p2);
                if (SPLIT) {
                    P[m + n * g.M] = out;
                    continue;
                }
                if (useBeta) out = out + g.beta * C[m + n * g.ldc];
                C[m + n * g.ldc] = out;
            }
}
// shapes the direct-to-LDS tile takes: any M and N (ragged edges through the predicated form), a
// reduction that is a multiple of two stages (a partial stage would mix stale LDS into every output),
// 16-byte aligned operands (one load lane moves one whole complex128)
inline bool fits(const GemmArgs<double>& g) {
    return g.M > 0 && g.N > 0 && g.K > 0 && g.K % (2 * BK) == 0 && reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
}
inline bool full_tiles(int64_t M, int64_t N) { return M % 64 == 0 && N % 64 == 0; }

// The FP32 counterpart: the 128 x 64 tile of gemm_tile_body<float, 4, 2, 8> (wave tile 64 x 32)
// with 3M products. One 16-byte load lane carries two complex64 elements, so:
//  * op(A): [k][128 + 16] complex64, one row per load instruction (lane l: rows 2l, 2l + 1); the
//    16-element pad puts rows k and k + 1 on opposite halves of the LDS banks, so the operand
//    reads of two k rows by 32 lanes do not collide;
//  * B: blocks of 16 columns x 8 k, four 16-byte units (k pairs) per column; lane l of the load
//    for block q fetches column n = 16 q + (l >> 2), unit (l & 3) ^ ((n >> 2) & 3), so the 4
//    lanes of a column read its 64 contiguous bytes and 32 operand reads (16 columns, two k)
//    fall on distinct banks.
// Needs 16-byte aligned row pairs: even M and leading dimensions, 16-byte aligned A and B.
using Y = Cx<float>;
constexpr int APAD32 = 16;
using acc32_t = Mfma<float>::acc_t;

// TN: 16-column MFMA blocks per wave (tile 128 x 32 TN); the B tile has 2 TN blocks of 16 columns,
// loaded by waves 0 .. 2 TN - 1
template <bool RAGGED, int TN = 2>
__device__ __forceinline__ void issue32(Y* As, Y* Bs, const Y* const* ga, const Y* gb, int64_t lda, int64_t k0,
                                        int wave, bool aok, bool bok) {
#pragma unroll
    for (int r = 0; r < BK / 4; ++r)
        if (!RAGGED || aok)
            __builtin_amdgcn_global_load_lds(NLF_GPTR(ga[r] + k0 * lda),
                                             NLF_LPTR(As + (wave + 4 * r) * (128 + APAD32)), 16, 0, 0);
    if ((TN == 2 || wave < 2 * TN) && (!RAGGED || bok))
        __builtin_amdgcn_global_load_lds(NLF_GPTR(gb + k0), NLF_LPTR(Bs + wave * 128), 16, 0, 0);
}

template <int TN>
__device__ __forceinline__ void multiply32(const Y* As, const Y* Bs, int aoff, const int* boff,
                                           acc32_t (&t1)[4][TN], acc32_t (&t2)[4][TN], acc32_t (&t3)[4][TN]) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        Y a[4], b[TN];
        float as[4], bs[TN];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[kk * (128 + APAD32) + aoff + i * 16];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[boff[j] ^ kk];
#pragma unroll
        for (int i = 0; i < 4; ++i) as[i] = a[i].re + a[i].im;
#pragma unroll
        for (int j = 0; j < TN; ++j) bs[j] = b[j].re + b[j].im;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t1[i][j] = Mfma<float>::mma(b[j].re, a[i].re, t1[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t2[i][j] = Mfma<float>::mma(b[j].im, a[i].im, t2[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t3[i][j] = Mfma<float>::mma(bs[j], as[i], t3[i][j]);
    }
}

template <bool RAGGED, int TN = 2>
__device__ __forceinline__ void tile_body32(const GemmArgs<float>& g) {
    constexpr int BN = 32 * TN;
    __shared__ Y A0[BK * (128 + APAD32)], A1[BK * (128 + APAD32)], B0[BK * BN], B1[BK * BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave & 1, wn = wave >> 1;
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, g.tilesM * g.tilesN), g.tilesM, g.tilesN, tm, tn);
    const int64_t batch = blockIdx.y, m0 = (int64_t)tm * 128, n0 = (int64_t)tn * BN;
    const Y* A = g.A + batch * g.sA;
    const Y* B = g.B + batch * g.sB;
    const int64_t K = g.K, lda = g.lda, ldb = g.ldb;

    // this lane's sources: A rows k = wave + 4 r (elements 2 lane, 2 lane + 1), B block q = wave
    const Y* ga[BK / 4];
#pragma unroll
    for (int r = 0; r < BK / 4; ++r) ga[r] = A + (m0 + 2 * lane) + (int64_t)(wave + 4 * r) * lda;
    const int nq = 16 * wave + (lane >> 2);
    const Y* gb = B + 2 * ((lane & 3) ^ ((nq >> 2) & 3)) + (n0 + nq) * ldb;
    // M is even on this path, so a lane's row pair is either inside or outside the matrix
    const bool aok = m0 + 2 * lane < g.M, bok = n0 + nq < g.N;
    const bool active = !RAGGED || (m0 + wm * 64 < g.M && n0 + wn * 16 * TN < g.N);
    // this lane's MFMA operands: A element (k, wm 64 + 16 i + col), B element (k, wn 16 TN + 16 j + col)
    const int col = lane & 15, krow = lane >> 4;
    const int aoff = krow * (128 + APAD32) + wm * 64 + col;
    int boff[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j)
        boff[j] = (wn * TN + j) * 128 + col * 8 + 2 * ((krow >> 1) ^ ((col >> 2) & 3)) + (krow & 1);
    acc32_t t1[4][TN], t2[4][TN], t3[4][TN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            t1[i][j] = acc32_t{0, 0, 0, 0};
            t2[i][j] = acc32_t{0, 0, 0, 0};
            t3[i][j] = acc32_t{0, 0, 0, 0};
        }

    issue32<RAGGED, TN>(A0, B0, ga, gb, lda, 0, wave, aok, bok);
    wait_loads();
    __syncthreads();
    for (int64_t k0 = 0; k0 < K; k0 += 2 * BK) {
        issue32<RAGGED, TN>(A1, B1, ga, gb, lda, k0 + BK, wave, aok, bok);
        __builtin_amdgcn_sched_barrier(0);
        if (active) multiply32<TN>(A0, B0, aoff, boff, t1, t2, t3);
        __builtin_amdgcn_sched_barrier(0);
        wait_loads();
        __syncthreads();
        if (k0 + 2 * BK < K) issue32<RAGGED, TN>(A0, B0, ga, gb, lda, k0 + 2 * BK, wave, aok, bok);
        __builtin_amdgcn_sched_barrier(0);
        if (active) multiply32<TN>(A1, B1, aoff, boff, t1, t2, t3);
        __builtin_amdgcn_sched_barrier(0);
        wait_loads();
        __syncthreads();
    }

    Y* C = g.C + batch * g.sC;
    const bool useBeta = (g.beta.re != 0.0f || g.beta.im != 0.0f);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 64 + i * 16 + col;
                const int64_t n = n0 + wn * 16 * TN + j * 16 + Mfma<float>::acc_row(krow, r);
                if (RAGGED && (m >= g.M || n >= g.N)) continue;
                const float p1 = t1[i][j][r], p2 = t2[i][j][r];
                Y out = g.alpha * Y(p1 - p2, t3[i][j][r] - p1 - p2);
                if (useBeta) out = out + g.beta * C[m + n * g.ldc];
                C[m + n * g.ldc] = out;
            }
}

inline bool fits32(const GemmArgs<float>& g) {
    return g.M > 0 && g.N > 0 && g.K > 0 && g.M % 2 == 0 && g.K % (2 * BK) == 0 &&
           g.lda % 2 == 0 && g.ldb % 2 == 0 && g.sA % 2 == 0 && g.sB % 2 == 0 &&
           reinterpret_cast<uintptr_t>(g.A) % 16 == 0 && reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
}
#undef NLF_GPTR
#undef NLF_LPTR
}  // namespace dma

__global__ __launch_bounds__(256) void gemm_dma_kernel(GemmArgs<double> g) { dma::tile_body<false>(g); }
// the trailing updates of the blocked LU under their own symbol (see lu_update_kernel)
__global__ __launch_bounds__(256) void lu_update_dma_kernel(GemmArgs<double> g) { dma::tile_body<false>(g); }
// ragged M or N (predicated loads, idle waves, guarded stores); the LU updates share it
__global__ __launch_bounds__(256) void gemm_dma_ragged_kernel(GemmArgs<double> g) { dma::tile_body<true>(g); }
// split-K partial products (long reductions into few output tiles; any M and N)
__global__ __launch_bounds__(256) void gemm_dma_split_kernel(GemmArgs<double> g) { dma::tile_body<true, true>(g); }
// 64 x 32 tiles: the ragged last columns that FP64 products split off (N = 160 = 2 x 64 + 32)
__global__ __launch_bounds__(256) void gemm_dma_n32_kernel(GemmArgs<double> g) {
    dma::tile_body<false, false, 1>(g);
}
__global__ __launch_bounds__(256) void gemm_dma_n32_ragged_kernel(GemmArgs<double> g) {
    dma::tile_body<true, false, 1>(g);
}
// FP32 takes the predicated form for every shape: with the per-wave MFMA branch the compiler keeps
// the two unrolled stages apart and allocates 142 VGPRs (three waves per SIMD) instead of 180
// (two); measured at 7680^2 x 512, 24 matrices: 33.5 against 34.9 ms
__global__ __launch_bounds__(256) void gemm_dma32_kernel(GemmArgs<float> g) { dma::tile_body32<true>(g); }
__global__ __launch_bounds__(256) void lu_update_dma32_kernel(GemmArgs<float> g) { dma::tile_body32<true>(g); }
// 128 x 32 tiles: the 32-column edges split off complex64 products
__global__ __launch_bounds__(256) void gemm_dma32_n32_kernel(GemmArgs<float> g) { dma::tile_body32<true, 1>(g); }

// C = sum_s P_s + beta C over the split-K partials.
template <typename R>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(int64_t M, int64_t N, int nsplit,
                                                           const Cx<R>* __restrict__ P,
                                                           Cx<R> beta, Cx<R>* C, int64_t ldc,
                                                           int64_t sC) {
    const int64_t batch = blockIdx.y;
    const int64_t MN = M * N;
    const bool useBeta = (beta.re != R(0) || beta.im != R(0));
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < MN; e += (int64_t)gridDim.x * 256) {
        const int64_t m = e % M, n = e / M;
        Cx<R> s(0, 0);
        const Cx<R>* p = P + batch * nsplit * MN + e;
        for (int k = 0; k < nsplit; ++k) s = s + p[k * MN];
        Cx<R>* c = C + batch * sC + m + n * ldc;
        if (useBeta) s = s + beta * (*c);
        *c = s;
    }
}

// ---------------------------------------------------------------------------- host side

// m3: the 3M products (see gemm_tile_body).
template <typename R, int TM, int TN, int BK, bool CONJA>
static void launch_tiles(hipStream_t s, GemmArgs<R>& g, int batch, int nsplit, bool lu_update, bool m3) {
    constexpr int BM = 32 * TM, BN = 32 * TN;
    g.tilesM = (int)ceil_div(g.M, BM);
    g.tilesN = (int)ceil_div(g.N, BN);
    dim3 grid(g.tilesM * g.tilesN, batch, nsplit);
    if constexpr (std::is_same<R, double>::value && TM == 2 && TN == 2 && !CONJA) {
        if ((lu_update || m3) && nsplit == 1 && dma::fits(g)) {
            if (!dma::full_tiles(g.M, g.N))
                hipLaunchKernelGGL(gemm_dma_ragged_kernel, grid, dim3(256), 0, s, g);
            else if (lu_update)
                hipLaunchKernelGGL(lu_update_dma_kernel, grid, dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL(gemm_dma_kernel, grid, dim3(256), 0, s, g);
            return;
        }
    }
    if constexpr (std::is_same<R, double>::value && TM == 2 && TN == 1 && !CONJA) {
        if ((lu_update || m3) && nsplit == 1 && dma::fits(g)) {
            if (g.M % 64 == 0 && g.N % 32 == 0)
                hipLaunchKernelGGL(gemm_dma_n32_kernel, grid, dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL(gemm_dma_n32_ragged_kernel, grid, dim3(256), 0, s, g);
            return;
        }
    }
    if constexpr (std::is_same<R, float>::value && TM == 4 && TN == 1 && !CONJA) {
        if ((lu_update || m3) && nsplit == 1 && dma::fits32(g)) {
            hipLaunchKernelGGL(gemm_dma32_n32_kernel, grid, dim3(256), 0, s, g);
            return;
        }
    }
    if constexpr (std::is_same<R, float>::value && TM == 4 && TN == 2 && !CONJA) {
        if ((lu_update || m3) && nsplit == 1 && dma::fits32(g)) {
            if (lu_update)
                hipLaunchKernelGGL(lu_update_dma32_kernel, grid, dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL(gemm_dma32_kernel, grid, dim3(256), 0, s, g);
            return;
        }
    }
    if constexpr (!CONJA) {
        if (lu_update && nsplit == 1) {
            hipLaunchKernelGGL((lu_update_kernel<R, TM, TN, BK>), grid, dim3(256), 0, s, g);
            return;
        }
    }
    if constexpr (!CONJA) {
        if (m3) {
            if (nsplit > 1)
                hipLaunchKernelGGL((gemm_kernel<R, TM, TN, BK, CONJA, true, true>), grid, dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL((gemm_kernel<R, TM, TN, BK, CONJA, false, true>), grid, dim3(256), 0, s, g);
            return;
        }
    }
    if (nsplit > 1)
        hipLaunchKernelGGL((gemm_kernel<R, TM, TN, BK, CONJA, true, false>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_kernel<R, TM, TN, BK, CONJA, false, false>), grid, dim3(256), 0, s, g);
}

// Default tile choice, from measured sweeps on MI355X: FP64 runs best with the 64 x 64 tile
// (two waves per SIMD); FP32 with 128 x 64 once there are enough tiles to fill the chip.
// Problems with fewer than four 64 x 64 tiles per compute unit take the 32 x 32 tile, which
// quadruples the number of workgroups and cuts the serial MFMA chain per tile by 4 (measured:
// A_j Q at 8192 x 160 x 8192, 38 -> 54 TFLOP/s; the 256 x 160 x 256 diagonal-block solves of
// 24 nodes, 23 -> 36 TFLOP/s; the 8192 x 160 x 640 block residual, 34 -> 45 TFLOP/s).
template <typename R>
static GemmConfig pick_config(int64_t M, int64_t N, int64_t K, int batch) {
    GemmConfig c;
    (void)K;
    if (sizeof(R) == 4 && ceil_div(M, 128) * ceil_div(N, 64) * batch >= 512) {
        c.tm = 4;
        c.tn = 2;
    } else if (ceil_div(M, 64) * ceil_div(N, 64) * batch < 1024) {
        c.tm = 1;
        c.tn = 1;
    }
    return c;
}

template <typename R>
void gemm(hipStream_t s, bool conjA, int64_t M, int64_t N, int64_t K, Cx<R> alpha,
          const Cx<R>* A, int64_t lda, int64_t sA, const Cx<R>* B, int64_t ldb, int64_t sB,
          Cx<R> beta, Cx<R>* C, int64_t ldc, int64_t sC, int batch, Cx<R>* ws,
          int64_t ws_elems, const GemmConfig* force, bool lu_update) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    GemmArgs<R> g;
    g.M = M; g.N = N; g.K = K;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = B; g.ldb = ldb; g.sB = sB;
    g.C = C; g.ldc = ldc; g.sC = sC;
    g.P = nullptr; g.nsplit = 1; g.kchunk = K;
    if (K <= 0) {
        // C = beta C
        g.K = 0;
    }
    GemmConfig c = force ? *force : pick_config<R>(M, N, K, batch);
    // FP64 3M products too small for 64 x 64 tiles take the 64 x 32 direct-to-LDS tile once it
    // gives 256 workgroups (measured against 32 x 32 tiles: the triangular solves' diagonal
    // blocks 256 x 160 x 256, 24 nodes, 55 -> 50 us; their chunk-internal updates 768 x 160 x 256
    // 125 -> 105 us; X = Q Y, 8192 x 160 x 160, 47 -> 45 us; the block residual 8192 x 160 x 640
    // 127 -> 116 us; below 256 workgroups, 256 x 64 x 256 with 16 nodes, 28 against 31 us)
    if (!force && sizeof(R) == 8 && c.tm == 1 && c.tn == 1 && !conjA && K >= 64 && K % (2 * dma::BK) == 0 &&
        ceil_div(M, 64) * ceil_div(N, 32) * batch >= 256)
        c = GemmConfig{2, 1};
    // split-K for small outputs with long reductions (projections, Gram matrices)
    int nsplit = 1;
    const int64_t tiles = ceil_div(M, 32 * c.tm) * ceil_div(N, 32 * c.tn) * batch;
    // FP64 3M products with a long reduction into fewer 64 x 64 tiles than three workgroups per
    // compute unit (the projections A_j Q, 8192 x 160 x 8192): the direct-to-LDS tile with the
    // reduction split so that at least two rounds of workgroups are in flight, partial products
    // summed by gemm_reduce (measured 8192 x 160 x 8192: 32 x 32 tiles, 1280 workgroups, against
    // 64 x 64 tiles with 4 splits, 1536 workgroups)
    if constexpr (sizeof(R) == 8) {
        const int64_t t64 = ceil_div(M, 64) * ceil_div(N, 64) * batch;
        if (!force && ws && !conjA && !lu_update && K >= 2048 && t64 < 768 && dma::fits(g)) {
            int want = (int)std::min<int64_t>(ceil_div(1536, t64), K / 1024);
            while (want > 1 && (int64_t)want * M * N * batch > ws_elems) --want;
            if (want >= 2 && t64 * want >= 768) {
                g.tilesM = (int)ceil_div(M, 64);
                g.tilesN = (int)ceil_div(N, 64);
                g.kchunk = ceil_div(ceil_div(K, want), 2 * dma::BK) * 2 * dma::BK;
                g.nsplit = (int)ceil_div(K, g.kchunk);
                g.P = ws;
                dim3 grid(g.tilesM * g.tilesN, batch, g.nsplit);
                hipLaunchKernelGGL(gemm_dma_split_kernel, grid, dim3(256), 0, s, g);
                NLF_HIP(hipGetLastError());
                const int64_t MN = M * N;
                dim3 rgrid((unsigned)std::min<int64_t>(ceil_div(MN, 256), 1024), batch);
                hipLaunchKernelGGL((gemm_reduce_kernel<R>), rgrid, dim3(256), 0, s, M, N, g.nsplit,
                                   (const Cx<R>*)g.P, beta, C, ldc, sC);
                NLF_HIP(hipGetLastError());
                return;
            }
        }
    }
    // A ragged last column of 64-wide tiles that would hold at most 32 columns (N = 160 = 2 x 64
    // + 32: a sixth of the tile's MFMA work wasted) goes to a second launch of 32 x 32 tiles.
    // Measured on the right-looking updates of the block triangular solves (n = 8192, 160
    // right-hand sides, 24 nodes, K = 256): 64 x 64 tiles 61 TFLOP/s, 32 x 32 tiles 62
    // With the edge on 64 x 32 (FP64) or 128 x 32 (FP32) direct-to-LDS tiles the split also beats
    // one launch whose last tile column idles half its waves: FP64 3.14 against 3.20 ms, and
    // 1920 x 80 x 256 with 128 nodes 0.66 against 0.77; complex64 7168 x 160 x 1024 with 24 nodes
    // 1.63 against 1.75 ms, 1920 x 80 x 256 with 128 nodes 0.39 against 0.44
    if (!force && !lu_update && c.tn == 2 && N > 64 && N % 64 != 0 && N % 64 <= 32 &&
        !(ws && tiles < 256 && K >= 512)) {
        const int64_t N0 = N - N % 64;
        gemm<R>(s, conjA, M, N0, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ws, ws_elems, &c,
                lu_update);
        // the remaining columns on 64 x 32 (FP64) or 128 x 32 (FP32) direct-to-LDS tiles where the 3M
        // product qualifies
        const bool dq = !conjA && K >= 64 && K % (2 * dma::BK) == 0;
        const GemmConfig c1 = dq ? (sizeof(R) == 8 ? GemmConfig{2, 1} : GemmConfig{4, 1}) : GemmConfig{1, 1};
        gemm<R>(s, conjA, M, N - N0, K, alpha, A, lda, sA, B + N0 * ldb, ldb, sB, beta, C + N0 * ldc, ldc, sC,
                batch, ws, ws_elems, &c1, lu_update);
        return;
    }
    if (ws && tiles < 256 && K >= 512) {
        int want = (int)std::min<int64_t>(ceil_div(512, tiles), ceil_div(K, 256));
        while (want > 1 && (int64_t)want * M * N * batch > ws_elems) --want;
        if (want > 1) {
            nsplit = want;
            g.kchunk = ceil_div(ceil_div(K, nsplit), 16) * 16;
            nsplit = (int)ceil_div(K, g.kchunk);
            g.P = ws;
            g.nsplit = nsplit;
        }
    }
// K step per LDS stage: 8 for the 64- and 128-row tiles (half the LDS, so four workgroups
// share a CU and hide each other's barriers; measured 4-6% faster), 16 otherwise
    // Products op(A) = A take 3M once the reduction is long enough to pay for the third
    // accumulator (every contraction of the path but the Gram and projection products Q^H X).
    // In FP32 these are the complex64 factorisation and solves of the precision form, whose
    // FP64 refinement absorbs the larger rounding (delay8192: solves 144 -> 123 ms per solve,
    // the same six iterations and refinement sweeps)
    const bool m3 = !conjA && K >= 64;
#define NLF_GEMM_CASE(TM_, TN_)                                                          \
    if (c.tm == TM_ && c.tn == TN_) {                                                   \
        constexpr int BKX = (TM_ == 1 || (TM_ == 4 && TN_ == 4)) ? 16 : 8;               \
        if (conjA) launch_tiles<R, TM_, TN_, BKX, true>(s, g, batch, nsplit, false, false);   \
        else       launch_tiles<R, TM_, TN_, BKX, false>(s, g, batch, nsplit, lu_update, m3); \
    } else
    NLF_GEMM_CASE(1, 1)
    NLF_GEMM_CASE(2, 1)
    NLF_GEMM_CASE(2, 2)
    NLF_GEMM_CASE(4, 2)
    if constexpr (sizeof(R) == 4) {
        NLF_GEMM_CASE(4, 1)
        NLF_GEMM_CASE(4, 4)
        { throw Error{1, "gemm: unsupported tile config"}; }
    } else {
        throw Error{1, "gemm: unsupported tile config"};
    }
#undef NLF_GEMM_CASE
    NLF_HIP(hipGetLastError());
    if (nsplit > 1) {
        const int64_t MN = M * N;
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(MN, 256), 1024), batch);
        hipLaunchKernelGGL((gemm_reduce_kernel<R>), grid, dim3(256), 0, s, M, N, nsplit,
                           (const Cx<R>*)g.P, beta, C, ldc, sC);
        NLF_HIP(hipGetLastError());
    }
}

template void gemm<double>(hipStream_t, bool, int64_t, int64_t, int64_t, Cx<double>,
                           const Cx<double>*, int64_t, int64_t, const Cx<double>*, int64_t,
                           int64_t, Cx<double>, Cx<double>*, int64_t, int64_t, int,
                           Cx<double>*, int64_t, const GemmConfig*, bool);
template void gemm<float>(hipStream_t, bool, int64_t, int64_t, int64_t, Cx<float>,
                          const Cx<float>*, int64_t, int64_t, const Cx<float>*, int64_t,
                          int64_t, Cx<float>, Cx<float>*, int64_t, int64_t, int, Cx<float>*,
                          int64_t, const GemmConfig*, bool);

}  // namespace nlf
