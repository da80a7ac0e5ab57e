// Batched complex LU with partial pivoting and the triangular solves that apply T(z_k)^{-1}
// (Step 4 of Algorithm 1 multiplies by T^{-1}(z_j) by solving linear systems; the shifts are
// fixed for the whole iteration, so each T(z_k) is factored once and the factors are reused).
//
// Factorisation: recursive (column-halving) LU.  Columns [k0, k0+nc) of the trailing rows are
// split into halves: factor the left half, apply its row exchanges to the right half, solve
// with the unit-lower diagonal block (recursive TRSM), update the lower-right block with a
// complex GEMM on MFMA, factor it, and apply its exchanges back to the left half.  Almost all
// flops land in large GEMMs; the recursion stops at panels of at most 32 columns.
//
// Panel kernel: one 1024-thread workgroup per matrix factors an (n-k0) x w panel (w <= 32).
// Each thread owns RPT fixed rows; the panel is processed in sub-blocks of SB columns held in
// registers (left-looking between sub-blocks: the sub-block is updated with the L columns
// already factored, through a small LDS forward substitution for its top rows).  Pivot search
// is a wavefront shuffle reduction followed by a 16-wave LDS reduction on |Re| + |Im|.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <climits>

namespace nlf {

constexpr int PANEL_NT = 1024;
constexpr int PANEL_WMAX = 32;
constexpr int TRSM_NB = 64;
constexpr int64_t LU_INV_NB = 256;   // diagonal block order of the explicit L/U block inverses
constexpr int64_t LU_PANEL_NB = 512; // panel width of the blocked LU (a multiple of LU_INV_NB)
static_assert(LU_PANEL_NB % LU_INV_NB == 0, "panel = whole inverse blocks");
constexpr int TRSM_CB = 8;      // right-hand-side columns per wavefront in the TRSM leaf

// One step of an argmax reduction: the lane pattern CTRL (a DPP control: quad permutation or
// row mirror) brings a partner's (value, row); the larger value wins, ties go to the lower row.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL, typename R>
__device__ __forceinline__ void argmax_dpp(R& v, int& row) {
    R ov;
    if constexpr (sizeof(R) == 8) {
        const long long bits = __double_as_longlong(v);
        const int lo = dpp_move<CTRL>((int)bits), hi = dpp_move<CTRL>((int)(bits >> 32));
        ov = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    } else {
        ov = __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
    }
    const int orow = dpp_move<CTRL>(row);
    const bool take = (ov > v) | ((ov == v) & (orow < row));   // bitwise: no branches
    v = take ? ov : v;
    row = take ? orow : row;
}

// Argmax within each row of 16 lanes: swap neighbours (quad_perm [1,0,3,2]), pairs
// ([2,3,0,1]), half rows (row_half_mirror), whole row (row_mirror); afterwards every lane of a
// row holds the row's winner.
template <typename R>
__device__ __forceinline__ void row16_argmax(R& v, int& row) {
    argmax_dpp<0xB1>(v, row);
    argmax_dpp<0x4E>(v, row);
    argmax_dpp<0x141>(v, row);
    argmax_dpp<0x140>(v, row);
}

template <typename R>
__device__ __forceinline__ void wave_argmax(R& v, int& row) {
    row16_argmax(v, row);
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
        R ov = __shfl_xor(v, off, 64);
        int orow = __shfl_xor(row, off, 64);
        const bool take = (ov > v) | ((ov == v) & (orow < row));
        v = take ? ov : v;
        row = take ? orow : row;
    }
}

// 1 / p with one real division: p is scaled by a power of two (exact) so that |p|^2 neither
// overflows nor underflows, and 1/p = conj(p) / |p|^2.
template <typename R>
__device__ __forceinline__ Cx<R> crecip(Cx<R> p) {
    const int e = ilogb(fmax(fabs(p.re), fabs(p.im)));
    const R a = scalbn(p.re, -e), b = scalbn(p.im, -e);
    const R d = R(1) / (a * a + b * b);
    return Cx<R>(scalbn(a * d, -e), scalbn(-b * d, -e));
}

// Buffer descriptor of `rows` consecutive complex values (raw addressing: a load at a byte
// offset at or beyond the length returns zero; rows <= 0 gives an empty range).
template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const Cx<R>* col, int rows) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Cx<R>*>(col), (short)0,
                                             max(rows, 0) * (int)sizeof(Cx<R>), 0x00020000);
}

template <typename R>
__device__ __forceinline__ Cx<R> buffer_load_cx(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    if constexpr (sizeof(R) == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        return Cx<R>(__longlong_as_double(((long long)v[1] << 32) | v[0]),
                     __longlong_as_double(((long long)v[3] << 32) | v[2]));
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        return Cx<R>(__uint_as_float(v[0]), __uint_as_float(v[1]));
    }
}

template <typename R, int RPT, int SB, int NT>
__global__ __launch_bounds__(NT) void panel_kernel(Cx<R>* A0, int64_t lda, int64_t sA,
                                                        int64_t n, int64_t k0, int w,
                                                        int32_t* ipiv, int32_t* info) {
    const int64_t bidx = blockIdx.x;
    Cx<R>* A = A0 + bidx * sA + k0 + k0 * lda;      // panel origin
    int32_t* piv = ipiv + bidx * n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mp = (int)(n - k0);

    __shared__ Cx<R> Ltop[PANEL_WMAX][PANEL_WMAX + 1];
    __shared__ Cx<R> Utop[PANEL_WMAX][SB];
    // per column, double-buffered by column parity: each wave's best candidate (value, row and
    // the row's sub-block entries) and the current row j, so one barrier per column suffices
    constexpr int NW = NT / 64;
    __shared__ R candv[2][NW];
    __shared__ int candr[2][NW];
    __shared__ Cx<R> candrow[2][NW][SB];
    __shared__ Cx<R> rowJbuf[2][SB];

    Cx<R> x[RPT][SB];

    for (int s0 = 0; s0 < w; s0 += SB) {
        const int bw = min(SB, w - s0);
        // (1) top rows of the sub-block: U = L11^{-1} A[0:s0, s0:s0+bw] (unit-lower L11)
        if (s0 > 0) {
            for (int e = tid; e < s0 * s0; e += NT) {
                const int t = e % s0, u = e / s0;
                if (u < t) Ltop[t][u] = A[t + (int64_t)u * lda];
            }
            for (int e = tid; e < s0 * bw; e += NT) {
                const int t = e % s0, c = e / s0;
                Utop[t][c] = A[t + (int64_t)(s0 + c) * lda];
            }
            __syncthreads();
            if (wave == 0) {
                for (int u = 0; u + 1 < s0; ++u) {
                    const int rows = s0 - 1 - u;
                    for (int e = lane; e < rows * bw; e += 64) {
                        const int t = u + 1 + e % rows, c = e / rows;
                        Cx<R> v = Utop[t][c];
                        cfms(v, Ltop[t][u], Utop[u][c]);
                        Utop[t][c] = v;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
            for (int e = tid; e < s0 * bw; e += NT) {
                const int t = e % s0, c = e / s0;
                A[t + (int64_t)(s0 + c) * lda] = Utop[t][c];
            }
        }
        // (2) load the sub-block rows >= s0 and (3) left-looking update with L[:, 0:s0]
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = tid + NT * i;
            const bool ok = r >= s0 && r < mp;
#pragma unroll
            for (int c = 0; c < SB; ++c)
                x[i][c] = (ok && c < bw) ? A[r + (int64_t)(s0 + c) * lda] : Cx<R>(0, 0);
        }
        // All RPT rows of a column of L are loaded together (one round trip per column): row
        // block i has its own buffer descriptor, so the rows share one lane offset and rows at
        // or beyond mp read zero; rows above s0 compute values that are never used.
        {
            const uint32_t loff = (uint32_t)tid * (uint32_t)sizeof(Cx<R>);
#pragma nounroll
            for (int u = 0; u < s0; ++u) {
                const Cx<R>* colu = A + (int64_t)u * lda;
                Cx<R> l[RPT];
#pragma unroll
                for (int i = 0; i < RPT; ++i) l[i] = buffer_load_cx<R>(column_rsrc(colu + NT * i, mp - NT * i), loff);
#pragma unroll
                for (int c = 0; c < SB; ++c) {
                    const Cx<R> uv = (c < bw) ? Utop[u][c] : Cx<R>(0, 0);
#pragma unroll
                    for (int i = 0; i < RPT; ++i) cfms(x[i][c], l[i], uv);
                }
            }
        }
        // (4) factor the sub-block column by column
#pragma unroll
        for (int c = 0; c < SB; ++c) {
          if (c < bw) {
            const int j = s0 + c, par = j & 1;
            R best = R(-1);
            int brow = INT_MAX;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = tid + NT * i;
                if (r >= j && r < mp) {
                    const R v = abs1(x[i][c]);
                    if (v > best) { best = v; brow = r; }
                }
            }
            wave_argmax(best, brow);
            if (lane == 0) { candv[par][wave] = best; candr[par][wave] = brow; }
            if (brow != INT_MAX && tid == brow % NT) {      // the wave's winner publishes its row
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (i == brow / NT)
#pragma unroll
                        for (int cc = 0; cc < SB; ++cc) candrow[par][wave][cc] = x[i][cc];
            }
            const int ownJ = j % NT, iJ = j / NT;
            if (tid == ownJ) {
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (i == iJ)
#pragma unroll
                        for (int cc = 0; cc < SB; ++cc) rowJbuf[par][cc] = x[i][cc];
            }
            __syncthreads();
            // every wave reduces the NW <= 16 candidates itself in its first row of lanes (lane q
            // holds candidate q; the candidate index travels in the low bits of the row key)
            static_assert(NW <= 16, "one DPP row per candidate set");
            R pv = lane < NW ? candv[par][lane] : R(-1);
            const int cand_row = lane < NW ? candr[par][lane] : INT_MAX;
            int key = cand_row == INT_MAX ? INT_MAX : (cand_row << 4) | (lane & 15);
            row16_argmax(pv, key);
            pv = __shfl(pv, 0, 64);
            key = __shfl(key, 0, 64);
            int pr = key == INT_MAX ? INT_MAX : (key >> 4);
            const int pq = key == INT_MAX ? 0 : (key & 15);
            if (pr == INT_MAX || !(pv > R(0))) {   // all zero (or NaN): no exchange
                pr = j;
                pv = R(0);
            }
            if (tid == 0) {
                piv[k0 + j] = (int32_t)(k0 + pr);
                if (pv == R(0) && info[bidx] == 0) info[bidx] = (int32_t)(k0 + j + 1);
            }
            Cx<R> prow[SB];
            if (pr != j) {
#pragma unroll
                for (int cc = 0; cc < SB; ++cc) prow[cc] = candrow[par][pq][cc];
                const int ownP = pr % NT, iP = pr / NT;
                if (tid == ownJ) {
#pragma unroll
                    for (int i = 0; i < RPT; ++i)
                        if (i == iJ)
#pragma unroll
                            for (int cc = 0; cc < SB; ++cc) x[i][cc] = prow[cc];
                }
                if (tid == ownP) {
#pragma unroll
                    for (int i = 0; i < RPT; ++i)
                        if (i == iP)
#pragma unroll
                            for (int cc = 0; cc < SB; ++cc) x[i][cc] = rowJbuf[par][cc];
                }
                if (tid < w && (tid < s0 || tid >= s0 + bw)) {
                    Cx<R>* a = A + (int64_t)tid * lda;
                    const Cx<R> t = a[j];
                    a[j] = a[pr];
                    a[pr] = t;
                }
            } else {
#pragma unroll
                for (int cc = 0; cc < SB; ++cc) prow[cc] = rowJbuf[par][cc];
            }
            if (pv > R(0)) {
                const Cx<R> inv = crecip(prow[c]);
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = tid + NT * i;
                    if (r > j && r < mp) {
                        const Cx<R> l = x[i][c] * inv;
                        x[i][c] = l;
#pragma unroll
                        for (int cc = 0; cc < SB; ++cc)
                            if (cc > c && cc < bw) cfms(x[i][cc], l, prow[cc]);
                    }
                }
            }
          }
        }
        // (5) store the sub-block
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = tid + NT * i;
            if (r >= s0 && r < mp) {
#pragma unroll
                for (int c = 0; c < SB; ++c)
                    if (c < bw) A[r + (int64_t)(s0 + c) * lda] = x[i][c];
            }
        }
        __syncthreads();
    }
}

// Composed permutation of all row exchanges: (P A)[i] = A[perm[i]].  One workgroup per matrix.
__global__ __launch_bounds__(1024) void perm_kernel(int64_t n, const int32_t* ipiv, int32_t* perm) {
    extern __shared__ int sp[];
    const int64_t b = blockIdx.x;
    for (int r = threadIdx.x; r < n; r += blockDim.x) sp[r] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t* p = ipiv + b * n;
        for (int k = 0; k < n; ++k) {
            const int q = p[k];
            const int t = sp[k];
            sp[k] = sp[q];
            sp[q] = t;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) perm[b * n + r] = sp[r];
}

// (dst, src) row pairs that realise the exchanges k in [k1, k2) (applied in order).
// list layout per matrix: [2][L] with L = 2 (k2 - k1); dst = -1 marks an unused entry.
__global__ __launch_bounds__(1024) void swaplist_kernel(int64_t n, int64_t k1, int64_t k2,
                                                        const int32_t* ipiv, int32_t* list) {
    extern __shared__ int sp[];               // rows [k1, n)
    const int64_t b = blockIdx.x;
    const int span = (int)(n - k1), cnt = (int)(k2 - k1), L = 2 * cnt;
    const int32_t* p = ipiv + b * n;
    int32_t* dst = list + b * 2 * (int64_t)L;
    int32_t* src = dst + L;
    for (int r = threadIdx.x; r < span; r += blockDim.x) sp[r] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < cnt; ++k) {
            const int q = p[k1 + k] - (int)k1;
            const int t = sp[k];
            sp[k] = sp[q];
            sp[q] = t;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        dst[e] = (int)k1 + e;
        src[e] = (int)k1 + sp[e];
        const int q = p[k1 + e];
        if (q >= k2) {
            dst[cnt + e] = q;
            src[cnt + e] = (int)k1 + sp[q - k1];
        } else {
            dst[cnt + e] = -1;
            src[cnt + e] = 0;
        }
    }
}

// Row exchanges as (dst, src) lists, applied to the columns [c0a, c0a + na) and [c0b, c0b + nb)
// (the left and right parts of a panel in one launch).  A 512-thread workgroup owns CW
// consecutive columns of the union: every thread gathers its EPT entries of all CW columns,
// the workgroup meets once, then every thread scatters them.  Entries whose row keeps its
// content (dst == src: the panel rows the pivoting left in place) are skipped.
template <typename R, int EPT, int CW>
__global__ __launch_bounds__(512) void laswp_apply_kernel(Cx<R>* A0, int64_t lda, int64_t sA,
                                                          int64_t c0a, int64_t na, int64_t c0b,
                                                          int64_t nb, const int32_t* list, int L) {
    const int64_t b = blockIdx.y;
    Cx<R>* A = A0 + b * sA;
    const int32_t* dst = list + b * 2 * (int64_t)L;
    const int32_t* src = dst + L;
    int d[EPT], sr[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + 512 * i;
        d[i] = e < L ? dst[e] : -1;
        sr[i] = e < L ? src[e] : 0;
        if (d[i] == sr[i]) d[i] = -1;   // a row that stays put moves no data
    }
    const int64_t total = na + nb, q0 = (int64_t)blockIdx.x * CW;
    Cx<R> v[CW][EPT];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int64_t q = q0 + c;
        if (q < total) {
            const Cx<R>* col = A + (q < na ? c0a + q : c0b + (q - na)) * lda;
#pragma unroll
            for (int i = 0; i < EPT; ++i)
                if (d[i] >= 0) v[c][i] = col[sr[i]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int64_t q = q0 + c;
        if (q < total) {
            Cx<R>* col = A + (q < na ? c0a + q : c0b + (q - na)) * lda;
#pragma unroll
            for (int i = 0; i < EPT; ++i)
                if (d[i] >= 0) col[d[i]] = v[c][i];
        }
    }
}

// B <- T^{-1} B for one diagonal block of order nb <= 64 (unit-lower or upper triangular T).
// Four wavefronts per workgroup share T, staged transposed in LDS (lane i reads T(i, t) from
// consecutive addresses); each wavefront owns CB columns of B with lane i holding row i in
// registers, and broadcasts the solved row t through its own LDS slot.  After T is staged all
// communication stays inside a wavefront, whose LDS operations complete in issue order, so
// the substitution itself needs no workgroup barrier.
template <typename R, bool UPPER, int CB>
__global__ __launch_bounds__(256) void trsm_leaf_kernel(int nb, int64_t N, const Cx<R>* T0,
                                                        int64_t ldt, int64_t sT, Cx<R>* B0,
                                                        int64_t ldb, int64_t sB) {
    __shared__ Cx<R> Tt[TRSM_NB][TRSM_NB + 1];      // Tt[t][i] = T(i, t)
    __shared__ Cx<R> xts[4][CB];
    const int64_t b = blockIdx.y;
    const Cx<R>* T = T0 + b * sT;
    Cx<R>* B = B0 + b * sB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cbase = ((int64_t)blockIdx.x * 4 + wave) * CB;
    Cx<R>* xt = xts[wave];
    // all loads are issued before any is used (clamped in-range addresses, out-of-block
    // elements replaced by zero afterwards), so the triangle and the right-hand sides arrive
    // in one round trip instead of one per loop iteration
    constexpr int PER = TRSM_NB * TRSM_NB / 256;
    Cx<R> tv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q, i = e % TRSM_NB, t = e / TRSM_NB;
        tv[q] = T[min(i, nb - 1) + (int64_t)min(t, nb - 1) * ldt];
    }
    Cx<R> x[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
        x[c] = B[min(lane, nb - 1) + min(cbase + c, N - 1) * ldb];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q, i = e % TRSM_NB, t = e / TRSM_NB;
        Tt[t][i] = (i < nb && t < nb) ? tv[q] : Cx<R>(0, 0);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (!(lane < nb && cbase + c < N)) x[c] = Cx<R>(0, 0);
    __syncthreads();
    if (!UPPER) {
        for (int t = 0; t + 1 < nb; ++t) {
            if (lane == t) {
#pragma unroll
                for (int c = 0; c < CB; ++c) xt[c] = x[c];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane > t) {
                const Cx<R> l = Tt[t][lane];
#pragma unroll
                for (int c = 0; c < CB; ++c) cfms(x[c], l, xt[c]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        // every lane inverts its own diagonal entry up front, off the substitution's critical path
        const Cx<R> dinv = lane < nb ? cdiv(Cx<R>(1, 0), Tt[lane][lane]) : Cx<R>(0, 0);
        for (int t = nb - 1; t >= 0; --t) {
            if (lane == t) {
                const Cx<R> inv = dinv;
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    x[c] = x[c] * inv;
                    xt[c] = x[c];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane < t) {
                const Cx<R> u = Tt[t][lane];
#pragma unroll
                for (int c = 0; c < CB; ++c) cfms(x[c], u, xt[c]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (lane < nb && cbase + c < N) B[lane + (cbase + c) * ldb] = x[c];
}

// X_b[i, c] = B_b[perm_b[i], c]
template <typename R>
__global__ __launch_bounds__(256) void gather_rows_kernel(int64_t n, int64_t ncols,
                                                          const int32_t* perm, const Cx<R>* B0,
                                                          int64_t ldb, int64_t sB, Cx<R>* X0,
                                                          int64_t ldx, int64_t sX) {
    const int64_t b = blockIdx.y;
    const int32_t* p = perm + b * n;
    const Cx<R>* B = B0 + b * sB;
    Cx<R>* X = X0 + b * sX;
    const int64_t total = n * ncols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, c = e / n;
        X[i + c * ldx] = B[p[i] + c * ldb];
    }
}

// X[perm[i]] = Z[i] per matrix: the row permutation P^T that ends a solve with (P A)^H.
template <typename R>
__global__ __launch_bounds__(256) void scatter_rows_kernel(int64_t n, int64_t ncols,
                                                           const int32_t* perm, const Cx<R>* Z0,
                                                           int64_t ldz, int64_t sZ, Cx<R>* X0,
                                                           int64_t ldx, int64_t sX) {
    const int64_t b = blockIdx.y;
    const int32_t* p = perm + b * n;
    const Cx<R>* Z = Z0 + b * sZ;
    Cx<R>* X = X0 + b * sX;
    const int64_t total = n * ncols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, c = e / n;
        X[p[i] + c * ldx] = Z[i + c * ldz];
    }
}

// Identity in every s x s block of a strided set (the right-hand sides of the block inversion).
template <typename R>
__global__ __launch_bounds__(256) void identity_blocks_kernel(int64_t s, int64_t ld, int64_t count,
                                                              int64_t stride, Cx<R>* out) {
    const int64_t per = s * s, total = per * count;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t q = e / per, r = e % per;
        const int64_t i = r % s, j = r / s;
        out[q * stride + i + j * ld] = Cx<R>(i == j ? R(1) : R(0), R(0));
    }
}

template <typename R>
__global__ __launch_bounds__(256) void copy_batched_kernel(int64_t rows, int64_t cols,
                                                           const Cx<R>* in, int64_t ldi, int64_t si,
                                                           Cx<R>* out, int64_t ldo, int64_t so) {
    const int64_t b = blockIdx.y, total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % rows, c = e / rows;
        out[b * so + i + c * ldo] = in[b * si + i + c * ldi];
    }
}

// ------------------------------------------------------------------------------ host side

template <typename R>
void trsm_lower_unit(hipStream_t s, int64_t n, int64_t N, int batch, const Cx<R>* L,
                     int64_t ldl, int64_t sL, Cx<R>* B, int64_t ldb, int64_t sB) {
    if (n <= 0 || N <= 0) return;
    if (n <= TRSM_NB) {
        ProfScope ps(trsm_class(), s, 4.0 * n * n * N * batch, 0);
        dim3 grid((unsigned)ceil_div(N, 4 * TRSM_CB), batch);
        hipLaunchKernelGGL((trsm_leaf_kernel<R, false, TRSM_CB>), grid, dim3(256), 0, s, (int)n, N,
                           L, ldl, sL, B, ldb, sB);
        NLF_HIP(hipGetLastError());
        return;
    }
    const int64_t n1 = std::max<int64_t>(TRSM_NB, (n / 2) / TRSM_NB * TRSM_NB);
    trsm_lower_unit<R>(s, n1, N, batch, L, ldl, sL, B, ldb, sB);
    {
        ProfScope ps(trsm_class(), s, 8.0 * (n - n1) * N * n1 * batch, 0);
        gemm<R>(s, false, n - n1, N, n1, Cx<R>(-1, 0), L + n1, ldl, sL, B, ldb, sB,
                Cx<R>(1, 0), B + n1, ldb, sB, batch);
    }
    trsm_lower_unit<R>(s, n - n1, N, batch, L + n1 + n1 * ldl, ldl, sL, B + n1, ldb, sB);
}

template <typename R>
void trsm_upper(hipStream_t s, int64_t n, int64_t N, int batch, const Cx<R>* U, int64_t ldu,
                int64_t sU, Cx<R>* B, int64_t ldb, int64_t sB) {
    if (n <= 0 || N <= 0) return;
    if (n <= TRSM_NB) {
        ProfScope ps(trsm_class(), s, 4.0 * n * n * N * batch, 0);
        dim3 grid((unsigned)ceil_div(N, 4 * TRSM_CB), batch);
        hipLaunchKernelGGL((trsm_leaf_kernel<R, true, TRSM_CB>), grid, dim3(256), 0, s, (int)n, N,
                           U, ldu, sU, B, ldb, sB);
        NLF_HIP(hipGetLastError());
        return;
    }
    const int64_t n1 = std::max<int64_t>(TRSM_NB, (n / 2) / TRSM_NB * TRSM_NB);
    trsm_upper<R>(s, n - n1, N, batch, U + n1 + n1 * ldu, ldu, sU, B + n1, ldb, sB);
    {
        ProfScope ps(trsm_class(), s, 8.0 * n1 * N * (n - n1) * batch, 0);
        gemm<R>(s, false, n1, N, n - n1, Cx<R>(-1, 0), U + n1 * ldu, ldu, sU, B + n1, ldb,
                sB, Cx<R>(1, 0), B, ldb, sB, batch);
    }
    trsm_upper<R>(s, n1, N, batch, U, ldu, sU, B, ldb, sB);
}

template <typename R>
static void launch_panel(hipStream_t s, int batch, Cx<R>* A, int64_t lda, int64_t sA,
                         int64_t n, int64_t k0, int w, int32_t* ipiv, int32_t* info) {
    const int64_t mp = n - k0;
    const double fl = 8.0 * batch * ((double)mp * w * w - (double)w * w * w / 3.0) / 2.0;
    ProfScope ps(NLF_PROF_PANEL, s, fl, 0);
#define NLF_PANEL(RPT_, SB_, NT_) \
    hipLaunchKernelGGL((panel_kernel<R, RPT_, SB_, NT_>), dim3(batch), dim3(NT_), 0, s, A, lda, sA, n, k0, w, ipiv, info)
    // RPT rows per thread (RPT x NT >= mp) and sub-block width SB: RPT x SB complex values per
    // thread stay within the VGPR budget (128 per thread at 1024 threads, 256 at 512)
    if constexpr (sizeof(R) == 8) {
        if (mp <= 1024) NLF_PANEL(1, 8, 1024);
        else if (mp <= 2048) NLF_PANEL(2, 8, 1024);
        else if (mp <= 4096) NLF_PANEL(4, 4, 1024);
        else if (mp <= 8192) NLF_PANEL(8, 2, 1024);
        else throw Error{1, "getrf: matrix order above 8192 is not supported"};
    } else {
        if (mp <= 1024) NLF_PANEL(1, 16, 1024);
        else if (mp <= 2048) NLF_PANEL(2, 8, 1024);
        else if (mp <= 4096) NLF_PANEL(4, 8, 1024);
        else if (mp <= 8192) NLF_PANEL(8, 4, 1024);
        else throw Error{1, "getrf: matrix order above 8192 is not supported"};
    }
#undef NLF_PANEL
    NLF_HIP(hipGetLastError());
}

template <typename R>
static void laswp(hipStream_t s, int batch, Cx<R>* A, int64_t lda, int64_t sA, int64_t n,
                  int64_t k1, int64_t k2, int64_t c0, int64_t ncols, const int32_t* ipiv,
                  int32_t* list, int64_t c0b = 0, int64_t ncolsb = 0) {
    if (ncols + ncolsb <= 0 || k2 <= k1) return;
    const int L = (int)(2 * (k2 - k1));
    ProfScope ps(NLF_PROF_LASWP, s, 0, 2.0 * L * (ncols + ncolsb) * sizeof(Cx<R>) * batch);
    hipLaunchKernelGGL(swaplist_kernel, dim3(batch), dim3(1024), (size_t)(n - k1) * sizeof(int), s,
                       n, k1, k2, ipiv, list);
    NLF_HIP(hipGetLastError());
    const int64_t total = ncols + ncolsb;
#define NLF_LASWP(EPT_, CW_)                                                                        \
    hipLaunchKernelGGL((laswp_apply_kernel<R, EPT_, CW_>), dim3((unsigned)ceil_div(total, CW_), batch), \
                       dim3(512), 0, s, A, lda, sA, c0, ncols, c0b, ncolsb, list, L)
    if (L <= 512) NLF_LASWP(1, 16);
    else if (L <= 1024) NLF_LASWP(2, 8);
    else if (L <= 2048) NLF_LASWP(4, 4);
    else if (L <= 4096) NLF_LASWP(8, 2);
    else if (L <= 8192) NLF_LASWP(16, 1);
    else throw Error{1, "laswp: exchange range too large"};
#undef NLF_LASWP
    NLF_HIP(hipGetLastError());
}

int& lu_panel_width() {
    static thread_local int w = PANEL_WMAX;
    return w;
}

GemmConfig& lu_update_tile() {
    static thread_local GemmConfig c{0, 0};
    return c;
}

std::function<void(LuUpdateLaunch&&)>*& lu_update_hook() {
    static thread_local std::function<void(LuUpdateLaunch&&)>* h = nullptr;
    return h;
}

// The tile of the trailing-update GEMMs: the override when one is set, else the default choice.
static const GemmConfig* update_tile() {
    const GemmConfig& c = lu_update_tile();
    return c.tm > 0 ? &c : nullptr;
}

template <typename R>
static void getrf_rec(hipStream_t s, int64_t n, int batch, Cx<R>* A, int64_t lda, int64_t sA,
                      int64_t k0, int64_t nc, int32_t* ipiv, int32_t* info, int32_t* list) {
    const int pw = std::max(4, std::min(lu_panel_width(), PANEL_WMAX));
    if (nc <= pw) {
        launch_panel<R>(s, batch, A, lda, sA, n, k0, (int)nc, ipiv, info);
        return;
    }
    int64_t n1 = (nc / 2) / pw * pw;
    if (n1 < pw) n1 = pw;
    const int64_t n2 = nc - n1;
    getrf_rec<R>(s, n, batch, A, lda, sA, k0, n1, ipiv, info, list);
    laswp<R>(s, batch, A, lda, sA, n, k0, k0 + n1, k0 + n1, n2, ipiv, list);
    trsm_lower_unit<R>(s, n1, n2, batch, A + k0 + k0 * lda, lda, sA, A + k0 + (k0 + n1) * lda,
                       lda, sA);
    const int64_t mrest = n - (k0 + n1);
    {
        ProfScope ps(NLF_PROF_LU_REC_GEMM, s, 8.0 * mrest * n2 * n1 * batch,
                     sizeof(Cx<R>) * (2.0 * mrest * n2 + (double)mrest * n1 + (double)n1 * n2) * batch);
        gemm<R>(s, false, mrest, n2, n1, Cx<R>(-1, 0), A + (k0 + n1) + k0 * lda, lda, sA,
                A + k0 + (k0 + n1) * lda, lda, sA, Cx<R>(1, 0),
                A + (k0 + n1) + (k0 + n1) * lda, lda, sA, batch, nullptr, 0, update_tile());
    }
    getrf_rec<R>(s, n, batch, A, lda, sA, k0 + n1, n2, ipiv, info, list);
    laswp<R>(s, batch, A, lda, sA, n, k0 + n1, k0 + nc, k0, n1, ipiv, list);
}

int64_t getrf_scratch_ints(int64_t n, int batch) { return (int64_t)batch * 2 * (2 * n); }

// I in the two NB x NB blocks at p + q * per and p + q * per + NB^2, q < batch.
template <typename R>
static void identity_pair(hipStream_t s, int batch, int64_t NB, int64_t per, Cx<R>* p) {
    for (int h = 0; h < 2; ++h) {
        const int64_t total = NB * NB * batch;
        hipLaunchKernelGGL((identity_blocks_kernel<R>), dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 4096)),
                           dim3(256), 0, s, NB, NB, (int64_t)batch, per, p + h * NB * NB);
        NLF_HIP(hipGetLastError());
    }
}

// Right-looking blocked LU with LU_PANEL_NB-column panels (two LU_INV_NB blocks each).  Per
// panel: factor the panel (rows k0.., recursive LU above) and apply its exchanges to the
// columns left and right of it; invert the diagonal LU_INV_NB blocks of L and U (kept for the
// solves: later exchanges only touch rows below a block, so both are final here); then
// U12 = L11^{-1} A12 block by block (X_a = La^{-1} A_a, X_b = Lc^{-1} (A_b - Lb X_a)) and
// the rank-LU_PANEL_NB trailing update A22 -= A21 U12, the dominant GEMM.
// With a look-ahead stream, the panel factorisations and diagonal-block inverses run there:
// the columns of the next panel are updated first, so that the next panel is factored while
// the rest of the trailing matrix is updated on the main stream.  A panel only touches its
// own columns, the trailing update only the columns after it, and the row exchanges of the
// next panel (main stream) wait for both.
// tmp holds LU_PANEL_NB x (n - LU_PANEL_NB) elements per matrix (getrf_tmp_elems).
template <typename R>
static void getrf_blocked(hipStream_t s, int64_t n, int batch, Cx<R>* A, int64_t lda, int64_t sA,
                          int32_t* ipiv, int32_t* info, int32_t* list, Cx<R>* dinv, Cx<R>* tmp,
                          const LuAux* aux) {
    const int64_t NB = LU_INV_NB, PB = LU_PANEL_NB, per = lu_inverse_elems(n);
    const int64_t st = getrf_tmp_elems(n);
    const Cx<R> one(1, 0), mone(-1, 0), zero(0, 0);
    const bool la = aux && aux->s && aux->panel_done && aux->next_ready;
    hipStream_t sp = la ? aux->s : s;
    if (la) {   // the first panel follows the work already queued on the main stream
        NLF_HIP(hipEventRecord(aux->next_ready, s));
        NLF_HIP(hipStreamWaitEvent(sp, aux->next_ready, 0));
    }
    for (int64_t k0 = 0; k0 < n; k0 += PB) {
        const int64_t kb = std::min<int64_t>(PB, n - k0), k1 = k0 + kb, rest = n - k1;
        getrf_rec<R>(sp, n, batch, A, lda, sA, k0, kb, ipiv, info, list);
        for (int64_t d0 = k0; d0 < k1; d0 += NB) {       // inverses of the diagonal blocks
            const int64_t db = std::min<int64_t>(NB, k1 - d0);
            Cx<R>* Li = dinv + 2 * (d0 / NB) * NB * NB;
            identity_pair<R>(sp, batch, NB, per, Li);
            const Cx<R>* D = A + d0 + d0 * lda;
            trsm_lower_unit<R>(sp, db, db, batch, D, lda, sA, Li, NB, per);
            trsm_upper<R>(sp, db, db, batch, D, lda, sA, Li + NB * NB, NB, per);
        }
        if (la) {
            NLF_HIP(hipEventRecord(aux->panel_done, sp));
            NLF_HIP(hipStreamWaitEvent(s, aux->panel_done, 0));
        }
        laswp<R>(s, batch, A, lda, sA, n, k0, k1, 0, k0, ipiv, list, k1, rest);
        // columns [c0, c0 + w) of the trailing matrix: U12 = L11^{-1} A12, A22 -= A21 U12
        auto update = [&](int64_t c0, int64_t w) {
            Cx<R>* A12 = A + k0 + c0 * lda;
            {
                dim3 grid((unsigned)std::min<int64_t>(ceil_div(kb * w, 256), 2048), batch);
                hipLaunchKernelGGL((copy_batched_kernel<R>), grid, dim3(256), 0, s, kb, w,
                                   (const Cx<R>*)A12, lda, sA, tmp, PB, st);
                NLF_HIP(hipGetLastError());
            }
            for (int64_t d0 = k0; d0 < k1; d0 += NB) {
                const int64_t db = std::min<int64_t>(NB, k1 - d0), off = d0 - k0;
                const Cx<R>* Li = dinv + 2 * (d0 / NB) * NB * NB;
                ProfScope ps(NLF_PROF_TRSM, s, 8.0 * db * w * (db + off) * batch, 0);
                if (off > 0)   // subtract the contributions of the blocks above: tmp_b -= L_ba X_a
                    gemm<R>(s, false, db, w, off, mone, A + d0 + k0 * lda, lda, sA, A12, lda, sA, one,
                            tmp + off, PB, st, batch);
                gemm<R>(s, false, db, w, db, one, Li, NB, per, tmp + off, PB, st, zero, A12 + off, lda, sA, batch);
            }
            const double fl = 8.0 * rest * w * kb * batch;
            const double by = sizeof(Cx<R>) * (2.0 * rest * w + (double)rest * kb + (double)kb * w) * batch;
            const GemmConfig* tile = update_tile();
            if (std::function<void(LuUpdateLaunch&&)>* hook = lu_update_hook()) {
                const GemmConfig cfg = tile ? *tile : GemmConfig{0, 0};
                const Cx<R>* L21 = A + k1 + k0 * lda;
                Cx<R>* A22 = A + k1 + c0 * lda;
                LuUpdateLaunch u;
                u.launch = [=](hipStream_t st) {
                    gemm<R>(st, false, rest, w, kb, mone, L21, lda, sA, A12, lda, sA, one, A22, lda, sA, batch,
                            nullptr, 0, cfg.tm > 0 ? &cfg : nullptr, true);
                };
                u.flops = fl;
                u.bytes = by;
                (*hook)(std::move(u));
                return;
            }
            ProfScope ps(NLF_PROF_LU_GEMM, s, fl, by);
            gemm<R>(s, false, rest, w, kb, mone, A + k1 + k0 * lda, lda, sA, A12, lda, sA, one,
                    A + k1 + c0 * lda, lda, sA, batch, nullptr, 0, tile, true);
        };
        if (rest > 0) {
            if (!la) {
                update(k1, rest);
            } else {
                const int64_t w1 = std::min<int64_t>(PB, rest);
                update(k1, w1);                       // the next panel's columns
                NLF_HIP(hipEventRecord(aux->next_ready, s));
                NLF_HIP(hipStreamWaitEvent(sp, aux->next_ready, 0));
                if (rest > w1) update(k1 + w1, rest - w1);
            }
        }
    }
}

int64_t getrf_tmp_elems(int64_t n) { return LU_PANEL_NB * std::max<int64_t>(n - LU_PANEL_NB, 1); }

template <typename R>
void getrf(hipStream_t s, int64_t n, int batch, Cx<R>* A, int64_t lda, int64_t sA,
           int32_t* ipiv, int32_t* perm, int32_t* info, int32_t* scratch, Cx<R>* dinv, Cx<R>* tmp,
           const LuAux* aux) {
    if (n <= 0 || batch <= 0) return;
    NLF_REQUIRE(n <= 8192, 1, "getrf: n > 8192 not supported");
    fill_i32(s, info, batch, 0);
    if (dinv && tmp)
        getrf_blocked<R>(s, n, batch, A, lda, sA, ipiv, info, scratch, dinv, tmp, aux);
    else
        getrf_rec<R>(s, n, batch, A, lda, sA, 0, n, ipiv, info, scratch);
    if (perm) {
        hipLaunchKernelGGL(perm_kernel, dim3(batch), dim3(1024), (size_t)n * sizeof(int), s, n,
                           (const int32_t*)ipiv, perm);
        NLF_HIP(hipGetLastError());
    }
}

template <typename R>
void getrs(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
           int64_t sA, const int32_t* perm, const Cx<R>* B, int64_t ldb, int64_t sB, Cx<R>* X,
           int64_t ldx, int64_t sX) {
    if (n <= 0 || nrhs <= 0 || batch <= 0) return;
    {
        ProfScope ps(trsm_class(), s, 0, 2.0 * n * nrhs * sizeof(Cx<R>) * batch);
        const int64_t total = n * nrhs;
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(total, 256), 2048), batch);
        hipLaunchKernelGGL((gather_rows_kernel<R>), grid, dim3(256), 0, s, n, (int64_t)nrhs,
                           perm, B, ldb, sB, X, ldx, sX);
        NLF_HIP(hipGetLastError());
    }
    trsm_lower_unit<R>(s, n, nrhs, batch, LU, lda, sA, X, ldx, sX);
    trsm_upper<R>(s, n, nrhs, batch, LU, lda, sA, X, ldx, sX);
}

int64_t lu_inverse_elems(int64_t n) {
    const int64_t nblk = ceil_div(n, LU_INV_NB);
    return nblk * 2 * LU_INV_NB * LU_INV_NB;
}

// Explicit inverses of the LU_INV_NB x LU_INV_NB diagonal blocks of L (unit lower) and U, per
// matrix: block b of matrix q holds L_bb^{-1} at dinv + q * lu_inverse_elems(n) + 2 b NB^2 and
// U_bb^{-1} NB^2 further, each NB x NB with leading dimension NB.  Solved as L_bb X = I and
// U_bb X = I with the recursive triangular solves, batched over the matrices.
template <typename R>
void lu_block_inverses(hipStream_t s, int64_t n, int batch, const Cx<R>* LU, int64_t lda,
                       int64_t sA, Cx<R>* dinv) {
    const int64_t NB = LU_INV_NB, nblk = ceil_div(n, NB), per = lu_inverse_elems(n);
    {
        const int64_t total = NB * NB * 2 * nblk * batch;
        hipLaunchKernelGGL((identity_blocks_kernel<R>), dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)),
                           dim3(256), 0, s, NB, NB, 2 * nblk * batch, NB * NB, dinv);
        NLF_HIP(hipGetLastError());
    }
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t s0 = b * NB, sb = std::min<int64_t>(NB, n - s0);
        const Cx<R>* D = LU + s0 + s0 * lda;
        trsm_lower_unit<R>(s, sb, sb, batch, D, lda, sA, dinv + 2 * b * NB * NB, NB, per);
        trsm_upper<R>(s, sb, sb, batch, D, lda, sA, dinv + (2 * b + 1) * NB * NB, NB, per);
    }
}

// X_b = A_b^{-1} B_b with the block inverses: forward substitution X_i = Linv_i X_i followed by
// the update of the rows below (right-looking), then the same upwards with U.  Every step is a
// batched MFMA GEMM; tmp holds NB x nrhs per matrix.  The rows outside a chunk of
// LU_SOLVE_CHUNK diagonal blocks are updated once per chunk, with a reduction of
// LU_SOLVE_CHUNK NB (the longer reduction keeps the matrix cores busier than one update per
// block: measured on one box at n = 8192, 160 right-hand sides, 24 nodes, 35.5 ms per
// iteration's solves with chunks of two blocks, 34.7 ms with four); the rows inside the chunk
// are updated block by block.
constexpr int64_t LU_SOLVE_CHUNK = 4;

template <typename R>
void getrs_inv(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
               int64_t sA, const int32_t* perm, const Cx<R>* dinv, const Cx<R>* B, int64_t ldb,
               int64_t sB, Cx<R>* X, int64_t ldx, int64_t sX, Cx<R>* tmp) {
    if (n <= 0 || nrhs <= 0 || batch <= 0) return;
    const int64_t NB = LU_INV_NB, nblk = ceil_div(n, NB), per = lu_inverse_elems(n);
    const int64_t st = NB * nrhs;
    const Cx<R> one(1, 0), mone(-1, 0), zero(0, 0);
    {
        ProfScope ps(trsm_class(), s, 0, 2.0 * n * nrhs * sizeof(Cx<R>) * batch);
        const int64_t total = n * nrhs;
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(total, 256), 2048), batch);
        hipLaunchKernelGGL((gather_rows_kernel<R>), grid, dim3(256), 0, s, n, (int64_t)nrhs, perm, B,
                           ldb, sB, X, ldx, sX);
        NLF_HIP(hipGetLastError());
    }
    auto solve_block = [&](int64_t b, bool upper) {
        const int64_t s0 = b * NB, sb = std::min<int64_t>(NB, n - s0);
        const Cx<R>* Dinv = dinv + (2 * b + (upper ? 1 : 0)) * NB * NB;
        ProfScope ps(trsm_class(), s, 8.0 * sb * sb * nrhs * batch, 0);
        gemm<R>(s, false, sb, nrhs, sb, one, Dinv, NB, per, X + s0, ldx, sX, zero, tmp, NB, st, batch);
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(sb * nrhs, 256), 1024), batch);
        hipLaunchKernelGGL((copy_batched_kernel<R>), grid, dim3(256), 0, s, sb, (int64_t)nrhs,
                           (const Cx<R>*)tmp, NB, st, X + s0, ldx, sX);
        NLF_HIP(hipGetLastError());
    };
    // X[r0:r1] -= A[r0:r1, k0:k1] X[k0:k1] (A = the stored L or U)
    auto update = [&](int64_t r0, int64_t r1, int64_t k0, int64_t k1) {
        if (r1 <= r0 || k1 <= k0) return;
        ProfScope ps(trsm_class(), s, 8.0 * (r1 - r0) * nrhs * (k1 - k0) * batch, 0);
        gemm<R>(s, false, r1 - r0, nrhs, k1 - k0, mone, LU + r0 + k0 * lda, lda, sA, X + k0, ldx, sX, one,
                X + r0, ldx, sX, batch);
    };
    for (int64_t c0 = 0; c0 < nblk; c0 += LU_SOLVE_CHUNK) {          // L, downwards
        const int64_t c1 = std::min(nblk, c0 + LU_SOLVE_CHUNK), e = std::min(n, c1 * NB);
        for (int64_t b = c0; b < c1; ++b) {
            solve_block(b, false);
            update((b + 1) * NB, e, b * NB, std::min(n, (b + 1) * NB));
        }
        update(e, n, c0 * NB, e);
    }
    for (int64_t c1 = nblk; c1 > 0; c1 -= LU_SOLVE_CHUNK) {           // U, upwards
        const int64_t c0 = std::max<int64_t>(0, c1 - LU_SOLVE_CHUNK), e = std::min(n, c1 * NB);
        for (int64_t b = c1 - 1; b >= c0; --b) {
            solve_block(b, true);
            update(c0 * NB, b * NB, b * NB, std::min(n, (b + 1) * NB));
        }
        update(0, c0 * NB, c0 * NB, e);
    }
}

// X_b = A_b^{-H} B_b with the factors P A = L U and the block inverses: A^H = U^H L^H P, so
// U^H V = B is solved forwards block by block (V_q = (U_qq^{-1})^H V_q, then the rows below
// lose (U_{q, below})^H V_q), L^H W = V backwards (W_q = (L_qq^{-1})^H W_q, the rows above
// lose (L_{q, above})^H W_q), and X = P^T W.  Every step is a batched MFMA GEMM on the
// conjugate transpose of a stored block.  Z (n x nrhs per matrix, ld n, stride n * nrhs) holds
// B and then W; Z == B (same strides) skips the copy; X must not overlap Z.
template <typename R>
void getrs_inv_adjoint(hipStream_t s, int64_t n, int nrhs, int batch, const Cx<R>* LU, int64_t lda,
                       int64_t sA, const int32_t* perm, const Cx<R>* dinv, const Cx<R>* B, int64_t ldb,
                       int64_t sB, Cx<R>* Z, Cx<R>* X, int64_t ldx, int64_t sX, Cx<R>* tmp) {
    if (n <= 0 || nrhs <= 0 || batch <= 0) return;
    const int64_t NB = LU_INV_NB, nblk = ceil_div(n, NB), per = lu_inverse_elems(n);
    const int64_t st = NB * nrhs, sZ = n * nrhs;
    const Cx<R> one(1, 0), mone(-1, 0), zero(0, 0);
    if (B != Z || ldb != n || sB != sZ) {
        ProfScope ps(trsm_class(), s, 0, 2.0 * n * nrhs * sizeof(Cx<R>) * batch);
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(n * nrhs, 256), 2048), batch);
        hipLaunchKernelGGL((copy_batched_kernel<R>), grid, dim3(256), 0, s, n, (int64_t)nrhs, B, ldb, sB, Z, n, sZ);
        NLF_HIP(hipGetLastError());
    }
    auto solve_block = [&](int64_t b, bool upper) {   // Z_b <- (D_bb^{-1})^H Z_b
        const int64_t s0 = b * NB, sb = std::min<int64_t>(NB, n - s0);
        const Cx<R>* Dinv = dinv + (2 * b + (upper ? 1 : 0)) * NB * NB;
        ProfScope ps(trsm_class(), s, 8.0 * sb * sb * nrhs * batch, 0);
        gemm<R>(s, true, sb, nrhs, sb, one, Dinv, NB, per, Z + s0, n, sZ, zero, tmp, NB, st, batch);
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(sb * nrhs, 256), 1024), batch);
        hipLaunchKernelGGL((copy_batched_kernel<R>), grid, dim3(256), 0, s, sb, (int64_t)nrhs,
                           (const Cx<R>*)tmp, NB, st, Z + s0, n, sZ);
        NLF_HIP(hipGetLastError());
    };
    // Z[r0:r1] -= (A[k0:k1, r0:r1])^H Z[k0:k1], A the stored U (above the diagonal) or L (below)
    auto update = [&](int64_t r0, int64_t r1, int64_t k0, int64_t k1) {
        if (r1 <= r0 || k1 <= k0) return;
        ProfScope ps(trsm_class(), s, 8.0 * (r1 - r0) * nrhs * (k1 - k0) * batch, 0);
        gemm<R>(s, true, r1 - r0, nrhs, k1 - k0, mone, LU + k0 + r0 * lda, lda, sA, Z + k0, n, sZ, one, Z + r0, n,
                sZ, batch);
    };
    // chunks of LU_SOLVE_CHUNK diagonal blocks, as in getrs_inv
    for (int64_t c0 = 0; c0 < nblk; c0 += LU_SOLVE_CHUNK) {          // U^H V = B, forwards
        const int64_t c1 = std::min(nblk, c0 + LU_SOLVE_CHUNK), e = std::min(n, c1 * NB);
        for (int64_t b = c0; b < c1; ++b) {
            solve_block(b, true);
            update((b + 1) * NB, e, b * NB, std::min(n, (b + 1) * NB));
        }
        update(e, n, c0 * NB, e);
    }
    for (int64_t c1 = nblk; c1 > 0; c1 -= LU_SOLVE_CHUNK) {           // L^H W = V, backwards
        const int64_t c0 = std::max<int64_t>(0, c1 - LU_SOLVE_CHUNK), e = std::min(n, c1 * NB);
        for (int64_t b = c1 - 1; b >= c0; --b) {
            solve_block(b, false);
            update(c0 * NB, b * NB, b * NB, std::min(n, (b + 1) * NB));
        }
        update(0, c0 * NB, c0 * NB, e);
    }
    {
        ProfScope ps(trsm_class(), s, 0, 2.0 * n * nrhs * sizeof(Cx<R>) * batch);
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(n * nrhs, 256), 2048), batch);
        hipLaunchKernelGGL((scatter_rows_kernel<R>), grid, dim3(256), 0, s, n, (int64_t)nrhs, perm,
                           (const Cx<R>*)Z, n, sZ, X, ldx, sX);
        NLF_HIP(hipGetLastError());
    }
}

template void getrs_inv_adjoint<double>(hipStream_t, int64_t, int, int, const Cx<double>*, int64_t, int64_t,
                                        const int32_t*, const Cx<double>*, const Cx<double>*, int64_t, int64_t,
                                        Cx<double>*, Cx<double>*, int64_t, int64_t, Cx<double>*);
template void getrs_inv_adjoint<float>(hipStream_t, int64_t, int, int, const Cx<float>*, int64_t, int64_t,
                                       const int32_t*, const Cx<float>*, const Cx<float>*, int64_t, int64_t,
                                       Cx<float>*, Cx<float>*, int64_t, int64_t, Cx<float>*);

template void lu_block_inverses<double>(hipStream_t, int64_t, int, const Cx<double>*, int64_t, int64_t,
                                        Cx<double>*);
template void lu_block_inverses<float>(hipStream_t, int64_t, int, const Cx<float>*, int64_t, int64_t,
                                       Cx<float>*);
template void getrs_inv<double>(hipStream_t, int64_t, int, int, const Cx<double>*, int64_t, int64_t,
                                const int32_t*, const Cx<double>*, const Cx<double>*, int64_t, int64_t,
                                Cx<double>*, int64_t, int64_t, Cx<double>*);
template void getrs_inv<float>(hipStream_t, int64_t, int, int, const Cx<float>*, int64_t, int64_t,
                               const int32_t*, const Cx<float>*, const Cx<float>*, int64_t, int64_t,
                               Cx<float>*, int64_t, int64_t, Cx<float>*);

template void getrf<double>(hipStream_t, int64_t, int, Cx<double>*, int64_t, int64_t, int32_t*,
                            int32_t*, int32_t*, int32_t*, Cx<double>*, Cx<double>*, const LuAux*);
template void getrf<float>(hipStream_t, int64_t, int, Cx<float>*, int64_t, int64_t, int32_t*,
                           int32_t*, int32_t*, int32_t*, Cx<float>*, Cx<float>*, const LuAux*);
template void getrs<double>(hipStream_t, int64_t, int, int, const Cx<double>*, int64_t, int64_t,
                            const int32_t*, const Cx<double>*, int64_t, int64_t, Cx<double>*,
                            int64_t, int64_t);
template void getrs<float>(hipStream_t, int64_t, int, int, const Cx<float>*, int64_t, int64_t,
                           const int32_t*, const Cx<float>*, int64_t, int64_t, Cx<float>*,
                           int64_t, int64_t);
template void trsm_lower_unit<double>(hipStream_t, int64_t, int64_t, int, const Cx<double>*,
                                      int64_t, int64_t, Cx<double>*, int64_t, int64_t);
template void trsm_lower_unit<float>(hipStream_t, int64_t, int64_t, int, const Cx<float>*,
                                     int64_t, int64_t, Cx<float>*, int64_t, int64_t);
template void trsm_upper<double>(hipStream_t, int64_t, int64_t, int, const Cx<double>*, int64_t,
                                 int64_t, Cx<double>*, int64_t, int64_t);
template void trsm_upper<float>(hipStream_t, int64_t, int64_t, int, const Cx<float>*, int64_t,
                                int64_t, Cx<float>*, int64_t, int64_t);

}  // namespace nlf
