/*
 * nlfeast.h -- C ABI of the MI355X (gfx950) nonlinear FEAST library.
 *
 * Computes the eigenpairs (lambda, x) of T(lambda) x = 0 whose eigenvalues lie inside one
 * or more closed contours in the complex plane (Gavin, Miedlar, Polizzi, "FEAST Eigensolver
 * for Nonlinear Eigenvalue Problems", arXiv 1801.09794: problem statement in Sec. 1 eq. nlevp
 * and Sec. 2 eq. NLEVP; the method is Algorithm 1 of Sec. 4.2), with
 *
 *     T(lambda) = sum_j f_j(lambda) A_j,   f_j(lambda) = lambda^p,  exp(-tau lambda)  or a
 *                                          scalar function supplied by the caller
 *
 * (polynomial form of Sec. 2 eq. polynomialeig; non-polynomial form named in Sec. 6).
 *
 * Conventions for every entry point below
 *   - complex numbers are stored as interleaved (re, im) pairs: "c128" = two doubles,
 *     "c64" = two floats;
 *   - matrices are column-major with a leading dimension ld >= rows: element (i, j) of a
 *     matrix at p is p[i + j * ld];
 *   - a "batch" of matrices is `batch` matrices at p + b * stride (elements), b = 0..batch-1;
 *   - pointers named *_dev are device (HBM) pointers on the device the call runs on; all
 *     other pointers are host pointers; device memory passed in is owned by the caller and
 *     only borrowed for the duration of the call (A_j: until the next set_coeffs/destroy);
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream); calls enqueue
 *     on it and, unless stated otherwise, return before the device work finishes;
 *   - no call throws; every call returns an nlfeast_status; NLF_ERR_ARG is returned, before
 *     any device work is enqueued, for null pointers, negative sizes or ld < rows.
 */
#ifndef NLFEAST_H
#define NLFEAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NLF_OK = 0,
    NLF_ERR_ARG = 1,             /* invalid argument (checked on the host before any launch) */
    NLF_ERR_NOMEM = 2,           /* workspace too small, or a host allocation failed */
    NLF_ERR_DEVICE = 3,          /* a HIP runtime call failed; see nlfeast_last_error */
    NLF_ERR_STATE = 4,           /* call out of order (e.g. solve before set_contour) */
    NLF_ERR_SINGULAR = 5,        /* exact zero pivot: a quadrature node sits on an eigenvalue */
    NLF_ERR_M0_TOO_SMALL = 6,    /* m0 or more Ritz values inside a contour (Algorithm 1
                                    requires fewer than m0 eigenvalues inside C) */
    NLF_ERR_NOT_CONVERGED = 7,   /* max_iter reached; outputs hold the last iterate */
    NLF_SPURIOUS = 8             /* not an error: every eigenpair inside converged, and some
                                    Ritz values inside were identified as spurious (Sec. 4.2:
                                    Ritz pairs that match no eigenpair of the full problem);
                                    they are flagged with inside_out = 2 */
} nlfeast_status;

typedef enum {
    NLF_F_POW = 0,               /* f(lambda) = lambda^p, param = p (integer 0..16) */
    NLF_F_EXP = 1,               /* f(lambda) = exp(-tau lambda), param = tau */
    NLF_F_USER = 2               /* f given by the caller's nlfeast_user_fn (set with
                                    nlfeast_set_user_function), which receives the term's
                                    position j and param */
} nlfeast_fkind;

/* A caller-supplied scalar function f of a term of kind NLF_F_USER (Sec. 6: T(lambda) of any
 * form).  For the term at position `term` with parameter `param`, writes f(z_i) to
 * f[2i], f[2i+1] and, when df is not NULL, f'(z_i) to df[2i], df[2i+1], for the `count` points
 * z_i = z[2i] + i z[2i+1].  f must be analytic inside the contour enlarged 1.5 times (the
 * reduced problem is solved on that enlarged ellipse) and on the contour's nodes.  Returns 0;
 * any other value makes the computation that asked fail with NLF_ERR_ARG.  The library calls
 * it from the calling thread and from its own host threads, possibly at the same time: it must
 * be safe to call concurrently. */
typedef int32_t (*nlfeast_user_fn)(void* user, int32_t term, double param, int64_t count,
                                   const double* z, double* f, double* df);

typedef enum {
    NLF_PREC_FP64 = 0,           /* LU and triangular solves in complex128 */
    NLF_PREC_FP32_REFINE = 1     /* LU and triangular solves in complex64 with FP32
                                    accumulation, FP64 iterative refinement of each solve;
                                    residuals, orthonormalisation, projections and the
                                    reduced problem stay in FP64 */
} nlfeast_precision;

typedef enum {
    NLF_QUAD_GAUSS_LEGENDRE = 0, /* Gauss-Legendre on the contour parameter [0, 2 pi] */
    NLF_QUAD_TRAPEZOID = 1       /* theta_k = 2 pi (k + 1/2) / n_c */
} nlfeast_quad;

typedef enum { NLF_C64 = 0, NLF_C128 = 1 } nlfeast_dtype;

typedef struct {
    double tol;                  /* Step 3 threshold on ||T(lambda_i) x_i||_2, ||x_i||_2 = 1 */
    int32_t max_iter;            /* cap on Step 4 executions (default 50) */
    int32_t precision;           /* nlfeast_precision */
    int32_t max_refine;          /* FP32_REFINE: refinement sweeps per solve, at most 5 */
    double refine_eta;           /* FP32_REFINE: stop sweeps once ||E_k||_F <= eta ||R||_F for
                                    every node; once the first check of an iteration passes,
                                    later iterations of that region skip the check */
    uint64_t seed;               /* X0 when the caller passes none (counter-based normal draws) */
    int32_t autotune;            /* 1: on first use of a (precision, n, node count) shape, time
                                    trial factorisations over panel width, trailing-update GEMM
                                    tile and stream groups, and keep the fastest (process-wide
                                    cache); explicit lu_streams / panel_width then act as fixed */
    int32_t verbose;             /* 1: one line per iteration on stderr */
    int32_t lu_streams;          /* factor the node matrices in this many groups on separate
                                    streams (1..4; 0 = default, one stream), so that one group's
                                    panel factorisations overlap another group's GEMMs */
    int32_t panel_width;         /* columns per single-workgroup panel of the LU, 4..32 (0 = 32) */
    int32_t region_streams;      /* 0 (default): with several regions, each region's iteration
                                    runs on its own stream and host thread after the shared
                                    factorisation; 1: regions one after another on the caller's
                                    stream */
    int32_t graph;               /* 1: capture assembly + batched factorisation of all nodes in
                                    hipGraphs on first use and replay them on later solves with
                                    the same shapes, coefficient pointers and workspace.  With one
                                    node group and no look-ahead the capture is cut at the
                                    trailing updates, which run eagerly between the graph segments
                                    and stay timed (NLF_K_LU_GEMM); the other kernels of the
                                    factorisation are then profiled only through NLF_K_FACTOR */
    int32_t lookahead;           /* blocked LU: 1 = factor panel k+1 on a second stream while
                                    the trailing update of panel k runs; -1 = one stream;
                                    0 = library default (one stream).  1 together with
                                    lu_streams > 1 is refused (NLF_ERR_ARG) */
    int32_t reduced_solver;      /* Steps 1-2 (Sec. 4.2: the projected problem may be solved by
                                    any suitable method).  Non-polynomial T: 0 (default) or 1 =
                                    the contour-integral solve (moments of the reduced resolvent
                                    on the contour enlarged 1.5 times, formed on the device; block
                                    Hankel matrices, Newton refinement); 2 = Taylor linearisation
                                    about the contour centre and Newton refinement (NLF_F_EXP
                                    terms).  Polynomial T: the exact companion linearisation for
                                    0..2; 3 = the contour-integral solve for every problem (for
                                    polynomial problems cheaper than the companion matrix of order
                                    degree x m0 once m0 reaches ~100, but it needs the enlarged
                                    contour to hold fewer than 3 m0 eigenvalues of the reduced
                                    problem).  Problems with an NLF_F_USER term always take the
                                    contour-integral solve */
} nlfeast_options;

typedef struct nlfeast_ctx* nlfeast_handle;

/* Library mechanics, not a step of the paper's method: a library-owned context for problems
 * of size n (the order of T(lambda), Sec. 1 eq. nlevp) on HIP device `device`, enqueuing on
 * `stream`.  The handle owns only host state, small device arrays (quadrature book-keeping) and
 * its own streams and events; all large device memory is the caller's workspace.  Host threads
 * it starts during a solve are joined before the solve returns.  Errors: NLF_ERR_ARG for
 * n outside 1..8192 or a bad device index. */
nlfeast_status nlfeast_create(nlfeast_handle* h, int64_t n, int device, void* stream);

/* The coefficients of T (Sec. 2 eq. polynomialeig; Sec. 4.2 block residual): J terms, term j
 * is fkind[j] with parameter fparam[j] times the c128 n x n matrix A_dev[j] (leading
 * dimension lda).  The A_j are borrowed, not copied.  Invalidates cached factorisations. */
nlfeast_status nlfeast_set_coeffs(nlfeast_handle h, int32_t J, const int32_t* fkind,
                                  const double* fparam, const void* const* A_dev, int64_t lda);

/* The function evaluated for every term of kind NLF_F_USER (see nlfeast_user_fn), with the
 * caller's `user` pointer passed back unchanged; both stay borrowed until replaced or the
 * handle is destroyed.  A solve with an NLF_F_USER term and no function returns NLF_ERR_STATE.
 * Invalidates cached factorisations. */
nlfeast_status nlfeast_set_user_function(nlfeast_handle h, nlfeast_user_fn fn, void* user);

/* nreg disjoint regions (Sec. 1 and Sec. 3: independent subregions of the plane).  Region r is
 * the axis-aligned ellipse with centre (centre[2r] + i centre[2r+1]) and semi-axes
 * semi_axes[2r] (real direction), semi_axes[2r+1] (imaginary direction) -- a circle when they
 * are equal -- with n_nodes[r] quadrature nodes (Algorithm 1 inputs) and subspace size m0[r].
 * Invalidates cached factorisations. */
nlfeast_status nlfeast_set_contour(nlfeast_handle h, int32_t nreg, const double* centre,
                                   const double* semi_axes, const int32_t* n_nodes,
                                   const int32_t* m0, int32_t quad_rule);

/* Library mechanics: the device workspace bytes that nlfeast_solve (or nlfeast_solve_left) needs
 * for these options, the coefficients and the contours (the node factors of T(z_k), Algorithm 1
 * Step 4, dominate: n^2 per node in the LU precision, plus n^2 complex128 per node in the FP32 +
 * refinement form).  NLF_ERR_STATE before set_coeffs / set_contour. */
nlfeast_status nlfeast_workspace_size(nlfeast_handle h, const nlfeast_options* opt, size_t* bytes);

/* Algorithm 1 for every region.  Blocks until the outputs are valid.
 *   ws_dev, ws_bytes   caller-owned device workspace (>= nlfeast_workspace_size)
 *   X0_dev             c128 n x sum(m0) initial blocks, region by region (ld n), or NULL for
 *                      seeded random blocks
 *   X_dev_out          c128 n x sum(m0): the Ritz vectors (unit 2-norm), region by region
 *   lambda_out         2 * sum(m0) doubles: the Ritz values (re, im), selection order
 *   resid_out          sum(m0) doubles: ||T(lambda_i) x_i||_2
 *   inside_out         sum(m0) int32: 0 outside its contour, 1 strictly inside, 2 strictly
 *                      inside and identified as a spurious Ritz value (see below)
 *   m_out, iters_out   per region: converged eigenpairs inside (resid <= tol), Step 4
 *                      executions
 * Step 3 stops a region when every Ritz value inside has converged.  Spurious Ritz values
 * (Sec. 4.2) are identified by their residuals: from iteration 2 on, each Ritz value is paired
 * with the nearest unpaired one of the previous iteration (nearest pairs first), and an
 * unconverged value inside is stagnant when its residual exceeds theta times its partner's,
 * theta = min(0.97, max(0.25, (rho_min / |rho(lambda)|)^(1/3))), where
 * rho(l) = sum_k omega_k / (z_k - l) is the quadrature filter and rho_min its smallest modulus
 * over the selected Ritz values (a genuine pair's residual falls by about that filter ratio per
 * iteration).  When at least one pair inside has converged and every other value inside is
 * stagnant, the region stops, those values are returned with inside_out = 2 and the status is
 * NLF_SPURIOUS.
 * Factorisations of T(z_k) are cached in the workspace and reused by the next solve with the
 * same handle, coefficients, contours, precision and workspace pointer.
 * Returns NLF_OK, NLF_SPURIOUS, NLF_ERR_NOT_CONVERGED, NLF_ERR_M0_TOO_SMALL or NLF_ERR_SINGULAR
 * (with several regions: a hard error first, then NOT_CONVERGED / M0_TOO_SMALL, then
 * NLF_SPURIOUS). */
nlfeast_status nlfeast_solve(nlfeast_handle h, const nlfeast_options* opt, void* ws_dev,
                             size_t ws_bytes, const void* X0_dev, void* X_dev_out,
                             double* lambda_out, double* resid_out, int32_t* inside_out,
                             int32_t* m_out, int32_t* iters_out);

/* Left eigenvectors (Sec. 2 eq. NLEVP: y^* T(lambda) = 0; (lambda, x, y) an eigentriple):
 * Algorithm 1 applied to the adjoint function S(mu) = T(conj mu)^H = sum_j conj(f_j(conj mu))
 * A_j^H on the conjugate of every contour, whose eigenpairs (conj lambda, y) are the left
 * eigenpairs of T.  The quadrature nodes of the conjugate contour are conj z_k with weights
 * conj omega_k, and S(conj z_k) = T(z_k)^H, so the cached LU factors of T(z_k) serve through
 * adjoint triangular solves (U^H, then L^H, then the row permutation); the factorisation is
 * done here first when no valid one is cached.  Arguments and statuses as nlfeast_solve, with
 * Y0_dev the initial blocks (or NULL), Y_dev_out the left eigenvectors y (unit 2-norm),
 * lambda_out the eigenvalues of T (conjugated back, so they match nlfeast_solve's), resid_out
 * ||T(lambda_i)^H y_i||_2 and inside_out relative to the caller's contours. */
nlfeast_status nlfeast_solve_left(nlfeast_handle h, const nlfeast_options* opt, void* ws_dev,
                                  size_t ws_bytes, const void* Y0_dev, void* Y_dev_out,
                                  double* lambda_out, double* resid_out, int32_t* inside_out,
                                  int32_t* m_out, int32_t* iters_out);

/* Per-kernel-class device time of the last solve, measured with HIP events on the solve's
 * stream when profiling is on (nlfeast_set_profiling).  For class c (see nlfeast_kernel_class):
 * launches[c], milliseconds[c], and the algorithmic flops[c] / bytes[c] of those launches. */
typedef enum {
    NLF_K_ASSEMBLE = 0, NLF_K_LU_GEMM = 1, NLF_K_LU_PANEL = 2, NLF_K_LU_TRSM = 3,
    NLF_K_LU_LASWP = 4, NLF_K_SOLVE = 5, NLF_K_REFINE = 6, NLF_K_RESIDUAL = 7,
    NLF_K_ACCUMULATE = 8, NLF_K_ORTH = 9, NLF_K_PROJECT = 10, NLF_K_HOST_REDUCED = 11,
    NLF_K_FACTOR = 12,           /* wall span of assembly + factorisation of all nodes on the
                                    solve stream (eager launches or one graph replay) */
    NLF_K_AUTOTUNE = 13,         /* trial factorisations of the LU tuner (first use of a shape) */
    NLF_K_LU_REC_GEMM = 14,      /* GEMM updates inside the recursive panel factorisation
                                    (NLF_K_LU_GEMM: the rank-512 trailing updates of the blocked
                                    LU, kernel symbols lu_update_dma_kernel and
                                    lu_update_dma32_kernel, or lu_update_kernel where the
                                    direct-to-LDS form does not apply) */
    NLF_K_REDUCED = 15,          /* device part of the contour-integral reduced solve: the reduced
                                    matrices at the enlarged contour's points, their batched LU
                                    and inverses, and the moment sums */
    NLF_K_COUNT = 16
} nlfeast_kernel_class;
nlfeast_status nlfeast_set_profiling(nlfeast_handle h, int32_t on);
nlfeast_status nlfeast_get_profile(nlfeast_handle h, int64_t* launches, double* milliseconds,
                                   double* flops, double* bytes);

/* Library mechanics: the message of the last failed call on h (or, with h = NULL, of the last
 * failed call without a handle on this thread); valid until the next call. */
const char* nlfeast_last_error(nlfeast_handle h);
/* Library mechanics: releases the handle, its streams and events (after the work it enqueued has
 * been synchronised by the caller); caller-owned memory is untouched.  NULL is a no-op. */
void nlfeast_destroy(nlfeast_handle h);

/* ------------------------------------------------------------------------------------------
 * Step-level entry points: each performs one step of Algorithm 1's hot path on caller-owned
 * device buffers, enqueued on `stream` (asynchronous).  The solver above is built from the
 * same kernels.  Unlike the solver, some of these allocate small temporary device memory on
 * the stream for the duration of the call (hipMallocAsync / hipFreeAsync: nlf_assemble its
 * coefficient table, nlf_getrf_batched and nlf_getrf_batched_blocked their row-exchange lists and
 * staging, nlf_block_residual a diagonal m x m block per term, nlf_accumulate its coefficient
 * table).
 * nlf_getrf_batched_noalloc is the variant that allocates nothing.
 * ---------------------------------------------------------------------------------------- */

/* T(z_k) = sum_j f_j(z_k) A_j for k = 0..nz-1 (the matrices whose inverses Step 4 applies).
 * A_dev[j]: c128 n x n (lda).  z: 2*nz doubles (host).  Outputs: T64_dev (c128, may be NULL)
 * and/or T32_dev (c64, rounded once from the FP64 sum, may be NULL), each a batch of nz n x n
 * matrices with leading dimension ldt and stride strideT.  Term kinds NLF_F_POW and NLF_F_EXP
 * only (NLF_ERR_ARG otherwise: caller-supplied functions belong to a handle). */
nlfeast_status nlf_assemble(int64_t n, int32_t J, const int32_t* fkind, const double* fparam,
                            const void* const* A_dev, int64_t lda, int32_t nz, const double* z,
                            void* T64_dev, void* T32_dev, int64_t ldt, int64_t strideT,
                            void* stream);

/* In-place LU with partial pivoting of a batch of n x n matrices (dtype c128 or c64):
 * P_b A_b = L_b U_b, unit-lower L below the diagonal, U on and above it (the factorisation
 * that makes each multiplication by T^{-1}(z_j) in Step 4 a pair of triangular solves).
 * The pivot of column k is the entry of largest |Re| + |Im| on or below the diagonal (first
 * on ties).  ipiv_dev: int32 batch x n, ipiv[b*n + k] = 0-based row exchanged with row k.
 * perm_dev (int32 batch x n, may be NULL): the composed permutation, (P A)[i] = A[perm[i]].
 * info_dev (int32 batch): 0, or k+1 for the first exact zero pivot U(k,k) = 0.
 * Blocked recursively; trailing updates are complex GEMMs on MFMA. */
nlfeast_status nlf_getrf_batched(int32_t dtype, int64_t n, int32_t batch, void* A_dev,
                                 int64_t lda, int64_t strideA, int32_t* ipiv_dev,
                                 int32_t* perm_dev, int32_t* info_dev, void* stream);

/* The same factorisation computed right-looking with 512-column panels (each panel factored as
 * above; U12 = L11^{-1} A12 by GEMMs with the explicit inverses of the panel's 256 x 256
 * diagonal blocks; rank-512 trailing updates on MFMA); it also writes the diagonal-block
 * inverses that nlf_lu_block_inverses would (dinv_dev: batch * nlf_lu_inverse_elems(n)
 * elements).  Temporary device memory of 512 * max(n - 512, 1) elements per matrix is
 * allocated on the stream for the call. */
nlfeast_status nlf_getrf_batched_blocked(int32_t dtype, int64_t n, int32_t batch, void* A_dev,
                                         int64_t lda, int64_t strideA, int32_t* ipiv_dev,
                                         int32_t* perm_dev, int32_t* info_dev, void* dinv_dev,
                                         void* stream);

/* Allocation-free variant of nlf_getrf_batched, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, factorisation, pivots and statuses; the row-exchange lists that
 * nlf_getrf_batched allocates per call live in a fixed device array of
 * NLF_NOALLOC_SCRATCH_INTS int32 (4 MiB) per GPU, held until the process ends.  Needs
 * 4 * n * batch <= NLF_NOALLOC_SCRATCH_INTS (n * batch <= 262144, e.g. n = 8192 with 32
 * matrices); larger calls return NLF_ERR_ARG before any launch.  Calls no hipMalloc/hipFree.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Nothing in the array carries from
 * one call to the next (each call writes every entry it reads). */
#define NLF_NOALLOC_SCRATCH_INTS (1 << 20)
nlfeast_status nlf_getrf_batched_noalloc(int32_t dtype, int64_t n, int32_t batch, void* A_dev,
                                         int64_t lda, int64_t strideA, int32_t* ipiv_dev,
                                         int32_t* perm_dev, int32_t* info_dev, void* stream);

/* X_b = A_b^{-1} B_b from nlf_getrf_batched factors (same dtype), nrhs columns.  B_dev
 * (ldb, strideB; strideB = 0 shares one right-hand side across the batch) is read, X_dev
 * (ldx, strideX) is written and must not overlap B.  perm_dev is the composed permutation
 * written by nlf_getrf_batched.  Forward substitution with unit L, then back substitution
 * with U, both blocked recursively with complex GEMMs on MFMA. */
nlfeast_status nlf_getrs_batched(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                 const void* LU_dev, int64_t lda, int64_t strideA,
                                 const int32_t* perm_dev, const void* B_dev, int64_t ldb,
                                 int64_t strideB, void* X_dev, int64_t ldx, int64_t strideX,
                                 void* stream);

/* Explicit inverses of the 256 x 256 diagonal blocks of the L and U factors written by
 * nlf_getrf_batched (same dtype): per matrix nlf_lu_inverse_elems(n) complex elements at
 * dinv_dev + b * nlf_lu_inverse_elems(n) (block q: L_qq^{-1} then U_qq^{-1}, each 256 x 256,
 * leading dimension 256).  Computed once per factorisation for nlf_getrs_batched_inv. */
int64_t nlf_lu_inverse_elems(int64_t n);
nlfeast_status nlf_lu_block_inverses(int32_t dtype, int64_t n, int32_t batch, const void* LU_dev,
                                     int64_t lda, int64_t strideA, void* dinv_dev, void* stream);

/* As nlf_getrs_batched, with the triangular solves done block by block: X_q = L_qq^{-1} X_q and
 * a rank-256 update of the rows below (then the same upwards with U), every step a batched
 * MFMA GEMM.  dinv_dev from nlf_lu_block_inverses; tmp_dev: 256 * nrhs * batch elements. */
nlfeast_status nlf_getrs_batched_inv(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                     const void* LU_dev, int64_t lda, int64_t strideA,
                                     const int32_t* perm_dev, const void* dinv_dev,
                                     const void* B_dev, int64_t ldb, int64_t strideB, void* X_dev,
                                     int64_t ldx, int64_t strideX, void* tmp_dev, void* stream);

/* As nlf_getrs_batched_inv for the conjugate-transposed matrices: X_b = A_b^{-H} B_b from the
 * same factors and inverses (the solves of the adjoint problem behind nlfeast_solve_left).
 * Z_dev: scratch of the same dtype, n x nrhs per matrix (ld n, stride n * nrhs); it may be B_dev
 * when B has exactly that layout (B is then overwritten); X_dev must not overlap Z_dev
 * (NLF_ERR_ARG). */
nlfeast_status nlf_getrs_batched_inv_adjoint(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                             const void* LU_dev, int64_t lda, int64_t strideA,
                                             const int32_t* perm_dev, const void* dinv_dev,
                                             const void* B_dev, int64_t ldb, int64_t strideB,
                                             void* Z_dev, void* X_dev, int64_t ldx, int64_t strideX,
                                             void* tmp_dev, void* stream);

/* C_b = alpha op(A_b) op(B_b) + beta C_b, complex (dtype c128 or c64), op 'N' or 'C'
 * (conjugate transpose); alpha, beta: 2 doubles each (host).  The MFMA GEMM used by every
 * dense contraction of the path. */
nlfeast_status nlf_gemm_batched(int32_t dtype, char opA, char opB, int64_t M, int64_t N,
                                int64_t K, const double* alpha, const void* A_dev, int64_t lda,
                                int64_t strideA, const void* B_dev, int64_t ldb, int64_t strideB,
                                const double* beta, void* C_dev, int64_t ldc, int64_t strideC,
                                int32_t batch, void* stream);

/* nlf_gemm_batched with an explicit workgroup tile of (32 tm) x (32 tn) complex elements,
 * (tm, tn) in {(1, 1), (2, 1), (2, 2), (4, 2)}, and (4, 1), (4, 4) for c64.  Used by the GEMM autotuner; returns NLF_ERR_ARG
 * for a tile that is not compiled. */
nlfeast_status nlf_gemm_batched_tile(int32_t dtype, char opA, int64_t M, int64_t N, int64_t K,
                                     const double* alpha, const void* A_dev, int64_t lda,
                                     int64_t strideA, const void* B_dev, int64_t ldb,
                                     int64_t strideB, const double* beta, void* C_dev, int64_t ldc,
                                     int64_t strideC, int32_t batch, int32_t tm, int32_t tn,
                                     void* stream);

/* Block residual T(X, Lambda) = sum_j A_j X f_j(Lambda) (Sec. 4.2) and its column 2-norms
 * (the Step 3 quantities).  X_dev: c128 n x m (ldx); lambda: 2*m doubles (host); R_dev: c128
 * n x m (ldr); norms_dev: m doubles (device).  ws_dev: c128 scratch of n * m elements.
 * Term kinds NLF_F_POW and NLF_F_EXP only. */
nlfeast_status nlf_block_residual(int64_t n, int32_t m, int32_t J, const int32_t* fkind,
                                  const double* fparam, const void* const* A_dev, int64_t lda,
                                  const void* X_dev, int64_t ldx, const double* lambda,
                                  void* R_dev, int64_t ldr, double* norms_dev, void* ws_dev,
                                  void* stream);

/* Step 4 accumulation: Q = sum_k omega_k (X - Y_k) (z_k I - Lambda)^{-1}, evaluated as
 * X rho(Lambda) - sum_k omega_k Y_k (z_k I - Lambda)^{-1} with rho(l) = sum_k omega_k/(z_k - l).
 * X_dev, Q_dev: c128 n x m (ld n); Y_dev: nz blocks c128 n x m (ld n, stride n*m);
 * z, omega: 2*nz doubles, lambda: 2*m doubles (host). */
nlfeast_status nlf_accumulate(int64_t n, int32_t m, int32_t nz, const void* X_dev,
                              const void* Y_dev, const double* z, const double* omega,
                              const double* lambda, void* Q_dev, void* stream);

/* Steps 0/5: orthonormalise the columns of the c128 n x m block Q_dev (ld n, m <= n) in
 * place, by Cholesky QR twice (Gram matrix on MFMA, m x m Cholesky on the host); a block whose
 * Gram matrix is numerically singular (Cholesky fails, or a pivot falls below 1e-12 of its
 * diagonal entry) goes through blocked Householder QR on the device instead.  ws_dev: c128
 * scratch of nlf_orth_workspace(n, m) elements.  Blocking (host Cholesky). */
int64_t nlf_orth_workspace(int64_t n, int32_t m);
nlfeast_status nlf_orthonormalize(int64_t n, int32_t m, void* Q_dev, void* ws_dev, void* stream);

/* Step 1 projections: W_j = A_j Q (c128 n x m each, stored side by side in W_dev, ld n) and
 * Ahat_j = Q^H W_j (c128 m x m each, stored in Ahat_dev with ld m, stride m*m).
 * ws_dev: c128 scratch of nlf_project_workspace(n, m, J) elements. */
int64_t nlf_project_workspace(int64_t n, int32_t m, int32_t J);
nlfeast_status nlf_project(int64_t n, int32_t m, int32_t J, const void* const* A_dev,
                           int64_t lda, const void* Q_dev, void* W_dev, void* Ahat_dev,
                           void* ws_dev, void* stream);

/* Contour quadrature (Algorithm 1 inputs): n_c nodes z and weights omega (2*nc doubles each)
 * of the rule `quad_rule` on the ellipse (centre, semi-axes a, b); the weights include
 * 1/(2 pi i), so sum_k omega_k g(z_k) approximates (1/2 pi i) oint g(z) dz. */
nlfeast_status nlf_quadrature(double cre, double cim, double a, double b, int32_t nc,
                              int32_t quad_rule, double* z, double* omega);

/* Step 1/2 on the host (the linearisation route: companion for polynomial terms, Taylor
 * surrogate and Newton for NLF_F_EXP terms): all eigenpairs of the reduced problem
 * sum_j f_j(lambda) Ahat_j y = 0
 * (m x m c128 matrices Ahat, host, ld m, stride m*m) near the ellipse (centre, a, b), of which
 * the m_keep closest to its interior (ascending normalised radius) are returned: lambda_out
 * (2*m_keep doubles) and Y_out (c128 m x m_keep, ld m, unit-norm columns).  The linearisation
 * is inverted about a shift inside the contour: the centre, unless one of the n_avoid values in
 * `avoid` (2*n_avoid doubles, e.g. the previous Ritz values; may be NULL) lies close to it. */
nlfeast_status nlf_reduced_solve(int32_t m, int32_t J, const int32_t* fkind,
                                 const double* fparam, const double* Ahat, double cre,
                                 double cim, double a, double b, int32_t m_keep,
                                 const double* avoid, int32_t n_avoid, double* lambda_out,
                                 double* Y_out);

/* As nlf_reduced_solve, with terms of kind NLF_F_USER evaluated by fn(user, ...) and the
 * choice `method` of nlfeast_options.reduced_solver (0..3).  The contour-integral solve
 * (Sec. 3 eq. cauchymoments applied to the reduced function; taken for NLF_F_USER terms, for
 * any non-polynomial term unless method is 2, and for every problem with method 3; here the
 * moments are formed on the host) needs m_keep <= m: it returns the eigenpairs found
 * inside the contour enlarged 1.5 times, Newton-refined and in ascending normalised radius,
 * followed, when fewer than m_keep were found, by completing pairs (unit vectors orthogonal to
 * those found, with values spread over the enlarged contour); found_out (m_keep int32, may be
 * NULL) receives 1 for a found pair and 0 for a completing one.  fn may be NULL when no term
 * is NLF_F_USER.  Errors: NLF_ERR_ARG (bad arguments, or fn reported a failure),
 * NLF_ERR_DEVICE (a singular reduced matrix on the enlarged contour, or too many eigenvalues
 * inside it to resolve). */
nlfeast_status nlf_reduced_solve_ex(int32_t m, int32_t J, const int32_t* fkind,
                                    const double* fparam, nlfeast_user_fn fn, void* user,
                                    int32_t method, const double* Ahat, double cre, double cim,
                                    double a, double b, int32_t m_keep, const double* avoid,
                                    int32_t n_avoid, double* lambda_out, double* Y_out,
                                    int32_t* found_out);

#ifdef __cplusplus
}
#endif

#endif /* NLFEAST_H */
