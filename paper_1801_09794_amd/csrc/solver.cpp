// Orchestration of Algorithm 1 (NLFEAST) on one GPU, and the C ABI of include/nlfeast.h.
//
// Per contour (fixed shifts): assemble T(z_k) = sum_j f_j(z_k) A_j for all nodes of all regions
// in one HBM pass, factor them in one batched LU (complex128, or complex64 for the precision
// form, which also keeps T(z_k) in complex128 for the refinement residuals), and keep the
// factors in the caller's workspace for the following solves.
//
// Per iteration and region (Sec. 4.2, Algorithm 1):
//   Step 1  W_j = A_j Q, Ahat_j = Q^H W_j on the device; the reduced problem on the host
//   Step 2  selection of m0 pairs; X = Q Y on the device
//   Step 3  R = T(X, Lambda) = sum_j W_j (Y f_j(Lambda)) as one GEMM, column norms
//   Step 4  Y_k = T(z_k)^{-1} R for all nodes (batched triangular solves; refinement sweeps in
//           the precision form), Q = X rho(Lambda) - sum_k omega_k Y_k (z_k I - Lambda)^{-1}
//   Step 5  Cholesky QR twice (Gram matrix on the device, m0 x m0 Cholesky on the host)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nlfeast.h"
#include "common.hpp"
#include "host_dense.hpp"
#include "kernels.hpp"

namespace nlf {

// ------------------------------------------------------------------------------- profiler
struct Profiler {
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double flops, bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    double ms[NLF_PROF_COUNT] = {}, flops[NLF_PROF_COUNT] = {}, bytes[NLF_PROF_COUNT] = {};
    int64_t launches[NLF_PROF_COUNT] = {};

    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            NLF_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset() {
        recs.clear();
        used = 0;
        std::fill(ms, ms + NLF_PROF_COUNT, 0.0);
        std::fill(flops, flops + NLF_PROF_COUNT, 0.0);
        std::fill(bytes, bytes + NLF_PROF_COUNT, 0.0);
        std::fill(launches, launches + NLF_PROF_COUNT, 0);
    }
    void collect() {   // call after the stream has been synchronised
        for (const Rec& r : recs) {
            float t = 0;
            NLF_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            flops[r.cls] += r.flops;
            bytes[r.cls] += r.bytes;
            launches[r.cls] += 1;
        }
        recs.clear();
        used = 0;
    }
    void merge(const Profiler& o) {   // add another profiler's collected totals
        for (int c = 0; c < NLF_PROF_COUNT; ++c) {
            ms[c] += o.ms[c];
            flops[c] += o.flops[c];
            bytes[c] += o.bytes[c];
            launches[c] += o.launches[c];
        }
    }
    ~Profiler() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

Profiler*& active_profiler() {
    static thread_local Profiler* p = nullptr;
    return p;
}

int& trsm_class() {
    static thread_local int c = NLF_PROF_TRSM;
    return c;
}

ProfScope::ProfScope(int cls_, hipStream_t s_, double fl, double by)
    : p(active_profiler()), cls(cls_), s(s_), flops(fl), bytes(by), ev0(nullptr) {
    if (p) {
        hipEvent_t e = p->get();
        NLF_HIP(hipEventRecord(e, s));
        ev0 = e;
    }
}

ProfScope::~ProfScope() {
    if (p) {
        hipEvent_t e = p->get();
        (void)hipEventRecord(e, s);
        p->recs.push_back({cls, (hipEvent_t)ev0, e, flops, bytes});
    }
}

struct TrsmClassGuard {
    int saved;
    explicit TrsmClassGuard(int c) : saved(trsm_class()) { trsm_class() = c; }
    ~TrsmClassGuard() { trsm_class() = saved; }
};

struct ProfilerGuard {
    Profiler* saved;
    explicit ProfilerGuard(Profiler* p) : saved(active_profiler()) { active_profiler() = p; }
    ~ProfilerGuard() { active_profiler() = saved; }
};

static thread_local std::string g_last_error;

void record_error(const std::string& msg) { g_last_error = msg; }

}  // namespace nlf

using namespace nlf;

// What a captured factorisation graph depends on (kernel arguments are baked into the graph).
struct GraphKey {
    const void* ws = nullptr;
    int prec = -1;
    int64_t n = 0;
    int NZ = 0, J = 0;
    int64_t lda = 0;
    std::vector<const void*> A;
    std::array<int, 5> tune{};
    bool operator==(const GraphKey& o) const {
        return ws == o.ws && prec == o.prec && n == o.n && NZ == o.NZ && J == o.J && lda == o.lda && A == o.A &&
               tune == o.tune;
    }
};

struct nlfeast_ctx {
    int64_t n = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    int J = 0;
    std::vector<Term> terms;
    UserFunction ufn;                                      // for terms of kind NLF_F_USER
    std::vector<const z128*> A;
    int64_t lda = 0;
    // per coefficient matrix: exactly the identity (then A_j Q is Q itself); checked on the
    // device at the first solve after set_coeffs
    std::vector<char> ident;
    bool ident_known = false;
    struct Region {
        Ellipse E;
        int nc = 0, m0 = 0;
        std::vector<cplx> z, w;
    };
    std::vector<Region> regions;
    int quad_rule = 0;
    bool factors_valid = false;
    const void* factors_ws = nullptr;
    int factors_prec = -1;
    bool profiling = false;
    Profiler prof;
    Profiler fprof;                                        // the factorisation thread's launches
    hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};   // factorisation streams
    hipEvent_t ev_join[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipStream_t> rstream;                      // one iteration stream per region
    std::vector<hipEvent_t> rdone;
    std::vector<std::unique_ptr<Profiler>> rprof;
    hipEvent_t ev_lufork = nullptr;
    hipStream_t la_stream[4] = {nullptr, nullptr, nullptr, nullptr};   // LU look-ahead streams
    hipEvent_t la_panel[4] = {nullptr, nullptr, nullptr, nullptr}, la_next[4] = {nullptr, nullptr, nullptr, nullptr};

    // iteration 0 of every region (Steps 0-3 need no factors) runs while the factorisation
    // is in flight: ev_start marks the caller's stream before the factorisation, ev_factored
    // after it and after the pivots' info flags have reached the pinned info_host
    hipEvent_t ev_start = nullptr, ev_factored = nullptr;
    int32_t* info_host = nullptr;
    int info_cap = 0;

    hipStream_t gstream = nullptr;                         // capture stream of the factorisation graph
    // the captured factorisation: graph segments, and between consecutive segments one
    // trailing update launched eagerly (so that its launches stay timed by events)
    std::vector<hipGraphExec_t> graph_segs;
    std::vector<LuUpdateLaunch> graph_mids;
    GraphKey graph_key;
    void drop_graph() {
        for (hipGraphExec_t g : graph_segs) (void)hipGraphExecDestroy(g);
        graph_segs.clear();
        graph_mids.clear();
    }
    ~nlfeast_ctx() {
        drop_graph();
        if (gstream) (void)hipStreamDestroy(gstream);
        for (int i = 0; i < 4; ++i) {
            if (la_stream[i]) (void)hipStreamDestroy(la_stream[i]);
            if (la_panel[i]) (void)hipEventDestroy(la_panel[i]);
            if (la_next[i]) (void)hipEventDestroy(la_next[i]);
        }
        if (ev_lufork) (void)hipEventDestroy(ev_lufork);
        for (hipStream_t r : rstream) (void)hipStreamDestroy(r);
        for (hipEvent_t e : rdone) (void)hipEventDestroy(e);
        for (int i = 0; i < 4; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
        }
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (ev_factored) (void)hipEventDestroy(ev_factored);
        if (info_host) (void)hipHostFree(info_host);
    }
};

namespace {

// Per-region iteration buffers (each region may run on its own stream and host thread).
struct RegionLayout {
    size_t Q = 0, X = 0, W = 0, R = 0, Ys = 0, QT = 0, stmp = 0, R32 = 0, Y32 = 0, E = 0, E32 = 0;
    size_t Ahat = 0, G = 0, Ymat = 0, Gall = 0, rho = 0, acoef = 0, norms = 0, splitws = 0, hh = 0;
    // contour-integral reduced solve on the device (non-polynomial problems): the reduced
    // matrices at the points (then their LU factors), their inverses, pivots, exchange lists,
    // the identity, the functions at the points, the moment weights, the moments, the norms
    size_t cpts = 0, cinv = 0, cpiv = 0, cperm = 0, cinfo = 0, clist = 0, cid = 0, ccoef = 0, cw = 0,
           cmom = 0, cnorm = 0;
    int64_t splitws_elems = 0;
    int node0 = 0, col0 = 0;
};

struct Layout {
    size_t total = 0;
    size_t fact = 0, t64 = 0, ipiv = 0, perm = 0, info = 0, list = 0, dinv = 0, ftmp = 0, coef = 0;
    size_t ident = 0;   // one flag per coefficient matrix: nonzero when it is not the identity
    std::vector<RegionLayout> reg;
    int NZ = 0, M = 0, mmax = 0, ncmax = 0;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(const nlfeast_ctx* h, int prec, bool contour) {
    Layout L;
    const int64_t n = h->n;
    for (const auto& r : h->regions) {
        L.NZ += r.nc;
        L.M += r.m0;
        L.mmax = std::max(L.mmax, r.m0);
        L.ncmax = std::max(L.ncmax, r.nc);
    }
    const int J = std::max(h->J, 1);
    const size_t nn = (size_t)n * n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const bool p32 = prec == NLF_PREC_FP32_REFINE;
    const size_t es = p32 ? 8 : 16;
    L.fact = take(nn * L.NZ * es);
    L.t64 = p32 ? take(nn * L.NZ * 16) : 0;
    L.ipiv = take(sizeof(int32_t) * n * L.NZ);
    L.perm = take(sizeof(int32_t) * n * L.NZ);
    L.info = take(sizeof(int32_t) * L.NZ);
    L.list = take(sizeof(int32_t) * getrf_scratch_ints(n, L.NZ));
    L.dinv = take((size_t)lu_inverse_elems(n) * L.NZ * es);
    L.ftmp = take((size_t)getrf_tmp_elems(n) * L.NZ * es);
    L.coef = take(16 * (size_t)L.NZ * J);
    L.ident = take(sizeof(int32_t) * J);
    int node0 = 0, col0 = 0;
    for (const auto& rg : h->regions) {
        RegionLayout R;
        const int m = rg.m0, nc = rg.nc;
        const size_t blk = (size_t)n * m, mm = (size_t)m * m;
        R.node0 = node0;
        R.col0 = col0;
        R.Q = take(16 * blk);
        R.X = take(16 * blk);
        R.W = take(16 * blk * J);
        R.R = take(16 * blk);
        R.Ys = take(16 * blk * nc);
        R.QT = take(16 * blk);
        R.stmp = take((size_t)256 * m * nc * es);
        R.E = take(16 * blk * nc);   // refinement residuals; the FP64 adjoint solves' scratch
        if (p32) {
            R.R32 = take(8 * blk);
            R.Y32 = take(8 * blk * nc);
            R.E32 = take(8 * blk * nc);
        }
        R.Ahat = take(16 * mm * J);
        R.G = take(16 * mm);
        R.Ymat = take(16 * mm);
        R.Gall = take(16 * mm * J);
        R.rho = take(16 * (size_t)m);
        R.acoef = take(16 * (size_t)m * nc);
        R.norms = take(8 * (size_t)(m + nc + 8 + block_sqnorms_scratch(nc)));
        R.splitws_elems = (int64_t)std::max<size_t>(std::max<size_t>(64 * mm * J, 8 * blk), 1 << 16);
        R.splitws = take(16 * (size_t)R.splitws_elems);
        R.hh = take(16 * (size_t)householder_scratch_elems(m));
        if (contour) {
            const int NP = CONTOUR_POINTS;
            R.cpts = take(16 * mm * NP);
            R.cinv = take(16 * mm * NP);
            R.cpiv = take(sizeof(int32_t) * (size_t)m * NP);
            R.cperm = take(sizeof(int32_t) * (size_t)m * NP);
            R.cinfo = take(sizeof(int32_t) * (size_t)NP);
            R.clist = take(sizeof(int32_t) * (size_t)getrf_scratch_ints(m, NP));
            R.cid = take(16 * mm);
            R.ccoef = take(16 * (size_t)NP * J);
            R.cw = take(16 * (size_t)NP * CONTOUR_MOMENTS);
            R.cmom = take(16 * mm * CONTOUR_MOMENTS);
            R.cnorm = take(8 * (size_t)(NP + block_sqnorms_scratch(NP)));
        }
        L.reg.push_back(R);
        node0 += nc;
        col0 += m;
    }
    L.total = off;
    return L;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

void h2d(hipStream_t s, void* dst, const void* src, size_t bytes) {
    NLF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}
void d2h_sync(hipStream_t s, void* dst, const void* src, size_t bytes) {
    NLF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    NLF_HIP(hipStreamSynchronize(s));
}

// Cholesky QR twice (Step 0 and Step 5).  The filtered block of Step 4 can be numerically rank
// deficient (components of eigenvectors far outside C are damped by rho(lambda) to rounding
// level, and the columns of far-outside Ritz values collapse onto the inside eigenspace);
// Cholesky QR cannot orthonormalise such a block.  When the Cholesky factor of the Gram matrix
// fails or shows a pivot below 1e-12 of its diagonal entry (a column with less than 1e-6 of
// its norm outside the span of the previous ones), the block goes through Householder QR
// instead, which is orthogonal to working precision at any rank.  V: n x m scratch; hh:
// householder_scratch_elems(m) elements.
void orthonormalize(hipStream_t s, int64_t n, int m, z128* Q, z128* QT, z128* Gd, z128* Rd,
                    z128* splitws, int64_t split_elems, z128* V, z128* hh) {
    std::vector<cplx> G((size_t)m * m), Rinv;
    for (int p = 0; p < 2; ++p) {
        {
            ProfScope ps(NLF_PROF_ORTH, s, 8.0 * n * m * m, 16.0 * n * m);
            gemm<double>(s, true, m, m, n, z128(1, 0), Q, n, 0, Q, n, 0, z128(0, 0), Gd, m, 0, 1,
                         splitws, split_elems);
        }
        d2h_sync(s, G.data(), Gd, sizeof(cplx) * m * m);
        double ratio = 0.0;
        if (!cholesky_upper_inverse(m, G.data(), Rinv, &ratio) || ratio < 1e-12) {
            ProfScope ps(NLF_PROF_ORTH, s, 32.0 * n * m * m, 64.0 * n * m);
            householder_orthonormalize(s, n, m, Q, QT, V, hh, splitws, split_elems);
            copy_block(s, n, m, QT, n, Q, n);
            return;
        }
        h2d(s, Rd, Rinv.data(), sizeof(cplx) * m * m);
        {
            ProfScope ps(NLF_PROF_ORTH, s, 8.0 * n * m * m, 32.0 * n * m);
            gemm<double>(s, false, n, m, m, z128(1, 0), Q, n, 0, Rd, m, 0, z128(0, 0), QT, n, 0, 1);
        }
        copy_block(s, n, m, QT, n, Q, n);
    }
}

// W_j = op(A_j) Q and Ahat_j = Q^H W_j, with op(A) = A^H for the adjoint problem.
void project(hipStream_t s, int64_t n, int m, int J, const z128* const* A, int64_t lda,
             const z128* Q, z128* W, z128* Ahat, z128* splitws, int64_t split_elems, bool adj = false,
             const char* ident = nullptr) {
    for (int j = 0; j < J; ++j) {
        if (ident && ident[j]) {   // A_j = I (and I^H = I): W_j = Q
            NLF_HIP(hipMemcpyAsync(W + (size_t)j * n * m, Q, sizeof(z128) * n * m, hipMemcpyDeviceToDevice, s));
            continue;
        }
        ProfScope ps(NLF_PROF_PROJECT, s, 8.0 * n * n * m, 16.0 * ((double)n * n + 2.0 * n * m));
        gemm<double>(s, adj, n, m, n, z128(1, 0), A[j], lda, 0, Q, n, 0, z128(0, 0),
                     W + (size_t)j * n * m, n, 0, 1, splitws, split_elems);
    }
    ProfScope ps(NLF_PROF_PROJECT, s, 8.0 * n * m * m * J, 16.0 * n * m * (J + 1));
    gemm<double>(s, true, m, m, n, z128(1, 0), Q, n, 0, W, n, (int64_t)n * m, z128(0, 0), Ahat, m,
                 (int64_t)m * m, J, splitws, split_elems);
}


// ------------------------------------------------------------------ factorisation of all nodes

// LU launch parameters: panel width, trailing-update GEMM tile, node groups on separate streams.
struct LuTuning {
    int panel_width = 32;
    int groups = 1;
    int tm = 0, tn = 0;   // 0: default tile choice
    int lookahead = 0;
    bool operator==(const LuTuning& o) const {
        return panel_width == o.panel_width && groups == o.groups && tm == o.tm && tn == o.tn &&
               lookahead == o.lookahead;
    }
};

LuTuning fixed_tuning(const nlfeast_options& o) {
    LuTuning t;
    if (o.panel_width) t.panel_width = o.panel_width;
    if (o.lu_streams) t.groups = o.lu_streams;
    if (o.lookahead) t.lookahead = o.lookahead > 0 ? 1 : 0;
    return t;
}

struct TuningScope {   // applies a tuning to this thread's LU launches
    int saved_pw;
    GemmConfig saved_tile;
    explicit TuningScope(const LuTuning& t) : saved_pw(lu_panel_width()), saved_tile(lu_update_tile()) {
        lu_panel_width() = t.panel_width;
        lu_update_tile() = GemmConfig{t.tm, t.tn};
    }
    ~TuningScope() {
        lu_panel_width() = saved_pw;
        lu_update_tile() = saved_tile;
    }
};

// Assemble T(z_k) for every node from the coefficients in the workspace and factor them all,
// enqueued on cs (node groups fork to the handle's side streams and join back to cs).
void factor_all(nlfeast_ctx* h, const Layout& L, void* ws, bool p32, hipStream_t cs, const LuTuning& t) {
    TuningScope ts(t);
    const int64_t n = h->n;
    const int J = h->J;
    const size_t nn = (size_t)n * n;
    if (p32)
        assemble(cs, n, J, h->A.data(), h->lda, L.NZ, at<z128>(ws, L.coef), at<z128>(ws, L.t64),
                 at<z64>(ws, L.fact), n, (int64_t)nn);
    else
        assemble(cs, n, J, h->A.data(), h->lda, L.NZ, at<z128>(ws, L.coef), at<z128>(ws, L.fact), nullptr,
                 n, (int64_t)nn);
    TrsmClassGuard tg(NLF_PROF_TRSM);
    // groups of node matrices on separate streams: the latency-bound panels of one group run
    // while the GEMMs of another fill the machine
    const int groups = std::max(1, std::min({t.groups, 4, L.NZ}));
    if (groups > 1) {
        if (!h->ev_lufork) NLF_HIP(hipEventCreateWithFlags(&h->ev_lufork, hipEventDisableTiming));
        NLF_HIP(hipEventRecord(h->ev_lufork, cs));
    }
    const int64_t dper = lu_inverse_elems(n);
    const int64_t lper = getrf_scratch_ints(n, 1);
    const int64_t tper = getrf_tmp_elems(n);
    if (t.lookahead)
        for (int g = 0; g < groups; ++g)
            if (!h->la_stream[g]) {
                NLF_HIP(hipStreamCreateWithFlags(&h->la_stream[g], hipStreamNonBlocking));
                NLF_HIP(hipEventCreateWithFlags(&h->la_panel[g], hipEventDisableTiming));
                NLF_HIP(hipEventCreateWithFlags(&h->la_next[g], hipEventDisableTiming));
            }
    for (int g = 0; g < groups; ++g) {
        const int q0 = (int)((int64_t)L.NZ * g / groups), q1 = (int)((int64_t)L.NZ * (g + 1) / groups);
        if (q1 <= q0) continue;
        const int nb = q1 - q0;
        hipStream_t sg = cs;
        LuAux aux;
        if (t.lookahead) {
            aux.s = h->la_stream[g];
            aux.panel_done = h->la_panel[g];
            aux.next_ready = h->la_next[g];
        }
        if (groups > 1) {
            if (!h->side[g]) {
                NLF_HIP(hipStreamCreateWithFlags(&h->side[g], hipStreamNonBlocking));
                NLF_HIP(hipEventCreateWithFlags(&h->ev_join[g], hipEventDisableTiming));
            }
            sg = h->side[g];
            NLF_HIP(hipStreamWaitEvent(sg, h->ev_lufork, 0));
        }
        int32_t* ipiv = at<int32_t>(ws, L.ipiv) + (size_t)q0 * n;
        int32_t* perm = at<int32_t>(ws, L.perm) + (size_t)q0 * n;
        int32_t* info = at<int32_t>(ws, L.info) + q0;
        int32_t* list = at<int32_t>(ws, L.list) + (size_t)q0 * lper;
        if (p32)
            getrf<float>(sg, n, nb, at<z64>(ws, L.fact) + (size_t)q0 * nn, n, (int64_t)nn, ipiv, perm, info, list,
                         at<z64>(ws, L.dinv) + (size_t)q0 * dper, at<z64>(ws, L.ftmp) + (size_t)q0 * tper, &aux);
        else
            getrf<double>(sg, n, nb, at<z128>(ws, L.fact) + (size_t)q0 * nn, n, (int64_t)nn, ipiv, perm, info,
                          list, at<z128>(ws, L.dinv) + (size_t)q0 * dper, at<z128>(ws, L.ftmp) + (size_t)q0 * tper,
                          &aux);
        if (groups > 1) {
            NLF_HIP(hipEventRecord(h->ev_join[g], sg));
            NLF_HIP(hipStreamWaitEvent(cs, h->ev_join[g], 0));
        }
    }
}

// Tuner: on first use of a (precision, n, node count) shape, time trial factorisations of the
// real node matrices over the candidate launch parameters and keep the fastest for the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int>, LuTuning> g_tune_cache;

LuTuning autotuned(nlfeast_ctx* h, const Layout& L, void* ws, bool p32, hipStream_t s, const nlfeast_options& o) {
    const auto key = std::make_tuple(o.precision, h->n, L.NZ);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    std::vector<int> pws = o.panel_width ? std::vector<int>{o.panel_width} : std::vector<int>{16, 32};
    // look-ahead is not combined with node groups on several streams (see the option check)
    std::vector<int> las = o.lookahead ? std::vector<int>{o.lookahead > 0 ? 1 : 0}
                           : o.lu_streams > 1 ? std::vector<int>{0}
                                              : std::vector<int>{0, 1};
    std::vector<std::pair<int, int>> tiles = p32 ? std::vector<std::pair<int, int>>{{0, 0}, {2, 2}, {4, 4}}
                                                 : std::vector<std::pair<int, int>>{{0, 0}, {4, 2}};
    const int g0 = o.lu_streams ? o.lu_streams : 1;
    std::vector<LuTuning> cand;
    for (int la : las)
        for (int pw : pws)
            for (auto tl : tiles) {
                LuTuning t;
                t.panel_width = pw;
                t.groups = g0;
                t.tm = tl.first;
                t.tn = tl.second;
                t.lookahead = la;
                cand.push_back(t);
            }
    if (!o.lu_streams) {   // two node groups on separate streams, other parameters at default
        LuTuning t = cand[0];
        t.groups = 2;
        cand.push_back(t);
    }
    Profiler* saved = active_profiler();
    active_profiler() = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LuTuning best = fixed_tuning(o);
    float best_ms = 0.f, total_ms = 0.f;
    try {
        NLF_HIP(hipEventCreate(&e0));
        NLF_HIP(hipEventCreate(&e1));
        factor_all(h, L, ws, p32, s, cand[0]);   // warm-up: code objects, caches
        for (size_t c = 0; c < cand.size(); ++c) {
            NLF_HIP(hipEventRecord(e0, s));
            factor_all(h, L, ws, p32, s, cand[c]);
            NLF_HIP(hipEventRecord(e1, s));
            NLF_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            NLF_HIP(hipEventElapsedTime(&ms, e0, e1));
            total_ms += ms;
            if (o.verbose)
                fprintf(stderr, "[nlfeast] tune pw %d groups %d tile %dx%d lookahead %d: %.3f ms\n",
                        cand[c].panel_width, cand[c].groups, cand[c].tm, cand[c].tn, cand[c].lookahead, ms);
            if (c == 0 || ms < best_ms) {
                best_ms = ms;
                best = cand[c];
            }
        }
    } catch (...) {
        active_profiler() = saved;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        throw;
    }
    active_profiler() = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (saved) {
        saved->ms[NLF_PROF_AUTOTUNE] += total_ms;
        saved->launches[NLF_PROF_AUTOTUNE] += (int64_t)cand.size();
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

GraphKey graph_key(const nlfeast_ctx* h, const Layout& L, const void* ws, int prec, const LuTuning& t) {
    GraphKey k;
    k.ws = ws;
    k.prec = prec;
    k.n = h->n;
    k.NZ = L.NZ;
    k.J = h->J;
    k.lda = h->lda;
    k.A.assign(h->A.begin(), h->A.end());
    k.tune = {t.panel_width, t.groups, t.tm, t.tn, t.lookahead};
    return k;
}

// Record factor_all on the handle's capture stream (nothing executes).  With one node group and
// no look-ahead the capture is cut at every trailing update: h->graph_segs holds the graph
// segments and h->graph_mids the updates that run eagerly between them; otherwise the whole
// factorisation is one segment.
void capture_factorisation(nlfeast_ctx* h, const Layout& L, void* ws, bool p32, const LuTuning& t) {
    if (!h->gstream) NLF_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    h->drop_graph();
    Profiler* saved = active_profiler();
    active_profiler() = nullptr;   // no event records inside the capture
    std::function<void(LuUpdateLaunch&&)>* saved_hook = lu_update_hook();
    std::vector<hipGraph_t> graphs;
    std::function<void(LuUpdateLaunch&&)> cut = [&](LuUpdateLaunch&& u) {
        hipGraph_t g = nullptr;
        NLF_HIP(hipStreamEndCapture(h->gstream, &g));
        graphs.push_back(g);
        h->graph_mids.push_back(std::move(u));
        NLF_HIP(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    };
    const bool segmented = !t.lookahead && t.groups <= 1;
    auto restore = [&] {
        active_profiler() = saved;
        lu_update_hook() = saved_hook;
    };
    auto discard = [&] {
        for (hipGraph_t g : graphs) (void)hipGraphDestroy(g);
        graphs.clear();
        h->graph_mids.clear();
    };
    try {
        NLF_HIP(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        if (segmented) lu_update_hook() = &cut;
        factor_all(h, L, ws, p32, h->gstream, t);
    } catch (...) {
        restore();
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(h->gstream, &g);
        if (g) (void)hipGraphDestroy(g);
        discard();
        throw;
    }
    restore();
    hipGraph_t last = nullptr;
    NLF_HIP(hipStreamEndCapture(h->gstream, &last));
    graphs.push_back(last);
    for (hipGraph_t g : graphs) {
        hipGraphExec_t e = nullptr;
        const hipError_t st = hipGraphInstantiateWithFlags(&e, g, 0);
        if (st != hipSuccess) {
            discard();
            h->drop_graph();
            throw Error{NLF_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(st)};
        }
        h->graph_segs.push_back(e);
    }
    for (hipGraph_t g : graphs) (void)hipGraphDestroy(g);   // the instantiated segments keep what they need
}

// Replay the captured factorisation on s: the segments in order, each followed by its eager
// trailing update (timed as NLF_K_LU_GEMM when profiling).
void replay_factorisation(nlfeast_ctx* h, hipStream_t s) {
    for (size_t i = 0; i < h->graph_segs.size(); ++i) {
        NLF_HIP(hipGraphLaunch(h->graph_segs[i], s));
        if (i < h->graph_mids.size()) {
            const LuUpdateLaunch& u = h->graph_mids[i];
            ProfScope ps(NLF_PROF_LU_GEMM, s, u.flops, u.bytes);
            u.launch(s);
        }
    }
}

// Spurious Ritz values (Sec. 4.2: Ritz pairs that match no eigenpair of the full problem).
// Each current Ritz value is paired with at most one of the previous iteration's, nearest pairs
// first (ties: lower current index, then lower previous index); -1 = unpaired.
std::vector<int> match_previous(const std::vector<cplx>& cur, const std::vector<cplx>& prev) {
    const int m = (int)cur.size(), p = (int)prev.size();
    std::vector<std::pair<double, int64_t>> d;
    d.reserve((size_t)m * p);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < p; ++j) {
            const double v = std::abs(cur[i] - prev[j]);
            if (std::isfinite(v)) d.emplace_back(v, (int64_t)i * p + j);
        }
    std::stable_sort(d.begin(), d.end(),
                     [](const std::pair<double, int64_t>& a, const std::pair<double, int64_t>& b) {
                         return a.first < b.first || (a.first == b.first && a.second < b.second);
                     });
    std::vector<int> partner(m, -1);
    std::vector<char> used(p, 0);
    for (const auto& e : d) {
        const int i = (int)(e.second / p), j = (int)(e.second % p);
        if (partner[i] < 0 && !used[j]) {
            partner[i] = j;
            used[j] = 1;
        }
    }
    return partner;
}

// The unconverged Ritz values inside C whose residual did not shrink by the filter's
// contraction bound: a genuine pair's residual falls by about |rho(lambda_out)| / |rho(lambda_i)|
// per iteration (rho the quadrature filter, lambda_out the first eigenvalue the subspace leaves
// out, bounded by the farthest selected value, rho_min); stagnant means res_i > theta_i times its
// partner's, theta_i = min(0.97, max(0.25, (rho_min / |rho(lambda_i)|)^(1/3))).
std::vector<char> stagnant(const std::vector<cplx>& lam, const std::vector<double>& res,
                           const std::vector<char>& unconv, const std::vector<cplx>& z,
                           const std::vector<cplx>& w, const std::vector<cplx>& prev_lam,
                           const std::vector<double>& prev_res) {
    const int m = (int)lam.size();
    std::vector<double> rho(m, 0.0);
    double rho_min = INFINITY;
    for (int i = 0; i < m; ++i) {
        if (!std::isfinite(lam[i].real()) || !std::isfinite(lam[i].imag())) continue;
        cplx sum = 0.0;
        for (size_t k = 0; k < z.size(); ++k) sum += w[k] / (z[k] - lam[i]);
        rho[i] = std::abs(sum);
        rho_min = std::min(rho_min, rho[i]);
    }
    if (!std::isfinite(rho_min)) rho_min = 0.0;
    const std::vector<int> partner = match_previous(lam, prev_lam);
    std::vector<char> out(m, 0);
    for (int i = 0; i < m; ++i) {
        if (!unconv[i]) continue;
        const double theta = std::min(0.97, std::max(0.25, std::cbrt(rho_min / std::max(rho[i], 1e-300))));
        const double before = partner[i] >= 0 ? prev_res[partner[i]] : 0.0;
        out[i] = !(res[i] <= theta * before);
    }
    return out;
}

// The moments of the reduced resolvent for the contour-integral reduced solve, on the device:
// T_red(z_q) = sum_j f_j(z_q) Ahat_j at the CONTOUR_POINTS points of the enlarged contour (the
// assembly kernel with n = m), their batched LU and inverses T_red(z_q)^{-1} (solves against
// the identity), the squared Frobenius norms of the inverses, and the CONTOUR_MOMENTS sums
// M_p = sum_q w_q mu_q^p T_red(z_q)^{-1} as one GEMM of the m^2 x CONTOUR_POINTS block of
// inverses with the weights.  Inputs in the region's buffers: ccoef (f_j(z_q) at q J + j), cw
// (w_q mu_q^p at q + p CONTOUR_POINTS), cid (the m x m identity).
void device_moments(hipStream_t s, int m, int J, const z128* Ahat_d, void* ws, const RegionLayout& RL) {
    const int NP = CONTOUR_POINTS, NM = CONTOUR_MOMENTS;
    const size_t mm = (size_t)m * m;
    const double flops = NP * (8.0 * J * mm + 8.0 / 3.0 * m * (double)mm + 8.0 * m * (double)mm) + 8.0 * mm * NP * NM;
    ProfScope ps(NLF_PROF_REDUCED, s, flops, 16.0 * mm * NP * 4);
    ProfilerGuard off(nullptr);   // the launches below are timed as one span
    std::vector<const z128*> A(J);
    for (int j = 0; j < J; ++j) A[j] = Ahat_d + (size_t)j * mm;
    z128* T = at<z128>(ws, RL.cpts);
    z128* Inv = at<z128>(ws, RL.cinv);
    int32_t* perm = at<int32_t>(ws, RL.cperm);
    assemble(s, m, J, A.data(), m, NP, at<z128>(ws, RL.ccoef), T, nullptr, m, (int64_t)mm);
    getrf<double>(s, m, NP, T, m, (int64_t)mm, at<int32_t>(ws, RL.cpiv), perm, at<int32_t>(ws, RL.cinfo),
                  at<int32_t>(ws, RL.clist));
    getrs<double>(s, m, m, NP, T, m, (int64_t)mm, perm, at<z128>(ws, RL.cid), m, 0, Inv, m, (int64_t)mm);
    block_sqnorms(s, m, m, NP, Inv, m, (int64_t)mm, at<double>(ws, RL.cnorm), at<double>(ws, RL.cnorm) + NP);
    gemm<double>(s, false, (int64_t)mm, NM, NP, z128(1, 0), Inv, (int64_t)mm, 0, at<z128>(ws, RL.cw), NP, 0,
                 z128(0, 0), at<z128>(ws, RL.cmom), (int64_t)mm, 0, 1);
}

struct RegionIO {
    const void* X0;
    void* Xout;
    double* lambda;
    double* resid;
    int32_t* inside;
    int32_t* m_out;
    int32_t* iters;
    // set once the factorisation has been enqueued by its host thread (the event passed to the
    // regions is recorded then); holds that thread's error if it failed.  Null: nothing to wait for
    const std::shared_future<void>* enqueued = nullptr;
};

struct RegionOutcome {
    int status = NLF_OK;
    std::string msg;
};

// Algorithm 1 Steps 0-5 for region ri, on stream s, with the node factorisations already in the
// workspace.  Writes the region's slice of the outputs; never throws.
// Algorithm 1 for region ri.  adj: the adjoint problem S(mu) = T(conj mu)^H on the conjugate
// contour (nodes conj z_k, weights conj omega_k, whose matrices T(z_k)^H reuse the factors of
// T(z_k) through adjoint solves): its eigenvectors are the left eigenvectors of T, its
// eigenvalues the conjugates of T's (returned conjugated back).
RegionOutcome run_region(nlfeast_ctx* h, const nlfeast_options& o, void* ws, const Layout& L, int ri,
                         hipStream_t s, Profiler* prof, const RegionIO& io, hipEvent_t factored,
                         std::atomic<int64_t>* active = nullptr, bool adj = false) {
    RegionOutcome res_out;
    try {
        ProfilerGuard pg(prof);
        const nlfeast_options* opt = &o;
        const int64_t n = h->n;
        const int J = h->J;
        const bool p32 = opt->precision == NLF_PREC_FP32_REFINE;
        const size_t nn = (size_t)n * n;
        const RegionLayout& RL = L.reg[ri];
        const int node0 = RL.node0, col0 = RL.col0;
        auto host_ms = [&](double ms) {
            if (prof) {
                prof->ms[NLF_PROF_HOST] += ms;
                prof->launches[NLF_PROF_HOST] += 1;
            }
        };
        const auto& reg = h->regions[ri];
        const int m = reg.m0, nc = reg.nc;
        std::vector<Term> terms = h->terms;
        std::vector<cplx> zn = reg.z, wn = reg.w;
        Ellipse E = reg.E;
        if (adj) {
            for (Term& t : terms) t.conj = true;
            for (cplx& v : zn) v = std::conj(v);
            for (cplx& v : wn) v = std::conj(v);
            E.c = std::conj(E.c);
        }
        z128* Q = at<z128>(ws, RL.Q);
        z128* X = at<z128>(ws, RL.X);
        z128* W = at<z128>(ws, RL.W);
        z128* R = at<z128>(ws, RL.R);
        z128* Ys = at<z128>(ws, RL.Ys);
        z128* QT = at<z128>(ws, RL.QT);
        z128* Ahat_d = at<z128>(ws, RL.Ahat);
        z128* Gd = at<z128>(ws, RL.G);
        z128* Ymat = at<z128>(ws, RL.Ymat);
        z128* Gall = at<z128>(ws, RL.Gall);
        z128* rho_d = at<z128>(ws, RL.rho);
        z128* acoef_d = at<z128>(ws, RL.acoef);
        double* norms_d = at<double>(ws, RL.norms);
        z128* splitws = at<z128>(ws, RL.splitws);
        const size_t blk = (size_t)n * m;
        // Step 0
        if (io.X0)
            copy_block(s, n, m, (const z128*)io.X0 + (size_t)col0 * n, n, Q, n);
        else
            random_normal(s, n, m, opt->seed * 0x9E3779B97F4A7C15ull + ri + 1, Q, n);
        orthonormalize(s, n, m, Q, QT, Gd, at<z128>(ws, RL.Ymat), splitws, RL.splitws_elems, Ys,
                       at<z128>(ws, RL.hh));

        std::vector<cplx> Ahat((size_t)J * m * m), lam(m), Gh((size_t)J * m * m), rho(m),
            acoef((size_t)nc * m);
        // contour-integral reduced solve: its moments are formed on the device; the points, the
        // functions there and the moment weights are fixed for the whole solve
        const bool cdev = takes_contour_route(terms, opt->reduced_solver);
        std::vector<cplx> cmom;
        std::vector<double> cnorm, isize;
        std::vector<int32_t> cinfo;
        std::vector<cplx> cwt;
        if (cdev) {
            const int NP = CONTOUR_POINTS, NM = CONTOUR_MOMENTS;
            std::vector<cplx> cz, cmu;
            contour_points(E, cz, cwt, cmu);
            std::vector<cplx> fz((size_t)J * NP), coef((size_t)NP * J), wts((size_t)NP * NM), ident((size_t)m * m, 0.0);
            for (int j = 0; j < J; ++j) term_values(terms[j], cz.data(), NP, &fz[(size_t)j * NP]);
            NLF_REQUIRE(!user_failed(terms), NLF_ERR_ARG, "solve: the user function reported an error");
            for (int q = 0; q < NP; ++q) {
                for (int j = 0; j < J; ++j) coef[(size_t)q * J + j] = fz[(size_t)j * NP + q];
                cplx wp = cwt[q];
                for (int p = 0; p < NM; ++p, wp *= cmu[q]) wts[q + (size_t)p * NP] = wp;
            }
            for (int i = 0; i < m; ++i) ident[i + (size_t)i * m] = 1.0;
            h2d(s, at<void>(ws, RL.ccoef), coef.data(), sizeof(cplx) * coef.size());
            h2d(s, at<void>(ws, RL.cw), wts.data(), sizeof(cplx) * wts.size());
            h2d(s, at<void>(ws, RL.cid), ident.data(), sizeof(cplx) * ident.size());
            NLF_HIP(hipStreamSynchronize(s));   // the host vectors above go out of scope
            cmom.resize((size_t)NM * m * m);
            cnorm.resize(NP);
            isize.resize(NP);
            cinfo.resize(NP);
        }
        std::vector<double> res(m), enorm(nc);
        // once a refinement check passes without a correction, the complex64 factors have shown
        // themselves accurate enough for this region's right-hand sides and later iterations
        // skip the check (the FP64 residual of Step 3 still decides convergence)
        bool refine_needed = true;
        ReducedResult rr;
        int it = 0, n_in = 0, n_conv = 0;
        std::vector<int> inside(m);
        std::vector<char> spurious(m, 0);
        std::vector<cplx> prev_lam;
        std::vector<double> prev_res;
        int rstatus = NLF_OK;
        const z128* LU128 = at<z128>(ws, L.fact) + (size_t)node0 * nn;
        const z64* LU64 = at<z64>(ws, L.fact) + (size_t)node0 * nn;
        const int32_t* perm = at<int32_t>(ws, L.perm) + (size_t)node0 * n;
        const int64_t dper = lu_inverse_elems(n);
        const z128* D128 = at<z128>(ws, L.dinv) + (size_t)node0 * dper;
        const z64* D64 = at<z64>(ws, L.dinv) + (size_t)node0 * dper;
        while (true) {
            // Step 1: projections and the reduced problem
            project(s, n, m, J, h->A.data(), h->lda, Q, W, Ahat_d, splitws, RL.splitws_elems, adj,
                    h->ident_known ? h->ident.data() : nullptr);
            if (cdev) {
                device_moments(s, m, J, Ahat_d, ws, RL);
                NLF_HIP(hipMemcpyAsync(cmom.data(), at<void>(ws, RL.cmom), sizeof(cplx) * cmom.size(),
                                       hipMemcpyDeviceToHost, s));
                NLF_HIP(hipMemcpyAsync(cnorm.data(), at<void>(ws, RL.cnorm), sizeof(double) * cnorm.size(),
                                       hipMemcpyDeviceToHost, s));
                NLF_HIP(hipMemcpyAsync(cinfo.data(), at<void>(ws, RL.cinfo), sizeof(int32_t) * cinfo.size(),
                                       hipMemcpyDeviceToHost, s));
            }
            d2h_sync(s, Ahat.data(), Ahat_d, sizeof(cplx) * Ahat.size());
            const auto t0 = std::chrono::steady_clock::now();
            std::vector<cplx> prev;
            if (it > 0) prev = rr.lambda;
            if (active) {   // share the host threads among the regions still iterating, in
                            // proportion to their reduced solves' work (m^3)
                const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
                const double share = (double)m * m * m / (double)std::max<int64_t>(1, active->load());
                host_thread_budget() = std::max(1, (int)std::lround(hw * std::min(1.0, share)));
            }
            if (cdev) {
                bool singular = false;
                for (int q = 0; q < CONTOUR_POINTS; ++q) {
                    singular = singular || cinfo[q] != 0;
                    isize[q] = std::abs(cwt[q]) * std::sqrt(cnorm[q]);
                }
                if (singular) {
                    rr = ReducedResult();
                    rr.ok = false;
                } else {
                    rr = contour_reduced_from_moments(m, terms, Ahat.data(), E, m, cmom, isize);
                }
            } else {
                rr = reduced_solve(m, terms, Ahat.data(), E, m, it > 0 ? &prev : nullptr, opt->reduced_solver);
            }
            const double hms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            host_ms(hms);
            if (opt->verbose)
                fprintf(stderr,
                        "[nlfeast] region %d it %d host reduced %.1f ms (points+moments %.1f, rank+eig %.1f, "
                        "newton %.1f: %d pairs %d steps, rank %d)\n",
                        ri, it, hms, rr.ms_points, rr.ms_rank_eig, rr.ms_newton, rr.newton_pairs, rr.newton_steps,
                        rr.rank);
            NLF_REQUIRE(!user_failed(terms), NLF_ERR_ARG, "solve: the user function reported an error");
            NLF_REQUIRE(rr.ok && (int)rr.lambda.size() == m, NLF_ERR_DEVICE,
                        "reduced eigenproblem failed (singular T at the contour centre or on the enlarged "
                        "contour, QR did not converge, or too many eigenvalues inside the enlarged contour)");
            // Step 2: X = Q Y
            for (int i = 0; i < m; ++i) lam[i] = std::isfinite(rr.lambda[i].real()) ? rr.lambda[i] : cplx(0.0);
            h2d(s, Ymat, rr.Y.data(), sizeof(cplx) * m * m);
            {
                ProfScope ps(NLF_PROF_RESIDUAL, s, 8.0 * n * m * m, 32.0 * n * m);
                gemm<double>(s, false, n, m, m, z128(1, 0), Q, n, 0, Ymat, m, 0, z128(0, 0), X, n, 0, 1);
            }
            // Step 3: R = sum_j W_j (Y f_j(Lambda)), res_i = ||R e_i||
            for (int j = 0; j < J; ++j)
                for (int c = 0; c < m; ++c) {
                    const cplx f = term_value(terms[j], lam[c]);
                    for (int r = 0; r < m; ++r)
                        Gh[(size_t)j * m + r + (size_t)c * J * m] = rr.Y[r + (size_t)c * m] * f;
                }
            NLF_REQUIRE(!user_failed(terms), NLF_ERR_ARG, "solve: the user function reported an error");
            h2d(s, Gall, Gh.data(), sizeof(cplx) * Gh.size());
            {
                ProfScope ps(NLF_PROF_RESIDUAL, s, 8.0 * n * m * m * J, 16.0 * n * m * (J + 1));
                gemm<double>(s, false, n, m, (int64_t)J * m, z128(1, 0), W, n, 0, Gall, (int64_t)J * m, 0,
                             z128(0, 0), R, n, 0, 1);
                col_norms(s, n, m, R, n, norms_d);
            }
            d2h_sync(s, res.data(), norms_d, sizeof(double) * m);
            n_in = 0;
            n_conv = 0;
            double maxres = 0.0;
            std::vector<char> unconv(m, 0);
            for (int i = 0; i < m; ++i) {
                if (!std::isfinite(rr.lambda[i].real())) res[i] = INFINITY;
                inside[i] = E.radius(rr.lambda[i]) < 1.0;
                if (inside[i]) {
                    ++n_in;
                    maxres = std::max(maxres, res[i]);
                    if (res[i] <= opt->tol) ++n_conv;
                    else unconv[i] = 1;
                }
            }
            if (opt->verbose)
                fprintf(stderr, "[nlfeast] region %d it %d inside %d converged %d max_res %.3e\n", ri, it, n_in,
                        n_conv, maxres);
            if (n_in >= m) { rstatus = NLF_ERR_M0_TOO_SMALL; break; }
            if (it >= 1 && n_in > 0 && maxres <= opt->tol) break;
            // spurious Ritz values inside C: stop once every inside value that has not
            // converged is stagnant
            if (it >= 2 && !prev_lam.empty() && n_conv > 0 && n_conv < n_in) {
                const std::vector<char> st = stagnant(rr.lambda, res, unconv, zn, wn, prev_lam, prev_res);
                bool all = true;
                int n_st = 0;
                for (int i = 0; i < m; ++i) {
                    if (unconv[i] && !st[i]) all = false;
                    n_st += st[i];
                }
                if (opt->verbose)
                    fprintf(stderr, "[nlfeast] region %d it %d stagnant %d of %d unconverged inside\n", ri, it, n_st,
                            n_in - n_conv);
                if (all) {
                    spurious = st;
                    rstatus = NLF_SPURIOUS;
                    break;
                }
            }
            prev_lam = rr.lambda;
            prev_res = res;
            if (it >= 3 && n_in == 0) break;
            if (it >= opt->max_iter) { rstatus = NLF_ERR_NOT_CONVERGED; break; }
            // the factors are needed from here on: wait for the factorisation launched before
            // iteration 0 and reject singular node matrices of this region
            if (factored) {
                if (io.enqueued) {   // the event must be recorded before it can be waited on
                    std::shared_future<void> f = *io.enqueued;
                    f.get();
                }
                NLF_HIP(hipEventSynchronize(factored));
                for (int q = 0; q < nc; ++q)
                    NLF_REQUIRE(h->info_host[node0 + q] == 0, NLF_ERR_SINGULAR,
                                "solve: T(z_k) is singular at node " + std::to_string(node0 + q) +
                                    " (exact zero pivot " + std::to_string(h->info_host[node0 + q]) + ")");
                NLF_HIP(hipStreamWaitEvent(s, factored, 0));
                factored = nullptr;
            }
            // Step 4: Y_k = T(z_k)^{-1} R for the region's nodes
            {
                TrsmClassGuard tg(NLF_PROF_SOLVE);
                if (!p32 && adj) {
                    getrs_inv_adjoint<double>(s, n, m, nc, LU128, n, (int64_t)nn, perm, D128, R, n, 0,
                                              at<z128>(ws, RL.E), Ys, n, (int64_t)blk, at<z128>(ws, RL.stmp));
                } else if (!p32) {
                    getrs_inv<double>(s, n, m, nc, LU128, n, (int64_t)nn, perm, D128, R, n, 0, Ys, n,
                                      (int64_t)blk, at<z128>(ws, RL.stmp));
                } else {
                    z64* R32 = at<z64>(ws, RL.R32);
                    z64* Y32 = at<z64>(ws, RL.Y32);
                    z128* E = at<z128>(ws, RL.E);
                    z64* E32 = at<z64>(ws, RL.E32);
                    const z128* T64 = at<z128>(ws, L.t64) + (size_t)node0 * nn;
                    cast_128_to_64(s, n, m, 1, R, n, 0, R32, n, 0);
                    if (adj)
                        getrs_inv_adjoint<float>(s, n, m, nc, LU64, n, (int64_t)nn, perm, D64, R32, n, 0, E32, Y32, n,
                                                 (int64_t)blk, at<z64>(ws, RL.stmp));
                    else
                        getrs_inv<float>(s, n, m, nc, LU64, n, (int64_t)nn, perm, D64, R32, n, 0, Y32, n,
                                         (int64_t)blk, at<z64>(ws, RL.stmp));
                    cast_64_to_128(s, n, m, nc, Y32, n, (int64_t)blk, Ys, n, (int64_t)blk, false);
                    double rn2 = 0.0;
                    for (int i = 0; i < m; ++i) rn2 += std::isfinite(res[i]) ? res[i] * res[i] : 0.0;
                    for (int sweep = 0; refine_needed && sweep < std::min(opt->max_refine, 5); ++sweep) {
                        TrsmClassGuard tg2(NLF_PROF_REFINE);
                        ProfScope ps(NLF_PROF_REFINE, s, 8.0 * n * n * m * nc, 16.0 * nn * nc);
                        // E_k = R - T(z_k) Y_k (adjoint: R - T(z_k)^H Y_k) in FP64
                        for (int q = 0; q < nc; ++q) copy_block(s, n, m, R, n, E + q * blk, n);
                        gemm<double>(s, adj, n, m, n, z128(-1, 0), T64, n, (int64_t)nn, Ys, n, (int64_t)blk,
                                     z128(1, 0), E, n, (int64_t)blk, nc);
                        block_sqnorms(s, n, m, nc, E, n, (int64_t)blk, norms_d, norms_d + m + nc + 8);
                        d2h_sync(s, enorm.data(), norms_d, sizeof(double) * nc);
                        double worst = 0.0;
                        for (int q = 0; q < nc; ++q) worst = std::max(worst, enorm[q]);
                        if (opt->verbose)
                            fprintf(stderr, "[nlfeast] region %d it %d refinement check %d: max ||E_k|| / ||R|| %.3e\n",
                                    ri, it, sweep, std::sqrt(worst / std::max(rn2, 1e-300)));
                        if (worst <= opt->refine_eta * opt->refine_eta * rn2) {
                            if (sweep == 0) refine_needed = false;
                            break;
                        }
                        cast_128_to_64(s, n, m, nc, E, n, (int64_t)blk, E32, n, (int64_t)blk);
                        if (adj)
                            getrs_inv_adjoint<float>(s, n, m, nc, LU64, n, (int64_t)nn, perm, D64, E32, n,
                                                     (int64_t)blk, E32, Y32, n, (int64_t)blk, at<z64>(ws, RL.stmp));
                        else
                            getrs_inv<float>(s, n, m, nc, LU64, n, (int64_t)nn, perm, D64, E32, n, (int64_t)blk,
                                             Y32, n, (int64_t)blk, at<z64>(ws, RL.stmp));
                        cast_64_to_128(s, n, m, nc, Y32, n, (int64_t)blk, Ys, n, (int64_t)blk, true);
                    }
                }
            }
            // Step 4 accumulation: Q = X rho(Lambda) - sum_k omega_k Y_k (z_k - Lambda)^{-1}
            for (int i = 0; i < m; ++i) {
                cplx rsum = 0.0;
                for (int q = 0; q < nc; ++q) {
                    const cplx cq = wn[q] / (zn[q] - lam[i]);
                    acoef[(size_t)q * m + i] = cq;
                    rsum += cq;
                }
                rho[i] = rsum;
            }
            h2d(s, rho_d, rho.data(), sizeof(cplx) * m);
            h2d(s, acoef_d, acoef.data(), sizeof(cplx) * acoef.size());
            accumulate(s, n, m, nc, X, Ys, (int64_t)blk, rho_d, acoef_d, Q);
            // Step 5
            orthonormalize(s, n, m, Q, QT, Gd, Ymat, splitws, RL.splitws_elems, Ys, at<z128>(ws, RL.hh));
            ++it;
        }
        // outputs for this region
        NLF_HIP(hipMemcpyAsync((z128*)io.Xout + (size_t)col0 * n, X, sizeof(z128) * blk,
                               hipMemcpyDeviceToDevice, s));
        for (int i = 0; i < m; ++i) {
            const cplx l = adj ? std::conj(rr.lambda[i]) : rr.lambda[i];   // eigenvalues of T
            io.lambda[2 * (col0 + i)] = l.real();
            io.lambda[2 * (col0 + i) + 1] = l.imag();
            io.resid[col0 + i] = res[i];
            io.inside[col0 + i] = spurious[i] ? 2 : inside[i];
        }
        io.m_out[ri] = n_conv;
        io.iters[ri] = it;
        NLF_HIP(hipStreamSynchronize(s));
        res_out.status = rstatus;
        if (rstatus == NLF_ERR_M0_TOO_SMALL) res_out.msg = "m0 or more Ritz values inside a contour";
        if (rstatus == NLF_ERR_NOT_CONVERGED) res_out.msg = "not converged within max_iter";
        if (rstatus == NLF_SPURIOUS) res_out.msg = "spurious Ritz values inside a contour (inside_out = 2)";
    } catch (const nlf::Error& e) {
        res_out.status = e.status;
        res_out.msg = e.msg;
    } catch (const std::exception& e) {
        res_out.status = NLF_ERR_DEVICE;
        res_out.msg = e.what();
    }
    return res_out;
}

}  // namespace

// =============================================================================== C ABI

#define NLF_TRY(h, ...)                                                         \
    try {                                                                       \
        __VA_ARGS__                                                             \
    } catch (const nlf::Error& e_) {                                            \
        g_last_error = e_.msg;                                                  \
        if (h) (h)->last_error = e_.msg;                                        \
        return (nlfeast_status)e_.status;                                       \
    } catch (const std::exception& e_) {                                        \
        g_last_error = e_.what();                                               \
        if (h) (h)->last_error = e_.what();                                     \
        return NLF_ERR_DEVICE;                                                  \
    }

extern "C" {

nlfeast_status nlfeast_create(nlfeast_handle* out, int64_t n, int device, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(out && n > 0 && n <= 8192, NLF_ERR_ARG, "create: need 0 < n <= 8192");
        int count = 0;
        NLF_HIP(hipGetDeviceCount(&count));
        NLF_REQUIRE(device >= 0 && device < count, NLF_ERR_ARG, "create: bad device index");
        NLF_HIP(hipSetDevice(device));
        h = new nlfeast_ctx();
        h->n = n;
        h->device = device;
        h->stream = (hipStream_t)stream;
        *out = h;
        return NLF_OK;
    })
}

void nlfeast_destroy(nlfeast_handle h) { delete h; }

const char* nlfeast_last_error(nlfeast_handle h) {
    return h ? h->last_error.c_str() : g_last_error.c_str();
}

nlfeast_status nlfeast_set_coeffs(nlfeast_handle h, int32_t J, const int32_t* fkind,
                                  const double* fparam, const void* const* A_dev, int64_t lda) {
    NLF_TRY(h, {
        NLF_REQUIRE(h, NLF_ERR_ARG, "null handle");
        NLF_REQUIRE(J >= 1 && J <= 8 && fkind && fparam && A_dev && lda >= h->n, NLF_ERR_ARG,
                    "set_coeffs: need 1 <= J <= 8, non-null arrays, lda >= n");
        std::vector<Term> terms(J);
        for (int j = 0; j < J; ++j) {
            NLF_REQUIRE(fkind[j] == NLF_F_POW || fkind[j] == NLF_F_EXP || fkind[j] == NLF_F_USER, NLF_ERR_ARG,
                        "set_coeffs: bad kind");
            if (fkind[j] == NLF_F_POW)
                NLF_REQUIRE(fparam[j] >= 0 && fparam[j] <= 16 && fparam[j] == std::floor(fparam[j]),
                            NLF_ERR_ARG, "set_coeffs: power must be an integer in 0..16");
            NLF_REQUIRE(std::isfinite(fparam[j]), NLF_ERR_ARG, "set_coeffs: parameter not finite");
            NLF_REQUIRE(A_dev[j], NLF_ERR_ARG, "set_coeffs: null matrix");
            terms[j] = Term{fkind[j], fparam[j], fkind[j] == NLF_F_USER ? &h->ufn : nullptr, j};
        }
        h->J = J;
        h->terms = terms;
        h->A.assign(J, nullptr);
        for (int j = 0; j < J; ++j) h->A[j] = (const z128*)A_dev[j];
        h->lda = lda;
        h->ident.assign(J, 0);
        h->ident_known = false;
        h->factors_valid = false;
        return NLF_OK;
    })
}

nlfeast_status nlfeast_set_user_function(nlfeast_handle h, nlfeast_user_fn fn, void* user) {
    NLF_TRY(h, {
        NLF_REQUIRE(h, NLF_ERR_ARG, "null handle");
        h->ufn.fn = fn;
        h->ufn.user = user;
        h->ufn.failed.store(0);
        h->factors_valid = false;
        h->drop_graph();
        return NLF_OK;
    })
}

nlfeast_status nlfeast_set_contour(nlfeast_handle h, int32_t nreg, const double* centre,
                                   const double* semi_axes, const int32_t* n_nodes,
                                   const int32_t* m0, int32_t quad_rule) {
    NLF_TRY(h, {
        NLF_REQUIRE(h, NLF_ERR_ARG, "null handle");
        NLF_REQUIRE(nreg >= 1 && centre && semi_axes && n_nodes && m0, NLF_ERR_ARG,
                    "set_contour: need nreg >= 1 and non-null arrays");
        NLF_REQUIRE(quad_rule == NLF_QUAD_GAUSS_LEGENDRE || quad_rule == NLF_QUAD_TRAPEZOID,
                    NLF_ERR_ARG, "set_contour: bad quadrature rule");
        std::vector<nlfeast_ctx::Region> regs(nreg);
        for (int r = 0; r < nreg; ++r) {
            NLF_REQUIRE(semi_axes[2 * r] > 0 && semi_axes[2 * r + 1] > 0, NLF_ERR_ARG,
                        "set_contour: semi-axes must be positive");
            NLF_REQUIRE(n_nodes[r] >= 1 && n_nodes[r] <= 256, NLF_ERR_ARG, "set_contour: 1 <= n_nodes <= 256");
            NLF_REQUIRE(m0[r] >= 1 && m0[r] <= h->n && m0[r] <= 512, NLF_ERR_ARG,
                        "set_contour: 1 <= m0 <= min(n, 512)");
            regs[r].E = Ellipse{cplx(centre[2 * r], centre[2 * r + 1]), semi_axes[2 * r], semi_axes[2 * r + 1]};
            regs[r].nc = n_nodes[r];
            regs[r].m0 = m0[r];
            quadrature(regs[r].E, regs[r].nc, quad_rule, regs[r].z, regs[r].w);
        }
        h->regions = regs;
        h->quad_rule = quad_rule;
        h->factors_valid = false;
        return NLF_OK;
    })
}

nlfeast_status nlfeast_workspace_size(nlfeast_handle h, const nlfeast_options* opt, size_t* bytes) {
    NLF_TRY(h, {
        NLF_REQUIRE(h && opt && bytes, NLF_ERR_ARG, "workspace_size: null argument");
        NLF_REQUIRE(!h->regions.empty() && h->J > 0, NLF_ERR_STATE,
                    "workspace_size: call set_coeffs and set_contour first");
        *bytes = make_layout(h, opt->precision, takes_contour_route(h->terms, opt->reduced_solver)).total;
        return NLF_OK;
    })
}

nlfeast_status nlfeast_set_profiling(nlfeast_handle h, int32_t on) {
    if (!h) return NLF_ERR_ARG;
    h->profiling = on != 0;
    return NLF_OK;
}

nlfeast_status nlfeast_get_profile(nlfeast_handle h, int64_t* launches, double* milliseconds,
                                   double* flops, double* bytes) {
    if (!h) return NLF_ERR_ARG;
    for (int c = 0; c < NLF_K_COUNT; ++c) {
        if (launches) launches[c] = h->prof.launches[c];
        if (milliseconds) milliseconds[c] = h->prof.ms[c];
        if (flops) flops[c] = h->prof.flops[c];
        if (bytes) bytes[c] = h->prof.bytes[c];
    }
    return NLF_OK;
}

// nlfeast_solve (adj = false) and nlfeast_solve_left (adj = true).
static nlfeast_status solve_impl(nlfeast_handle h, const nlfeast_options* opt, void* ws, size_t ws_bytes,
                                 const void* X0_dev, void* X_dev_out, double* lambda_out, double* resid_out,
                                 int32_t* inside_out, int32_t* m_out, int32_t* iters_out, bool adj) {
    NLF_TRY(h, {
        NLF_REQUIRE(h && opt, NLF_ERR_ARG, "solve: null argument");
        NLF_REQUIRE(!h->regions.empty() && h->J > 0, NLF_ERR_STATE,
                    "solve: call set_coeffs and set_contour first");
        NLF_REQUIRE(ws && X_dev_out && lambda_out && resid_out && inside_out && m_out && iters_out,
                    NLF_ERR_ARG, "solve: null output or workspace");
        NLF_REQUIRE(opt->precision == NLF_PREC_FP64 || opt->precision == NLF_PREC_FP32_REFINE,
                    NLF_ERR_ARG, "solve: bad precision");
        NLF_REQUIRE(opt->tol > 0 && opt->max_iter >= 1, NLF_ERR_ARG, "solve: need tol > 0, max_iter >= 1");
        NLF_REQUIRE(opt->lu_streams >= 0 && opt->lu_streams <= 4, NLF_ERR_ARG, "solve: lu_streams in 0..4");
        NLF_REQUIRE(opt->panel_width == 0 || (opt->panel_width >= 4 && opt->panel_width <= 32), NLF_ERR_ARG,
                    "solve: panel_width 0 or 4..32");
        NLF_REQUIRE((opt->region_streams == 0 || opt->region_streams == 1) && (opt->graph == 0 || opt->graph == 1) &&
                        (opt->autotune == 0 || opt->autotune == 1),
                    NLF_ERR_ARG, "solve: region_streams, graph and autotune are 0 or 1");
        NLF_REQUIRE(opt->lookahead >= -1 && opt->lookahead <= 1 && opt->reduced_solver >= 0 && opt->reduced_solver <= 3,
                    NLF_ERR_ARG, "solve: lookahead in -1..1, reduced_solver in 0..3");
        // look-ahead streams inside node groups on separate streams: the process has ended in a
        // segmentation fault with both on (graph-captured factorisation, delay8192) and the cause
        // is not identified, so the pair is refused (each alone is unaffected)
        NLF_REQUIRE(!(opt->lookahead > 0 && opt->lu_streams > 1), NLF_ERR_ARG,
                    "solve: lookahead = 1 together with lu_streams > 1 is not supported");
        bool has_user = false;
        for (const Term& t : h->terms) has_user = has_user || t.kind == NLF_F_USER;
        NLF_REQUIRE(!has_user || h->ufn.fn, NLF_ERR_STATE,
                    "solve: a term of kind NLF_F_USER needs nlfeast_set_user_function first");
        h->ufn.failed.store(0);
        const Layout L = make_layout(h, opt->precision, takes_contour_route(h->terms, opt->reduced_solver));
        NLF_REQUIRE(ws_bytes >= L.total, NLF_ERR_NOMEM, "solve: workspace too small");
        NLF_HIP(hipSetDevice(h->device));
        hipStream_t s = h->stream;
        const int64_t n = h->n;
        const int J = h->J;
        const bool p32 = opt->precision == NLF_PREC_FP32_REFINE;
        if (h->profiling) h->prof.reset();
        ProfilerGuard pg(h->profiling ? &h->prof : nullptr);
        // which coefficient matrices are exactly the identity (once per set_coeffs: the A_j are
        // borrowed unmodified until the next one)
        if (!h->ident_known) {
            int32_t* flags = at<int32_t>(ws, L.ident);
            identity_flags(s, n, J, h->A.data(), h->lda, flags);
            std::vector<int32_t> f(J);
            NLF_HIP(hipMemcpyAsync(f.data(), flags, sizeof(int32_t) * J, hipMemcpyDeviceToHost, s));
            NLF_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < J; ++j) h->ident[j] = f[j] == 0;
            h->ident_known = true;
        }

        // ---- fixed shifts: assemble and factor T(z_k) once per contour; the regions start
        // from ev_start (the caller's prior work) and wait for ev_factored before Step 4
        if (!h->ev_start) NLF_HIP(hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming));
        if (!h->ev_factored) NLF_HIP(hipEventCreateWithFlags(&h->ev_factored, hipEventDisableTiming));
        NLF_HIP(hipEventRecord(h->ev_start, s));
        hipEvent_t factored = nullptr;
        std::shared_future<void> enqueued;
        struct Joiner {   // joins the factorisation thread on every exit path
            std::thread t;
            ~Joiner() {
                if (t.joinable()) t.join();
            }
        } fthread;
        if (!(h->factors_valid && h->factors_ws == ws && h->factors_prec == opt->precision)) {
            h->factors_valid = false;
            std::vector<cplx> coef((size_t)L.NZ * J);
            int k = 0;
            for (const auto& r : h->regions)
                for (int q = 0; q < r.nc; ++q, ++k)
                    for (int j = 0; j < J; ++j) coef[(size_t)k * J + j] = term_value(h->terms[j], r.z[q]);
            NLF_REQUIRE(!user_failed(h->terms), NLF_ERR_ARG, "solve: the user function reported an error");
            h2d(s, at<void>(ws, L.coef), coef.data(), sizeof(cplx) * coef.size());
            LuTuning tune = fixed_tuning(*opt);
            // tall panels: 16-column panel leaves halve the left-looking re-reads of the leaf
            // kernel (measured at n = 8192 x 24 nodes: factorisation 644 -> 632 ms; no change at
            // n = 4096)
            if (!opt->panel_width && h->n > 4096) tune.panel_width = 16;
            if (opt->autotune) tune = autotuned(h, L, ws, p32, s, *opt);
            if (opt->graph) {
                GraphKey key = graph_key(h, L, ws, opt->precision, tune);
                if (h->graph_segs.empty() || !(h->graph_key == key)) {
                    capture_factorisation(h, L, ws, p32, tune);
                    h->graph_key = key;
                }
            }
            if (h->info_cap < L.NZ) {
                if (h->info_host) NLF_HIP(hipHostFree(h->info_host));
                h->info_host = nullptr;
                h->info_cap = 0;
                NLF_HIP(hipHostMalloc((void**)&h->info_host, sizeof(int32_t) * L.NZ, hipHostMallocDefault));
                h->info_cap = L.NZ;
            }
            // enqueuing the factorisation blocks the host (a graph launch waits for the GPU, and
            // so do eager launches once the queue is full).  With the regions on one stream, it is
            // enqueued from a thread of its own, so that Steps 0-3 (which need no factors) run
            // meanwhile; with concurrent region threads the same overlap measured no gain (the
            // batched eight-region workload: 333-358 ms with it, 341-346 ms without), so it is
            // enqueued here before they start
            auto enqueue = [h, &L, ws, p32, s, tune, opt](Profiler* fp) {
                NLF_HIP(hipSetDevice(h->device));
                ProfilerGuard fpg(fp);
                {
                    ProfScope ps(NLF_PROF_FACTOR, s, 8.0 / 3.0 * (double)h->n * h->n * h->n * L.NZ, 0);
                    if (opt->graph) replay_factorisation(h, s);
                    else factor_all(h, L, ws, p32, s, tune);
                }
                NLF_HIP(hipMemcpyAsync(h->info_host, at<void>(ws, L.info), sizeof(int32_t) * L.NZ,
                                       hipMemcpyDeviceToHost, s));
                NLF_HIP(hipEventRecord(h->ev_factored, s));
            };
            factored = h->ev_factored;
            const bool concurrent_regions = h->regions.size() > 1 && opt->region_streams == 0;
            if (concurrent_regions) {
                enqueue(h->profiling ? &h->prof : nullptr);
            } else {
                if (h->profiling) h->fprof.reset();
                std::shared_ptr<std::promise<void>> done = std::make_shared<std::promise<void>>();
                enqueued = done->get_future().share();
                fthread.t = std::thread([h, enqueue, done] {
                    try {
                        enqueue(h->profiling ? &h->fprof : nullptr);
                        done->set_value();
                    } catch (...) {
                        done->set_exception(std::current_exception());
                    }
                });
            }
        }

        const int nreg = (int)h->regions.size();
        std::vector<RegionOutcome> out(nreg);
        RegionIO io{X0_dev, X_dev_out, lambda_out, resid_out, inside_out, m_out, iters_out,
                    enqueued.valid() ? &enqueued : nullptr};
        const bool concurrent = nreg > 1 && opt->region_streams == 0;
        // region streams: one per region when they run concurrently, else one shared stream
        const int nrs = concurrent ? nreg : 1;
        for (int ri = (int)h->rstream.size(); ri < nrs; ++ri) {
            hipStream_t rs;
            hipEvent_t ev;
            NLF_HIP(hipStreamCreateWithFlags(&rs, hipStreamNonBlocking));
            NLF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            h->rstream.push_back(rs);
            h->rdone.push_back(ev);
            h->rprof.emplace_back(new Profiler());
        }
        for (int ri = 0; ri < nrs; ++ri) NLF_HIP(hipStreamWaitEvent(h->rstream[ri], h->ev_start, 0));
        if (!concurrent) {
            for (int ri = 0; ri < nreg; ++ri) {
                out[ri] = run_region(h, *opt, ws, L, ri, h->rstream[0], h->profiling ? &h->prof : nullptr, io,
                                     factored, nullptr, adj);
                // a hard error ends the sequence; the convergence statuses (spurious values
                // flagged, not converged, m0 too small) leave the later regions to run
                if (out[ri].status != NLF_OK && out[ri].status != NLF_SPURIOUS &&
                    out[ri].status != NLF_ERR_NOT_CONVERGED && out[ri].status != NLF_ERR_M0_TOO_SMALL)
                    break;
            }
            NLF_HIP(hipEventRecord(h->rdone[0], h->rstream[0]));
            NLF_HIP(hipStreamWaitEvent(s, h->rdone[0], 0));
        } else {
            // every region iterates on its own stream and host thread (iteration 0 overlaps the
            // shared factorisation); the caller's stream waits for all of them
            for (int ri = 0; ri < nreg; ++ri) h->rprof[ri]->reset();
            std::vector<std::thread> threads;
            threads.reserve(nreg);
            // the regions' pending reduced-solve work (sum of m0^3 over the regions still
            // iterating), by which they share the host threads
            auto work = [&](int ri) { const int64_t m = h->regions[ri].m0; return m * m * m; };
            std::atomic<int64_t> active{0};
            for (int ri = 0; ri < nreg; ++ri) active.fetch_add(work(ri));
            for (int ri = 0; ri < nreg; ++ri)
                threads.emplace_back([&, ri] {
                    if (hipSetDevice(h->device) != hipSuccess) {
                        out[ri].status = NLF_ERR_DEVICE;
                        out[ri].msg = "hipSetDevice failed in a region thread";
                        active.fetch_sub(work(ri));
                        return;
                    }
                    out[ri] = run_region(h, *opt, ws, L, ri, h->rstream[ri],
                                         h->profiling ? h->rprof[ri].get() : nullptr, io, factored, &active, adj);
                    active.fetch_sub(work(ri));
                });
            for (auto& t : threads) t.join();
            for (int ri = 0; ri < nreg; ++ri) {
                NLF_HIP(hipEventRecord(h->rdone[ri], h->rstream[ri]));
                NLF_HIP(hipStreamWaitEvent(s, h->rdone[ri], 0));
            }
            NLF_HIP(hipStreamSynchronize(s));
            if (h->profiling)
                for (int ri = 0; ri < nreg; ++ri) {
                    h->rprof[ri]->collect();
                    h->prof.merge(*h->rprof[ri]);
                }
        }
        if (fthread.t.joinable()) {
            fthread.t.join();
            enqueued.get();   // rethrows the factorisation thread's error
        }
        NLF_HIP(hipStreamSynchronize(s));
        if (h->profiling) {
            h->prof.collect();
            if (enqueued.valid()) {
                h->fprof.collect();
                h->prof.merge(h->fprof);
            }
        }
        // a hard error (device, argument) wins over the convergence statuses
        int status = NLF_OK;
        std::string msg;
        if (factored) {
            // regions that stopped before Step 4 never looked at the pivots
            for (int q = 0; q < L.NZ; ++q)
                if (h->info_host[q] != 0) {
                    status = NLF_ERR_SINGULAR;
                    msg = "solve: T(z_k) is singular at node " + std::to_string(q) + " (exact zero pivot " +
                          std::to_string(h->info_host[q]) + ")";
                    break;
                }
            if (status == NLF_OK) {
                h->factors_valid = true;
                h->factors_ws = ws;
                h->factors_prec = opt->precision;
            }
        }
        // precedence: hard errors, then NOT_CONVERGED / M0_TOO_SMALL, then SPURIOUS, then OK
        auto rank = [](int st) {
            if (st == NLF_OK) return 0;
            if (st == NLF_SPURIOUS) return 1;
            if (st == NLF_ERR_NOT_CONVERGED || st == NLF_ERR_M0_TOO_SMALL) return 2;
            return 3;
        };
        for (int ri = 0; ri < nreg; ++ri) {
            const int st = out[ri].status;
            const bool keep_hard = rank(status) == 3;
            if (rank(st) > rank(status) || (rank(st) == 2 && rank(status) == 2 && !keep_hard)) {
                status = st;
                msg = out[ri].msg;
            }
        }
        if (status != NLF_OK) h->last_error = msg;
        return (nlfeast_status)status;
    })
}

nlfeast_status nlfeast_solve(nlfeast_handle h, const nlfeast_options* opt, void* ws,
                             size_t ws_bytes, const void* X0_dev, void* X_dev_out,
                             double* lambda_out, double* resid_out, int32_t* inside_out,
                             int32_t* m_out, int32_t* iters_out) {
    return solve_impl(h, opt, ws, ws_bytes, X0_dev, X_dev_out, lambda_out, resid_out, inside_out, m_out, iters_out,
                      false);
}

nlfeast_status nlfeast_solve_left(nlfeast_handle h, const nlfeast_options* opt, void* ws,
                                  size_t ws_bytes, const void* Y0_dev, void* Y_dev_out,
                                  double* lambda_out, double* resid_out, int32_t* inside_out,
                                  int32_t* m_out, int32_t* iters_out) {
    return solve_impl(h, opt, ws, ws_bytes, Y0_dev, Y_dev_out, lambda_out, resid_out, inside_out, m_out, iters_out,
                      true);
}

// ------------------------------------------------------------------ step-level entry points

static hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// The step-level calls take built-in terms only: a caller-supplied function lives on a handle.
static void require_builtin_kinds(int J, const int32_t* fkind, const char* who) {
    for (int j = 0; j < J; ++j)
        NLF_REQUIRE(fkind[j] == NLF_F_POW || fkind[j] == NLF_F_EXP, NLF_ERR_ARG,
                    std::string(who) + ": term kinds are NLF_F_POW or NLF_F_EXP");
}

nlfeast_status nlf_assemble(int64_t n, int32_t J, const int32_t* fkind, const double* fparam,
                            const void* const* A_dev, int64_t lda, int32_t nz, const double* z,
                            void* T64_dev, void* T32_dev, int64_t ldt, int64_t strideT, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && J >= 1 && J <= 8 && fkind && fparam && A_dev && lda >= n && nz >= 1 && z &&
                        (T64_dev || T32_dev) && ldt >= n && strideT >= ldt * n,
                    NLF_ERR_ARG, "nlf_assemble: bad arguments");
        require_builtin_kinds(J, fkind, "nlf_assemble");
        std::vector<cplx> coef((size_t)nz * J);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < J; ++j)
                coef[(size_t)k * J + j] = term_value(Term{fkind[j], fparam[j]}, cplx(z[2 * k], z[2 * k + 1]));
        z128* coef_d = nullptr;
        NLF_HIP(hipMallocAsync((void**)&coef_d, sizeof(cplx) * coef.size(), as_stream(stream)));
        h2d(as_stream(stream), coef_d, coef.data(), sizeof(cplx) * coef.size());
        assemble(as_stream(stream), n, J, (const z128* const*)A_dev, lda, nz, coef_d, (z128*)T64_dev,
                 (z64*)T32_dev, ldt, strideT);
        NLF_HIP(hipFreeAsync(coef_d, as_stream(stream)));
        NLF_HIP(hipStreamSynchronize(as_stream(stream)));
        return NLF_OK;
    })
}

nlfeast_status nlf_getrf_batched(int32_t dtype, int64_t n, int32_t batch, void* A_dev, int64_t lda,
                                 int64_t strideA, int32_t* ipiv_dev, int32_t* perm_dev,
                                 int32_t* info_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && n <= 8192 && batch >= 1 && A_dev && lda >= n && strideA >= lda * n &&
                        ipiv_dev && info_dev && (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrf_batched: bad arguments");
        hipStream_t s = as_stream(stream);
        int32_t* list = nullptr;
        NLF_HIP(hipMallocAsync((void**)&list, sizeof(int32_t) * getrf_scratch_ints(n, batch), s));
        if (dtype == NLF_C128)
            getrf<double>(s, n, batch, (z128*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list);
        else
            getrf<float>(s, n, batch, (z64*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list);
        NLF_HIP(hipFreeAsync(list, s));
        return NLF_OK;
    })
}

nlfeast_status nlf_getrf_batched_blocked(int32_t dtype, int64_t n, int32_t batch, void* A_dev,
                                         int64_t lda, int64_t strideA, int32_t* ipiv_dev,
                                         int32_t* perm_dev, int32_t* info_dev, void* dinv_dev,
                                         void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && n <= 8192 && batch >= 1 && A_dev && lda >= n && strideA >= lda * n &&
                        ipiv_dev && info_dev && dinv_dev && (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrf_batched_blocked: bad arguments");
        hipStream_t s = as_stream(stream);
        int32_t* list = nullptr;
        void* tmp = nullptr;
        const size_t es = dtype == NLF_C128 ? 16 : 8;
        NLF_HIP(hipMallocAsync((void**)&list, sizeof(int32_t) * getrf_scratch_ints(n, batch), s));
        NLF_HIP(hipMallocAsync(&tmp, es * getrf_tmp_elems(n) * batch, s));
        TrsmClassGuard tg(NLF_PROF_TRSM);
        if (dtype == NLF_C128)
            getrf<double>(s, n, batch, (z128*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list,
                          (z128*)dinv_dev, (z128*)tmp);
        else
            getrf<float>(s, n, batch, (z64*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list,
                         (z64*)dinv_dev, (z64*)tmp);
        NLF_HIP(hipFreeAsync(tmp, s));
        NLF_HIP(hipFreeAsync(list, s));
        return NLF_OK;
    })
}

nlfeast_status nlf_getrs_batched(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                 const void* LU_dev, int64_t lda, int64_t strideA,
                                 const int32_t* perm_dev, const void* B_dev, int64_t ldb,
                                 int64_t strideB, void* X_dev, int64_t ldx, int64_t strideX,
                                 void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && nrhs >= 1 && batch >= 1 && LU_dev && perm_dev && B_dev && X_dev &&
                        lda >= n && ldb >= n && ldx >= n && strideB >= 0 && strideX >= ldx * nrhs &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrs_batched: bad arguments");
        TrsmClassGuard tg(NLF_PROF_SOLVE);
        if (dtype == NLF_C128)
            getrs<double>(as_stream(stream), n, nrhs, batch, (const z128*)LU_dev, lda, strideA, perm_dev,
                          (const z128*)B_dev, ldb, strideB, (z128*)X_dev, ldx, strideX);
        else
            getrs<float>(as_stream(stream), n, nrhs, batch, (const z64*)LU_dev, lda, strideA, perm_dev,
                         (const z64*)B_dev, ldb, strideB, (z64*)X_dev, ldx, strideX);
        return NLF_OK;
    })
}

int64_t nlf_lu_inverse_elems(int64_t n) { return n > 0 ? lu_inverse_elems(n) : 0; }

nlfeast_status nlf_lu_block_inverses(int32_t dtype, int64_t n, int32_t batch, const void* LU_dev,
                                     int64_t lda, int64_t strideA, void* dinv_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && batch >= 1 && LU_dev && dinv_dev && lda >= n && strideA >= lda * n &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_lu_block_inverses: bad arguments");
        TrsmClassGuard tg(NLF_PROF_TRSM);
        if (dtype == NLF_C128)
            lu_block_inverses<double>(as_stream(stream), n, batch, (const z128*)LU_dev, lda, strideA, (z128*)dinv_dev);
        else
            lu_block_inverses<float>(as_stream(stream), n, batch, (const z64*)LU_dev, lda, strideA, (z64*)dinv_dev);
        return NLF_OK;
    })
}

nlfeast_status nlf_getrs_batched_inv(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                     const void* LU_dev, int64_t lda, int64_t strideA,
                                     const int32_t* perm_dev, const void* dinv_dev,
                                     const void* B_dev, int64_t ldb, int64_t strideB, void* X_dev,
                                     int64_t ldx, int64_t strideX, void* tmp_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && nrhs >= 1 && batch >= 1 && LU_dev && perm_dev && dinv_dev && B_dev && X_dev &&
                        tmp_dev && lda >= n && ldb >= n && ldx >= n && strideB >= 0 && strideX >= ldx * nrhs &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrs_batched_inv: bad arguments");
        TrsmClassGuard tg(NLF_PROF_SOLVE);
        if (dtype == NLF_C128)
            getrs_inv<double>(as_stream(stream), n, nrhs, batch, (const z128*)LU_dev, lda, strideA, perm_dev,
                              (const z128*)dinv_dev, (const z128*)B_dev, ldb, strideB, (z128*)X_dev, ldx, strideX,
                              (z128*)tmp_dev);
        else
            getrs_inv<float>(as_stream(stream), n, nrhs, batch, (const z64*)LU_dev, lda, strideA, perm_dev,
                             (const z64*)dinv_dev, (const z64*)B_dev, ldb, strideB, (z64*)X_dev, ldx, strideX,
                             (z64*)tmp_dev);
        return NLF_OK;
    })
}

nlfeast_status nlf_getrs_batched_inv_adjoint(int32_t dtype, int64_t n, int32_t nrhs, int32_t batch,
                                             const void* LU_dev, int64_t lda, int64_t strideA,
                                             const int32_t* perm_dev, const void* dinv_dev, const void* B_dev,
                                             int64_t ldb, int64_t strideB, void* Z_dev, void* X_dev, int64_t ldx,
                                             int64_t strideX, void* tmp_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && nrhs >= 1 && batch >= 1 && LU_dev && perm_dev && dinv_dev && B_dev && Z_dev && X_dev &&
                        tmp_dev && lda >= n && ldb >= n && ldx >= n && strideB >= 0 && strideX >= ldx * nrhs &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrs_batched_inv_adjoint: bad arguments");
        const size_t es = dtype == NLF_C128 ? 16 : 8;
        const char* z0 = (const char*)Z_dev;
        const char* z1 = z0 + es * (size_t)n * nrhs * batch;
        const char* x0 = (const char*)X_dev;
        const char* x1 = x0 + es * ((size_t)(batch - 1) * strideX + (size_t)ldx * nrhs);
        NLF_REQUIRE(x1 <= z0 || z1 <= x0, NLF_ERR_ARG, "nlf_getrs_batched_inv_adjoint: X overlaps Z");
        TrsmClassGuard tg(NLF_PROF_SOLVE);
        if (dtype == NLF_C128)
            getrs_inv_adjoint<double>(as_stream(stream), n, nrhs, batch, (const z128*)LU_dev, lda, strideA, perm_dev,
                                      (const z128*)dinv_dev, (const z128*)B_dev, ldb, strideB, (z128*)Z_dev,
                                      (z128*)X_dev, ldx, strideX, (z128*)tmp_dev);
        else
            getrs_inv_adjoint<float>(as_stream(stream), n, nrhs, batch, (const z64*)LU_dev, lda, strideA, perm_dev,
                                     (const z64*)dinv_dev, (const z64*)B_dev, ldb, strideB, (z64*)Z_dev,
                                     (z64*)X_dev, ldx, strideX, (z64*)tmp_dev);
        return NLF_OK;
    })
}

nlfeast_status nlf_gemm_batched(int32_t dtype, char opA, char opB, int64_t M, int64_t N, int64_t K,
                                const double* alpha, const void* A_dev, int64_t lda, int64_t strideA,
                                const void* B_dev, int64_t ldb, int64_t strideB, const double* beta,
                                void* C_dev, int64_t ldc, int64_t strideC, int32_t batch, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        const bool cA = opA == 'C' || opA == 'c';
        NLF_REQUIRE((opA == 'N' || opA == 'n' || cA) && (opB == 'N' || opB == 'n'), NLF_ERR_ARG,
                    "nlf_gemm_batched: opA in {N, C}, opB = N");
        NLF_REQUIRE(M >= 0 && N >= 0 && K >= 0 && batch >= 1 && alpha && beta && C_dev && ldc >= M &&
                        (K == 0 || (A_dev && B_dev && ldb >= K && lda >= (cA ? K : M))) &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_gemm_batched: bad arguments");
        hipStream_t s = as_stream(stream);
        if (dtype == NLF_C128)
            gemm<double>(s, cA, M, N, K, z128(alpha[0], alpha[1]), (const z128*)A_dev, lda, strideA,
                         (const z128*)B_dev, ldb, strideB, z128(beta[0], beta[1]), (z128*)C_dev, ldc,
                         strideC, batch);
        else
            gemm<float>(s, cA, M, N, K, z64((float)alpha[0], (float)alpha[1]), (const z64*)A_dev, lda,
                        strideA, (const z64*)B_dev, ldb, strideB, z64((float)beta[0], (float)beta[1]),
                        (z64*)C_dev, ldc, strideC, batch);
        return NLF_OK;
    })
}

nlfeast_status nlf_gemm_batched_tile(int32_t dtype, char opA, int64_t M, int64_t N, int64_t K,
                                     const double* alpha, const void* A_dev, int64_t lda,
                                     int64_t strideA, const void* B_dev, int64_t ldb,
                                     int64_t strideB, const double* beta, void* C_dev, int64_t ldc,
                                     int64_t strideC, int32_t batch, int32_t tm, int32_t tn,
                                     void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        const bool cA = opA == 'C' || opA == 'c';
        NLF_REQUIRE(M >= 0 && N >= 0 && K >= 0 && batch >= 1 && alpha && beta && C_dev && ldc >= M &&
                        (K == 0 || (A_dev && B_dev && ldb >= K && lda >= (cA ? K : M))) &&
                        (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_gemm_batched_tile: bad arguments");
        const bool ok = (tm == 1 && tn == 1) || (tm == 2 && tn == 1) || (tm == 2 && tn == 2) || (tm == 4 && tn == 2) ||
                        (tm == 4 && tn == 4 && dtype == NLF_C64) || (tm == 4 && tn == 1 && dtype == NLF_C64);
        NLF_REQUIRE(ok, NLF_ERR_ARG, "nlf_gemm_batched_tile: tile not compiled");
        GemmConfig c;
        c.tm = tm;
        c.tn = tn;
        hipStream_t s = as_stream(stream);
        if (dtype == NLF_C128)
            gemm<double>(s, cA, M, N, K, z128(alpha[0], alpha[1]), (const z128*)A_dev, lda, strideA,
                         (const z128*)B_dev, ldb, strideB, z128(beta[0], beta[1]), (z128*)C_dev, ldc,
                         strideC, batch, nullptr, 0, &c);
        else
            gemm<float>(s, cA, M, N, K, z64((float)alpha[0], (float)alpha[1]), (const z64*)A_dev, lda,
                        strideA, (const z64*)B_dev, ldb, strideB, z64((float)beta[0], (float)beta[1]),
                        (z64*)C_dev, ldc, strideC, batch, nullptr, 0, &c);
        return NLF_OK;
    })
}

nlfeast_status nlf_block_residual(int64_t n, int32_t m, int32_t J, const int32_t* fkind,
                                  const double* fparam, const void* const* A_dev, int64_t lda,
                                  const void* X_dev, int64_t ldx, const double* lambda, void* R_dev,
                                  int64_t ldr, double* norms_dev, void* ws_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && m >= 1 && J >= 1 && J <= 8 && fkind && fparam && A_dev && lda >= n && X_dev &&
                        ldx >= n && lambda && R_dev && ldr >= n && norms_dev && ws_dev,
                    NLF_ERR_ARG, "nlf_block_residual: bad arguments");
        require_builtin_kinds(J, fkind, "nlf_block_residual");
        hipStream_t s = as_stream(stream);
        z128* XF = (z128*)ws_dev;     // X f_j(Lambda), one term at a time
        std::vector<cplx> f((size_t)m);
        ProfScope ps(NLF_PROF_RESIDUAL, s, 8.0 * n * n * m * J, 16.0 * n * n * J);
        for (int j = 0; j < J; ++j) {
            // R += A_j (X diag f_j): scale columns through a diagonal GEMM-free path: copy then
            // fold the scaling into the GEMM's B operand by one small diagonal product per column
            std::vector<cplx> D((size_t)m * m, 0.0);
            for (int c = 0; c < m; ++c)
                D[c + (size_t)c * m] = term_value(Term{fkind[j], fparam[j]}, cplx(lambda[2 * c], lambda[2 * c + 1]));
            z128* Dd = nullptr;
            NLF_HIP(hipMallocAsync((void**)&Dd, sizeof(cplx) * m * m, s));
            h2d(s, Dd, D.data(), sizeof(cplx) * m * m);
            gemm<double>(s, false, n, m, m, z128(1, 0), (const z128*)X_dev, ldx, 0, Dd, m, 0, z128(0, 0), XF, n,
                         0, 1);
            gemm<double>(s, false, n, m, n, z128(1, 0), (const z128*)A_dev[j], lda, 0, XF, n, 0,
                         z128(j == 0 ? 0.0 : 1.0, 0), (z128*)R_dev, ldr, 0, 1);
            NLF_HIP(hipFreeAsync(Dd, s));
        }
        col_norms(s, n, m, (const z128*)R_dev, ldr, norms_dev);
        NLF_HIP(hipStreamSynchronize(s));
        return NLF_OK;
    })
}

nlfeast_status nlf_accumulate(int64_t n, int32_t m, int32_t nz, const void* X_dev, const void* Y_dev,
                              const double* z, const double* omega, const double* lambda, void* Q_dev,
                              void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && m >= 1 && nz >= 1 && X_dev && Y_dev && z && omega && lambda && Q_dev,
                    NLF_ERR_ARG, "nlf_accumulate: bad arguments");
        hipStream_t s = as_stream(stream);
        std::vector<cplx> rho(m), coef((size_t)nz * m);
        for (int i = 0; i < m; ++i) {
            const cplx l(lambda[2 * i], lambda[2 * i + 1]);
            cplx rs = 0.0;
            for (int k = 0; k < nz; ++k) {
                const cplx c = cplx(omega[2 * k], omega[2 * k + 1]) / (cplx(z[2 * k], z[2 * k + 1]) - l);
                coef[(size_t)k * m + i] = c;
                rs += c;
            }
            rho[i] = rs;
        }
        z128* buf = nullptr;
        NLF_HIP(hipMallocAsync((void**)&buf, sizeof(cplx) * (m + coef.size()), s));
        h2d(s, buf, rho.data(), sizeof(cplx) * m);
        h2d(s, buf + m, coef.data(), sizeof(cplx) * coef.size());
        accumulate(s, n, m, nz, (const z128*)X_dev, (const z128*)Y_dev, n * m, buf, buf + m, (z128*)Q_dev);
        NLF_HIP(hipFreeAsync(buf, s));
        NLF_HIP(hipStreamSynchronize(s));
        return NLF_OK;
    })
}

int64_t nlf_orth_workspace(int64_t n, int32_t m) {
    return 2 * n * m + 2 * (int64_t)m * m + std::max<int64_t>(64 * (int64_t)m * m, 1 << 16) +
           householder_scratch_elems(m);
}

nlfeast_status nlf_orthonormalize(int64_t n, int32_t m, void* Q_dev, void* ws_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && m >= 1 && m <= n && Q_dev && ws_dev, NLF_ERR_ARG, "nlf_orthonormalize: bad arguments");
        z128* w = (z128*)ws_dev;
        z128* QT = w;
        z128* G = QT + n * m;
        z128* Rd = G + (int64_t)m * m;
        z128* sp = Rd + (int64_t)m * m;
        const int64_t spn = std::max<int64_t>(64 * (int64_t)m * m, 1 << 16);
        z128* V = sp + spn;
        z128* hh = V + n * m;
        orthonormalize(as_stream(stream), n, m, (z128*)Q_dev, QT, G, Rd, sp, spn, V, hh);
        NLF_HIP(hipStreamSynchronize(as_stream(stream)));
        return NLF_OK;
    })
}

int64_t nlf_project_workspace(int64_t n, int32_t m, int32_t J) {
    return std::max<int64_t>(std::max<int64_t>(64 * (int64_t)m * m * J, 8 * n * (int64_t)m), 1 << 16);
}

nlfeast_status nlf_project(int64_t n, int32_t m, int32_t J, const void* const* A_dev, int64_t lda,
                           const void* Q_dev, void* W_dev, void* Ahat_dev, void* ws_dev, void* stream) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(n > 0 && m >= 1 && J >= 1 && A_dev && lda >= n && Q_dev && W_dev && Ahat_dev && ws_dev,
                    NLF_ERR_ARG, "nlf_project: bad arguments");
        project(as_stream(stream), n, m, J, (const z128* const*)A_dev, lda, (const z128*)Q_dev, (z128*)W_dev,
                (z128*)Ahat_dev, (z128*)ws_dev, nlf_project_workspace(n, m, J));
        return NLF_OK;
    })
}

nlfeast_status nlf_quadrature(double cre, double cim, double a, double b, int32_t nc, int32_t quad_rule,
                              double* z, double* omega) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        NLF_REQUIRE(a > 0 && b > 0 && nc >= 1 && z && omega && (quad_rule == 0 || quad_rule == 1),
                    NLF_ERR_ARG, "nlf_quadrature: bad arguments");
        std::vector<cplx> zz, ww;
        quadrature(Ellipse{cplx(cre, cim), a, b}, nc, quad_rule, zz, ww);
        for (int k = 0; k < nc; ++k) {
            z[2 * k] = zz[k].real();
            z[2 * k + 1] = zz[k].imag();
            omega[2 * k] = ww[k].real();
            omega[2 * k + 1] = ww[k].imag();
        }
        return NLF_OK;
    })
}

// Shared body of nlf_reduced_solve and nlf_reduced_solve_ex.
static void reduced_solve_c(int32_t m, int32_t J, const int32_t* fkind, const double* fparam, const UserFunction* uf,
                            int32_t method, const double* Ahat, double cre, double cim, double a, double b,
                            int32_t m_keep, const double* avoid, int32_t n_avoid, double* lambda_out, double* Y_out,
                            int32_t* found_out, const char* who) {
    NLF_REQUIRE(m >= 1 && J >= 1 && J <= 8 && fkind && fparam && Ahat && a > 0 && b > 0 && m_keep >= 1 &&
                    lambda_out && Y_out && method >= 0 && method <= 3,
                NLF_ERR_ARG, std::string(who) + ": bad arguments");
    std::vector<Term> terms(J);
    bool user = false;
    for (int j = 0; j < J; ++j) {
        NLF_REQUIRE(fkind[j] == NLF_F_POW || fkind[j] == NLF_F_EXP || (uf && fkind[j] == NLF_F_USER), NLF_ERR_ARG,
                    std::string(who) + ": bad term kind");
        terms[j] = Term{fkind[j], fparam[j], fkind[j] == NLF_F_USER ? uf : nullptr, j};
        user = user || fkind[j] == NLF_F_USER;
    }
    NLF_REQUIRE(!user || uf->fn, NLF_ERR_ARG, std::string(who) + ": NLF_F_USER terms need a function");
    bool poly = true;
    for (const Term& t : terms) poly = poly && t.kind == NLF_F_POW;
    NLF_REQUIRE(!(user || (method != 2 && !poly)) || m_keep <= m, NLF_ERR_ARG,
                std::string(who) + ": the contour-integral solve needs m_keep <= m");
    std::vector<cplx> av;
    for (int i = 0; avoid && i < n_avoid; ++i) av.push_back(cplx(avoid[2 * i], avoid[2 * i + 1]));
    ReducedResult rr = reduced_solve(m, terms, (const cplx*)Ahat, Ellipse{cplx(cre, cim), a, b}, m_keep,
                                     av.empty() ? nullptr : &av, method);
    NLF_REQUIRE(!user_failed(terms), NLF_ERR_ARG, std::string(who) + ": the user function reported an error");
    NLF_REQUIRE(rr.ok, NLF_ERR_DEVICE, std::string(who) + ": eigen-decomposition failed");
    const int keep = (int)rr.lambda.size();
    for (int q = 0; q < keep; ++q) {
        lambda_out[2 * q] = rr.lambda[q].real();
        lambda_out[2 * q + 1] = rr.lambda[q].imag();
        if (found_out) found_out[q] = rr.found[q];
    }
    std::memcpy(Y_out, rr.Y.data(), sizeof(cplx) * rr.Y.size());
}

nlfeast_status nlf_reduced_solve(int32_t m, int32_t J, const int32_t* fkind, const double* fparam,
                                 const double* Ahat, double cre, double cim, double a, double b,
                                 int32_t m_keep, const double* avoid, int32_t n_avoid,
                                 double* lambda_out, double* Y_out) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        reduced_solve_c(m, J, fkind, fparam, nullptr, 2, Ahat, cre, cim, a, b, m_keep, avoid, n_avoid, lambda_out,
                        Y_out, nullptr, "nlf_reduced_solve");
        return NLF_OK;
    })
}

nlfeast_status nlf_reduced_solve_ex(int32_t m, int32_t J, const int32_t* fkind, const double* fparam,
                                    nlfeast_user_fn fn, void* user, int32_t method, const double* Ahat,
                                    double cre, double cim, double a, double b, int32_t m_keep,
                                    const double* avoid, int32_t n_avoid, double* lambda_out, double* Y_out,
                                    int32_t* found_out) {
    nlfeast_ctx* h = nullptr;
    NLF_TRY(h, {
        UserFunction uf;
        uf.fn = fn;
        uf.user = user;
        reduced_solve_c(m, J, fkind, fparam, &uf, method, Ahat, cre, cim, a, b, m_keep, avoid, n_avoid, lambda_out,
                        Y_out, found_out, "nlf_reduced_solve_ex");
        return NLF_OK;
    })
}

}  // extern "C"
