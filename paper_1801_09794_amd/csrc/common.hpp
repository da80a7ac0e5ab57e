// Shared device/host helpers of the nonlinear FEAST library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace nlf {

// Interleaved complex number of real type R (float or double); layout-compatible with the
// (re, im) pairs of the C ABI.
template <typename R>
struct alignas(2 * sizeof(R)) Cx {
    R re, im;
    __host__ __device__ Cx() = default;
    __host__ __device__ constexpr Cx(R r, R i = R(0)) : re(r), im(i) {}
};

template <typename R>
__host__ __device__ inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ inline Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__host__ __device__ inline R abs1(Cx<R> a) { return fabs(a.re) + fabs(a.im); }
template <typename R>
__host__ __device__ inline R norm2(Cx<R> a) { return a.re * a.re + a.im * a.im; }
// a / b by Smith's scaling (avoids overflow of |b|^2 for large or tiny b)
template <typename R>
__host__ __device__ inline Cx<R> cdiv(Cx<R> a, Cx<R> b) {
    if (fabs(b.re) >= fabs(b.im)) {
        R r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        R r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
// a -= b * c
template <typename R>
__host__ __device__ inline void cfms(Cx<R>& a, Cx<R> b, Cx<R> c) {
    a.re = a.re - b.re * c.re + b.im * c.im;
    a.im = a.im - b.re * c.im - b.im * c.re;
}
// a += b * c
template <typename R>
__host__ __device__ inline void cfma(Cx<R>& a, Cx<R> b, Cx<R> c) {
    a.re = a.re + b.re * c.re - b.im * c.im;
    a.im = a.im + b.re * c.im + b.im * c.re;
}

using z128 = Cx<double>;
using z64 = Cx<float>;

// Error carried from a HIP call up to the C ABI.
struct Error {
    int status;          // nlfeast_status
    std::string msg;
};

#define NLF_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::nlf::Error{3, std::string(#call) + ": " + hipGetErrorString(e_)};     \
    } while (0)

#define NLF_REQUIRE(cond, code, text)                                                     \
    do {                                                                                  \
        if (!(cond)) throw ::nlf::Error{(code), std::string(text)};                       \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The text nlfeast_last_error(NULL) returns for a failed call without a handle.
void record_error(const std::string& msg);

// Kernel classes of the launch profiler (same numbering as nlfeast_kernel_class).
enum ProfClass {
    NLF_PROF_ASSEMBLE = 0, NLF_PROF_LU_GEMM = 1, NLF_PROF_PANEL = 2, NLF_PROF_TRSM = 3,
    NLF_PROF_LASWP = 4, NLF_PROF_SOLVE = 5, NLF_PROF_REFINE = 6, NLF_PROF_RESIDUAL = 7,
    NLF_PROF_ACCUMULATE = 8, NLF_PROF_ORTH = 9, NLF_PROF_PROJECT = 10, NLF_PROF_HOST = 11,
    NLF_PROF_FACTOR = 12, NLF_PROF_AUTOTUNE = 13, NLF_PROF_LU_REC_GEMM = 14, NLF_PROF_REDUCED = 15,
    NLF_PROF_COUNT = 16
};
// Class charged for triangular-solve launches (TRSM inside the factorisation, SOLVE inside
// the per-iteration solves); set by the caller around a group of launches.
int& trsm_class();

// Launch profiling hook: when a Profiler is active on this thread, launches of kernel class
// `cls` are bracketed with HIP events on their stream.
struct Profiler;
Profiler*& active_profiler();
struct ProfScope {
    Profiler* p;
    int cls;
    hipStream_t s;
    double flops, bytes;
    void* ev0;
    ProfScope(int cls, hipStream_t s, double flops, double bytes);
    ~ProfScope();
};

}  // namespace nlf
