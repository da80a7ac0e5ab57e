// nlf_getrf_batched_noalloc: the batched LU of nlf_getrf_batched for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The row-exchange lists that nlf_getrf_batched allocates for the call
// live here in a fixed device array instead.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/nlfeast.h"
#include "common.hpp"
#include "kernels.hpp"

namespace {

// The fixed scratch: NLF_NOALLOC_SCRATCH_INTS int32 per device, held until the process ends.
// getrf writes every list entry it later reads (swaplist_kernel fills all 2 (k2 - k1) slots of
// each matrix before laswp_apply_kernel reads them), so nothing has to be cleared between calls.
static __device__ __align__(256) int32_t scratch[NLF_NOALLOC_SCRATCH_INTS];

std::mutex g_mu;
std::vector<int32_t*> g_dev_ptr;   // per device: scratch's device address (null: not looked up)

// The device address of `scratch` on the current device, looked up once per device with that
// device current.  In host code the array's name is only a stand-in for the symbol.
int32_t* scratch_on_current_device() {
    int dev = -1;
    NLF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev_ptr.size() <= dev) g_dev_ptr.resize(dev + 1, nullptr);
    if (!g_dev_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw nlf::Error{NLF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_dev_ptr[dev] = static_cast<int32_t*>(p);
    }
    return g_dev_ptr[dev];
}

}  // namespace

extern "C" nlfeast_status nlf_getrf_batched_noalloc(int32_t dtype, int64_t n, int32_t batch, void* A_dev,
                                                    int64_t lda, int64_t strideA, int32_t* ipiv_dev,
                                                    int32_t* perm_dev, int32_t* info_dev, void* stream) {
    try {
        NLF_REQUIRE(n > 0 && n <= 8192 && batch >= 1 && A_dev && lda >= n && strideA >= lda * n && ipiv_dev &&
                        info_dev && (dtype == NLF_C64 || dtype == NLF_C128),
                    NLF_ERR_ARG, "nlf_getrf_batched_noalloc: bad arguments");
        const int64_t need = nlf::getrf_scratch_ints(n, batch);
        NLF_REQUIRE(need <= NLF_NOALLOC_SCRATCH_INTS, NLF_ERR_ARG,
                    "nlf_getrf_batched_noalloc: 4 n batch = " + std::to_string(need) +
                        " exchange-list entries exceed the fixed scratch of " +
                        std::to_string((long long)NLF_NOALLOC_SCRATCH_INTS) + " (n * batch <= " +
                        std::to_string((long long)NLF_NOALLOC_SCRATCH_INTS / 4) + ")");
        int32_t* list = scratch_on_current_device();
        hipStream_t s = (hipStream_t)stream;
        struct NoProfiler {   // no timing events around these launches
            nlf::Profiler* saved = nlf::active_profiler();
            NoProfiler() { nlf::active_profiler() = nullptr; }
            ~NoProfiler() { nlf::active_profiler() = saved; }
        } off;
        if (dtype == NLF_C128)
            nlf::getrf<double>(s, n, batch, (nlf::z128*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list);
        else
            nlf::getrf<float>(s, n, batch, (nlf::z64*)A_dev, lda, strideA, ipiv_dev, perm_dev, info_dev, list);
        return NLF_OK;
    } catch (const nlf::Error& e) {
        nlf::record_error(e.msg);
        return (nlfeast_status)e.status;
    } catch (const std::exception& e) {
        nlf::record_error(e.what());
        return NLF_ERR_DEVICE;
    }
}
