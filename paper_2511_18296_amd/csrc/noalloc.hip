// noalloc.hip -- the top-k selection with a library-owned workspace, for
// callers that cannot allocate device memory.  The workspace is a device
// array of this translation unit (its own code object, so that the launches
// of the selection kernels are not those of a module with a large global);
// each device holds its own copy for the life of the process.  The part of
// the workspace that must be zero when a selection starts (its level-0
// histogram and counters) is zero when the code object is loaded (the array
// has no initializer) and each selection leaves it zero again; the rest is
// written before it is read in every call.
#include <stdio.h>

#include <mutex>

#include "internal.h"

namespace mps {

constexpr int64_t kNoAllocMaxN = (int64_t)1 << 21;
// holds the selection's workspace for kNoAllocMaxN items and k = MPS_MAX_TOPK
// (checked against topk_ws_bytes on every call)
constexpr size_t kScratchBytes = (size_t)33 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this device's copy of `scratch` (the host-side name is
// only a stand-in and must never reach a kernel).  Looked up once per device.
static hipError_t scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace mps

extern "C" mps_status mps_topk_noalloc(const float *score, const uint8_t *flags, int64_t n,
                                       int32_t k, uint8_t require, uint8_t forbid,
                                       int64_t *idx, float *top_score, int32_t *count,
                                       void *stream) {
    using namespace mps;
    char msg[160];
    if (k < 1 || k > MPS_MAX_TOPK) {
        snprintf(msg, sizeof(msg), "k must be in 1..%d (got %d)", MPS_MAX_TOPK, k);
        return report_error(MPS_E_INVALID_ARG, msg);
    }
    if (n < 0 || n > kNoAllocMaxN || topk_ws_bytes(n, k) > kScratchBytes) {
        snprintf(msg, sizeof(msg),
                 "n = %lld exceeds the %lld items the library-owned top-k workspace holds",
                 (long long)n, (long long)kNoAllocMaxN);
        return report_error(MPS_E_INVALID_ARG, msg);
    }
    if ((n > 0 && (!score || !flags)) || !idx || !count)
        return report_error(MPS_E_INVALID_ARG, "score, flags, idx and count are required");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        snprintf(msg, sizeof(msg), "no usable current device (%s)", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    void *ws = nullptr;
    e = scratch_address(dev, &ws);
    if (e != hipSuccess) {
        snprintf(msg, sizeof(msg), "address of the top-k scratch: %s", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    e = launch_topk(score, flags, n, k, require, forbid, idx, top_score, count, ws,
                    (hipStream_t)stream);
    if (e != hipSuccess) {
        snprintf(msg, sizeof(msg), "topk: %s", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    return MPS_OK;
}
