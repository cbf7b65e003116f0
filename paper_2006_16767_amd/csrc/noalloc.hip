// Column-major SpMSpV for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
// the same kernels as spmspv_csc, with the workspace taken from a
// file-scope device array instead of a caller argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

// 64 MiB per device, held by every GPU the library runs on until the
// process ends. Host code must never pass this name to a kernel or a copy:
// on the host it is a stand-in, not a device address. The device address
// comes from hipGetSymbolAddress, taken once per device below.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// The device address of `scratch` on device dev, looked up on the first call
// for that device with dev current (each GPU holds its own copy of the array
// at its own address). Restores the caller's current device.
static spx_status scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SPX_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        SPX_HIP(hipGetDevice(&cur));
        if (cur != dev) SPX_HIP(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) SPX_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(SPX_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPX_OK;
}

}  // namespace spx

using namespace spx;

extern "C" size_t spmspv_csc_noalloc_capacity(void) { return kScratchBytes; }

extern "C" spx_status spmspv_csc_noalloc(const spx_csc* A, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                                         void* y, const spx_plan* plan, void* stream) {
    SPX_TRY(check_csc(A));
    SPX_TRY(spx_check_plan(plan, A->dtype));
    if (plan->pattern != SPX_PAT_CSC_SPMSPV)
        return fail(SPX_ERR_ARG, "spmspv_csc_noalloc needs pattern SPX_PAT_CSC_SPMSPV");
    if (nnz_x < 0 || nnz_x > A->n) return fail(SPX_ERR_SHAPE, "nnz_x must be in [0, n]");
    if (nnz_x > 0 && (!x_idx || (A->dtype != SPX_BOOL && !x_val))) return fail(SPX_ERR_ARG, "x arrays are null");
    if (A->m > 0 && !y) return fail(SPX_ERR_ARG, "y is null");
    const size_t need = spmspv_csc_ws(A->m, A->n, A->nnz, nnz_x, A->dtype, plan);
    if (need > kScratchBytes)
        return fail(SPX_ERR_WORKSPACE, "spmspv_csc_noalloc: this plan needs " + std::to_string(need) +
                                           " bytes of scratch, more than the fixed " +
                                           std::to_string(kScratchBytes) + "; use spmspv_csc with a workspace");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (s) {
        SPX_HIP(hipStreamGetDevice(s, &dev));
    } else {
        SPX_HIP(hipGetDevice(&dev));
    }
    void* base = nullptr;
    SPX_TRY(scratch_on(dev, &base));
    // The kernels take no state from the workspace across calls (every
    // buffer in it is written before it is read within one call), so the
    // contents the last call left need no clearing. The scan counter of the
    // one-launch length scan lives in the handle, not here: with none, the
    // scan takes its two-launch form.
    CscArgs a{A->m, A->n, A->nnz, A->dtype, A->col_ptr, A->row_idx, A->vals, nullptr, nullptr, -1};
    Arena ws(base, kScratchBytes);
    return launch_spmspv_csc(a, nnz_x, x_idx, x_val, y, plan, ws, s);
}
