// MLP backward pass without any allocation or caller workspace
// (sj_run_mlp_bwd_noalloc).
//
// The backward pass of the cost model needs a workspace of rows * (4 width + 2)
// floats (per-row activations and deltas).  sj_run takes it from the caller;
// this entry point uses a static device array instead, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).  Each device
// the library runs on holds its own copy of the array, kScratchFloats floats
// (4 MiB), until the process ends.  In host code the array's name is only a
// host-side stand-in: its device address is resolved once per device with
// hipGetSymbolAddress (at sj_init, or at the first call on a device) and only
// that address is handed to kernels.  Every call on one device shares that
// device's array, so calls that overlap on one device (concurrent streams)
// race; every workspace value is written before it is read, so nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>

#include "sj_internal.h"

namespace {
constexpr size_t kScratchFloats = size_t(1) << 20;
}

static __device__ __align__(256) float scratch[kScratchFloats];

namespace {
struct DevScratch {
    std::atomic<int> state{0};   // 0 not resolved, 1 resolved, -1 lookup failed
    float *ptr = nullptr;        // device address of this device's copy
};
DevScratch g_scratch[64];
std::mutex g_scratch_mu;
}  // namespace

namespace sj {

sj_status noalloc_setup(int device)
{
    if (device < 0 || device >= 64) return fail(SJ_ERR_INVALID_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    DevScratch &d = g_scratch[device];
    if (d.state.load(std::memory_order_acquire) == 1) return SJ_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        d.state.store(-1, std::memory_order_release);
        return fail(SJ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    d.ptr = static_cast<float *>(p);
    d.state.store(1, std::memory_order_release);
    return SJ_OK;
}

}  // namespace sj

using namespace sj;

// Device address of `device`'s scratch copy, resolving it (with that device
// current) on first use.
static sj_status scratch_for(int device, float **out)
{
    if (device < 0 || device >= 64) return fail(SJ_ERR_INVALID_ARG, "handle has no device");
    DevScratch &d = g_scratch[device];
    if (d.state.load(std::memory_order_acquire) != 1) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return fail(SJ_ERR_HIP, "hipGetDevice failed");
        if (cur != device && hipSetDevice(device) != hipSuccess) return fail(SJ_ERR_HIP, "hipSetDevice failed");
        const sj_status s = noalloc_setup(device);
        if (cur != device) (void)hipSetDevice(cur);
        if (s != SJ_OK) return s;
    }
    *out = d.ptr;
    return SJ_OK;
}

extern "C" sj_status sj_run_mlp_bwd_noalloc(sj_handle h, void *const *ptrs, int nptrs, void *stream)
{
    clear_error();
    if (!h) return fail(SJ_ERR_INVALID_ARG, "null handle");
    if (!h->runnable) return fail(SJ_ERR_INVALID_ARG, "handle was compiled with SJ_FLAG_COMPILE_ONLY and cannot run");
    const SpecKey &k = h->key;
    if (k.kernel != SJ_MLP_BWD) return fail(SJ_ERR_INVALID_ARG, "sj_run_mlp_bwd_noalloc takes an SJ_MLP_BWD handle");
    const size_t R = (size_t)k.rows, F = (size_t)k.inputs, H = (size_t)k.width;
    const size_t need = R * (4 * H + 2);
    if (need > kScratchFloats)
        return fail(SJ_ERR_INVALID_ARG, "rows * (4 width + 2) = " + std::to_string(need) +
                                            " floats exceeds the static scratch of " +
                                            std::to_string(kScratchFloats) + " floats");
    const size_t P = (size_t)mlp_nparams(k.inputs, k.width);
    const size_t bytes[5] = {P * 4, R * F * 4, R * 4, P * 4, 4};
    sj_status s = check_ptrs(ptrs, nptrs, 5, bytes, 3);
    if (s != SJ_OK) return s;
    float *ws = nullptr;
    s = scratch_for(k.device, &ws);
    if (s != SJ_OK) return s;
    return launch_mlp_bwd(h, ptrs[0], ptrs[1], ptrs[2], ptrs[3], ptrs[4], ws, (hipStream_t)stream);
}
