// Batched small products: host plans, the persistent launch and HIP graph
// replay (ClangJIT section 5.1: the cost that matters for small products is
// looking the instantiation up and launching it per call; a plan resolves the
// specialization once, sorts the batch into size classes once, and a captured
// graph replays the single launch).
#include <algorithm>
#include <array>
#include <cstring>
#include <string>
#include <vector>

#include "sj_internal.h"

using namespace sj;

struct sj_plan_ {
    sj_handle_ *h = nullptr;
    int device = -1;
    int64_t count = 0, total = 0;
    int nwin = 0;
    unsigned grid = 0;
    int32_t *n_dev = nullptr;      // caller's order (generic kernel)
    int64_t *off_dev = nullptr;    // caller's order (generic kernel)
    int32_t *win_dev = nullptr;    // 8 ints per window (see the kernel template)
    int32_t *meta_dev = nullptr;   // per window: packed work items, then 16-bit instance offsets
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(sj_plan_ *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->n_dev);
    (void)hipFree(p->off_dev);
    (void)hipFree(p->win_dev);
    (void)hipFree(p->meta_dev);
    delete p;
}

sj_status check_abc(const sj_plan_ *p, const double *A, const double *B, const double *C)
{
    if (!A || !B || !C) return fail(SJ_ERR_INVALID_ARG, "null A, B or C");
    if ((((uintptr_t)A) | ((uintptr_t)B) | ((uintptr_t)C)) & 7u) return fail(SJ_ERR_ALIGN, "A, B, C must be 8-byte aligned");
    const size_t bytes = (size_t)p->total * 8;
    auto overlap = [&](const void *x, const void *y) {
        const char *a = (const char *)x, *b = (const char *)y;
        return bytes && a < b + bytes && b < a + bytes;
    };
    if (overlap(A, C) || overlap(B, C)) return fail(SJ_ERR_ALIAS, "C overlaps A or B");
    return SJ_OK;
}

sj_status launch(sj_plan_ *p, const double *A, const double *B, double *C, hipStream_t st)
{
    if (p->nwin == 0) return SJ_OK;
    const int32_t *win = p->win_dev, *meta = p->meta_dev;
    int nwin = p->nwin;
    void *args[] = {&win, &nwin, &meta, &A, &B, &C};
    hipError_t e = hipModuleLaunchKernel(p->h->fn, p->grid, 1, 1, p->h->geom.block, 1, 1, 0, st, args, nullptr);
    if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    return SJ_OK;
}

}  // namespace

extern "C" {

sj_status sj_batch_plan(sj_handle h, const int32_t *n_host, int64_t count, sj_plan *out)
{
    clear_error();
    if (!h || !out || (count > 0 && !n_host)) return fail(SJ_ERR_INVALID_ARG, "null argument");
    if (h->key.kernel != SJ_BGEMM) return fail(SJ_ERR_INVALID_ARG, "handle is not a BGEMM specialization");
    if (!h->runnable) return fail(SJ_ERR_INVALID_ARG, "handle was compiled with SJ_FLAG_COMPILE_ONLY");
    if (count < 0 || count > 2147483647LL) return fail(SJ_ERR_INVALID_ARG, "count must be in [0, 2^31-1]");
    const uint32_t mask = h->key.class_mask;
    // Offsets in the caller's order.
    std::vector<int64_t> off((size_t)count);
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const int32_t n = n_host[i];
        if (n < 1 || n > 16) return fail(SJ_ERR_INVALID_ARG, "instance size out of [1, 16]");
        if (!(mask & (1u << n))) return fail(SJ_ERR_INVALID_ARG, "instance size " + std::to_string(n) + " not in the handle's class mask");
        off[(size_t)i] = total;
        total += (int64_t)n * n;
    }
    // Windows: runs of consecutive whole instances with at most `wmax` elements
    // per array.  Inside a window, instances are grouped by size class (stable)
    // into work items of up to floor(16/n) * u instances.  Windows stay in memory order, so
    // each array is read and written as one contiguous stream.  Per window:
    //   win[8w .. 8w+7] = {first element lo, hi, element count, first meta word,
    //                      item count, meta word count, 0, 0}
    //   meta words      = items (n | (count-1) << 5 | first offset index << 12),
    //                     then the instances' element offsets inside the window
    //                     as 16-bit values, two per word (first in the low half).
    const int64_t wmax = h->key.tile_n, u = h->key.unroll;
    std::vector<int32_t> win, meta;
    std::vector<int64_t> bucket[17];
    std::vector<int32_t> items;
    std::vector<uint16_t> lo;
    int64_t i0 = 0;
    while (i0 < count) {
        int64_t i1 = i0, len = 0;
        while (i1 < count && len + (int64_t)n_host[i1] * n_host[i1] <= wmax) len += (int64_t)n_host[i1] * n_host[i1], ++i1;
        const int64_t base = off[(size_t)i0];
        for (int n = 1; n <= 16; ++n) bucket[n].clear();
        for (int64_t i = i0; i < i1; ++i) bucket[n_host[i]].push_back(i);
        items.clear();
        lo.clear();
        for (int n = 1; n <= 16; ++n) {
            // floor(16/n) instances share one 16x16 MFMA tile; an item holds u such groups
            const size_t chunk = (size_t)(16 / n) * (size_t)u;
            for (size_t s0 = 0; s0 < bucket[n].size(); s0 += chunk) {
                const size_t s1 = std::min(bucket[n].size(), s0 + chunk);
                items.push_back(n | (int32_t)((s1 - s0 - 1) << 5) | (int32_t)(lo.size() << 12));
                for (size_t t = s0; t < s1; ++t) lo.push_back((uint16_t)(off[(size_t)bucket[n][t]] - base));
            }
        }
        const int64_t m0 = (int64_t)meta.size();
        meta.insert(meta.end(), items.begin(), items.end());
        for (size_t t = 0; t < lo.size(); t += 2)
            meta.push_back((int32_t)((uint32_t)lo[t] | ((uint32_t)(t + 1 < lo.size() ? lo[t + 1] : 0) << 16)));
        const int64_t mlen = (int64_t)meta.size() - m0;
        if (m0 > INT32_MAX - mlen) return fail(SJ_ERR_UNSUPPORTED, "batch plan metadata exceeds 2^31 words");
        win.push_back((int32_t)(uint32_t)(base & 0xffffffffu));
        win.push_back((int32_t)(base >> 32));
        win.push_back((int32_t)len);
        win.push_back((int32_t)m0);
        win.push_back((int32_t)items.size());
        win.push_back((int32_t)mlen);
        win.push_back(0);
        win.push_back(0);
        i0 = i1;
    }
    auto p = new sj_plan_();
    p->h = h;
    p->count = count;
    p->total = total;
    p->nwin = (int)(win.size() / 8);
    if (hipGetDevice(&p->device) != hipSuccess) {
        free_plan(p);
        return fail(SJ_ERR_HIP, "hipGetDevice failed");
    }
    // Wave form: one wave per window.  Workgroup form: a persistent grid of as
    // many workgroups as the device holds at once (from the compiler's
    // occupancy and LDS figures), each walking windows grid-stride.
    const int64_t waves_per_wg = h->geom.block / 64;
    int cus = 0;
    int64_t resident = 2048;
    const sj_kernel_info &ki = h->info;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0 &&
        ki.occupancy > 0) {
        int64_t per_cu = std::max<int64_t>(1, (int64_t)ki.occupancy * 4 / waves_per_wg);
        if (ki.lds_bytes > 0) per_cu = std::min<int64_t>(per_cu, std::max(1, (160 * 1024) / ki.lds_bytes));
        resident = (int64_t)cus * std::min<int64_t>(per_cu, 16);
    }
    p->grid = (h->key.variant == SJ_VAR_DIRECT) ? (unsigned)((p->nwin + waves_per_wg - 1) / waves_per_wg)
                                                : (unsigned)std::min<int64_t>(p->nwin, resident);
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (!bytes) return true;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    std::vector<int32_t> n_copy(n_host, n_host + count);
    if (!up((void **)&p->n_dev, n_copy.data(), (size_t)count * 4) ||
        !up((void **)&p->off_dev, off.data(), (size_t)count * 8) ||
        !up((void **)&p->win_dev, win.data(), win.size() * 4) ||
        !up((void **)&p->meta_dev, meta.data(), meta.size() * 4)) {
        free_plan(p);
        return fail(SJ_ERR_OOM, "device allocation or upload of the plan failed");
    }
    *out = p;
    return SJ_OK;
}

sj_status sj_batch_run(sj_plan p, const double *A, const double *B, double *C, void *stream)
{
    clear_error();
    if (!p) return fail(SJ_ERR_INVALID_ARG, "null plan");
    sj_status s = check_abc(p, A, B, C);
    if (s != SJ_OK) return s;
    return launch(p, A, B, C, (hipStream_t)stream);
}

sj_status sj_batch_graph_capture(sj_plan p, const double *A, const double *B, double *C, void *stream)
{
    clear_error();
    (void)stream;
    if (!p) return fail(SJ_ERR_INVALID_ARG, "null plan");
    sj_status s = check_abc(p, A, B, C);
    if (s != SJ_OK) return s;
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
        return fail(SJ_ERR_HIP, "hipStreamCreate failed");
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(SJ_ERR_HIP, "hipStreamBeginCapture failed");
    s = launch(p, A, B, C, p->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (s != SJ_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(SJ_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(SJ_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return SJ_OK;
}

sj_status sj_batch_graph_launch(sj_plan p, void *stream)
{
    clear_error();
    if (!p) return fail(SJ_ERR_INVALID_ARG, "null plan");
    if (!p->exec) return fail(SJ_ERR_INVALID_ARG, "no graph captured for this plan");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return SJ_OK;
}

sj_status sj_batch_plan_arrays(sj_plan p, const int32_t **n_dev, const int64_t **off_dev, int64_t *total_elems)
{
    if (!p || !n_dev || !off_dev || !total_elems) return fail(SJ_ERR_INVALID_ARG, "null argument");
    *n_dev = p->n_dev;
    *off_dev = p->off_dev;
    *total_elems = p->total;
    return SJ_OK;
}

sj_status sj_plan_destroy(sj_plan p)
{
    if (!p) return fail(SJ_ERR_INVALID_ARG, "null plan");
    free_plan(p);
    return SJ_OK;
}

}  // extern "C"
