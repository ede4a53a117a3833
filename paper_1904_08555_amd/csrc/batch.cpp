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
    int32_t *win_dev = nullptr;    // per window: first element (lo, hi), element count
    int32_t *witem_dev = nullptr;  // per window: first work item; one extra entry
    int32_t *item_dev = nullptr;   // per item: n, first loff index, count, 0
    int32_t *loff_dev = nullptr;   // per instance: element offset inside its window
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
    (void)hipFree(p->witem_dev);
    (void)hipFree(p->item_dev);
    (void)hipFree(p->loff_dev);
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
    const int32_t *win = p->win_dev, *witem = p->witem_dev, *item = p->item_dev, *loff = p->loff_dev;
    int nwin = p->nwin;
    void *args[] = {&win, &witem, &nwin, &item, &loff, &A, &B, &C};
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
    // into work items of up to `u` instances.  Windows stay in memory order, so
    // each array is read and written as one contiguous stream.
    const int64_t wmax = h->key.tile_n, u = h->key.unroll;
    std::vector<int32_t> win, witem, item, loff;
    loff.reserve((size_t)count);
    std::vector<int64_t> bucket[17];
    int64_t i0 = 0;
    while (i0 < count) {
        int64_t i1 = i0, len = 0;
        while (i1 < count && len + (int64_t)n_host[i1] * n_host[i1] <= wmax) len += (int64_t)n_host[i1] * n_host[i1], ++i1;
        const int64_t base = off[(size_t)i0];
        win.push_back((int32_t)(uint32_t)(base & 0xffffffffu));
        win.push_back((int32_t)(base >> 32));
        win.push_back((int32_t)len);
        witem.push_back((int32_t)(item.size() / 4));
        for (int n = 1; n <= 16; ++n) bucket[n].clear();
        for (int64_t i = i0; i < i1; ++i) bucket[n_host[i]].push_back(i);
        for (int n = 1; n <= 16; ++n)
            for (size_t s0 = 0; s0 < bucket[n].size(); s0 += (size_t)u) {
                const size_t s1 = std::min(bucket[n].size(), s0 + (size_t)u);
                item.push_back(n);
                item.push_back((int32_t)loff.size());
                item.push_back((int32_t)(s1 - s0));
                item.push_back(0);
                for (size_t t = s0; t < s1; ++t) loff.push_back((int32_t)(off[(size_t)bucket[n][t]] - base));
            }
        i0 = i1;
    }
    witem.push_back((int32_t)(item.size() / 4));
    auto p = new sj_plan_();
    p->h = h;
    p->count = count;
    p->total = total;
    p->nwin = (int)(win.size() / 3);
    if (hipGetDevice(&p->device) != hipSuccess) {
        free_plan(p);
        return fail(SJ_ERR_HIP, "hipGetDevice failed");
    }
    // Persistent grid: as many workgroups as the device holds at once (from the
    // compiler's occupancy and LDS figures), each walking windows grid-stride.
    int cus = 0;
    int64_t resident = 2048;
    const sj_kernel_info &ki = h->info;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0 &&
        ki.occupancy > 0) {
        const int64_t waves_per_wg = h->geom.block / 64;
        int64_t per_cu = std::max<int64_t>(1, (int64_t)ki.occupancy * 4 / waves_per_wg);
        if (ki.lds_bytes > 0) per_cu = std::min<int64_t>(per_cu, std::max(1, (160 * 1024) / ki.lds_bytes));
        resident = (int64_t)cus * std::min<int64_t>(per_cu, 16);
    }
    p->grid = (unsigned)std::min<int64_t>(p->nwin, resident);
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (!bytes) return true;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    std::vector<int32_t> n_copy(n_host, n_host + count);
    if (!up((void **)&p->n_dev, n_copy.data(), (size_t)count * 4) ||
        !up((void **)&p->off_dev, off.data(), (size_t)count * 8) ||
        !up((void **)&p->win_dev, win.data(), win.size() * 4) ||
        !up((void **)&p->witem_dev, witem.data(), witem.size() * 4) ||
        !up((void **)&p->item_dev, item.data(), item.size() * 4) ||
        !up((void **)&p->loff_dev, loff.data(), loff.size() * 4)) {
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
