// Batched small products: host plans, the persistent launch and HIP graph
// replay (ClangJIT section 5.1: the cost that matters for small products is
// looking the instantiation up and launching it per call; a plan resolves the
// specialization once, sorts the batch into size classes once, and a captured
// graph replays the single launch).
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "sj_internal.h"

using namespace sj;

struct sj_plan_ {
    sj_handle_ *h = nullptr;
    int device = -1;
    int64_t count = 0, total = 0;
    int nwork = 0;
    unsigned grid = 0;
    int32_t *n_dev = nullptr;
    int64_t *off_dev = nullptr;
    int32_t *order_dev = nullptr;
    int32_t *work_dev = nullptr;
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
    (void)hipFree(p->order_dev);
    (void)hipFree(p->work_dev);
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
    if (p->nwork == 0) return SJ_OK;
    const int32_t *work = p->work_dev;
    int nwork = p->nwork;
    const int32_t *order = p->order_dev;
    const int64_t *off = p->off_dev;
    void *args[] = {&work, &nwork, &order, &off, &A, &B, &C};
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
    const int R = h->key.unroll, block = h->key.block;
    // Counting sort by size class; offsets in the caller's order.
    std::vector<int64_t> off((size_t)count);
    std::vector<int64_t> per_class(17, 0);
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const int32_t n = n_host[i];
        if (n < 1 || n > 16) return fail(SJ_ERR_INVALID_ARG, "instance size out of [1, 16]");
        if (!(mask & (1u << n))) return fail(SJ_ERR_INVALID_ARG, "instance size " + std::to_string(n) + " not in the handle's class mask");
        off[(size_t)i] = total;
        total += (int64_t)n * n;
        per_class[n]++;
    }
    std::vector<int64_t> first(17, 0);
    for (int n = 2; n <= 16; ++n) first[n] = first[n - 1] + per_class[n - 1];
    std::vector<int32_t> order((size_t)count);
    {
        std::vector<int64_t> pos = first;
        for (int64_t i = 0; i < count; ++i) order[(size_t)pos[n_host[i]]++] = (int32_t)i;
    }
    std::vector<int32_t> work;
    for (int n = 1; n <= 16; ++n) {
        if (!per_class[n]) continue;
        const int64_t rn = R * n <= 16 ? R : std::max(1, 16 / n);   // rows per thread, as in the kernel
        const int64_t slots = block / ((n + rn - 1) / rn);
        for (int64_t s = 0; s < per_class[n]; s += slots) {
            work.push_back(n);
            work.push_back((int32_t)(first[n] + s));
            work.push_back((int32_t)std::min<int64_t>(slots, per_class[n] - s));
            work.push_back(0);
        }
    }
    auto p = new sj_plan_();
    p->h = h;
    p->count = count;
    p->total = total;
    p->nwork = (int)(work.size() / 4);
    p->grid = (unsigned)std::min<int64_t>(p->nwork, 2048);
    if (hipGetDevice(&p->device) != hipSuccess) {
        free_plan(p);
        return fail(SJ_ERR_HIP, "hipGetDevice failed");
    }
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (!bytes) return true;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    std::vector<int32_t> n_copy(n_host, n_host + count);
    if (!up((void **)&p->n_dev, n_copy.data(), (size_t)count * 4) ||
        !up((void **)&p->off_dev, off.data(), (size_t)count * 8) ||
        !up((void **)&p->order_dev, order.data(), (size_t)count * 4) ||
        !up((void **)&p->work_dev, work.data(), work.size() * 4)) {
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
