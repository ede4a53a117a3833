// Exported C ABI: device set-up, the program-global specialization cache and
// the launch path.
//
// Cache (ClangJIT section 4, Algorithm 1: look the instantiation up, build it
// on a miss, store it, return it): an unordered_map from the canonical key to
// an entry.  A hit takes only a shared (reader) lock on the map, so hits from
// many threads proceed together; a miss takes the build mutex, inserts a
// "building" entry and compiles outside every lock; concurrent requests for
// the same key wait for that entry instead of compiling again.  A failed
// build removes its entry, so a later request retries.  The paper reports that the lookup itself is what costs
// (section 5.1); here the lookup happens once, in sj_specialize, and sj_run
// launches from the handle without touching the cache.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "sj_internal.h"

namespace sj {

namespace {

enum EntryState { kBuilding = 0, kReady = 1, kFailed = 2 };

struct Entry {
    std::atomic<int> state{kBuilding};   // h is set before state becomes kReady (release)
    sj_handle_ *h = nullptr;
    sj_status err = SJ_OK;
    std::string msg;
};

// Lock order: g_mu, then g_rw.  Map insertions and removals hold both; hits
// hold g_rw shared only; the miss path reads the map under g_mu.
std::mutex g_mu;                 // builds, statistics, the in-flight condition
std::shared_mutex g_rw;          // the map's structure
std::condition_variable g_cv;
std::unordered_map<SpecKey, std::shared_ptr<Entry>, KeyHashF, KeyEqF> g_map;
sj_stats_t g_stats{};
std::atomic<uint64_t> g_lookups{0}, g_hits{0};

struct DeviceState {
    std::atomic<bool> ready{false};   // arch is written before ready (release)
    std::string arch;
};
std::mutex g_dev_mu;
DeviceState g_dev[64];

// Per-thread front cache: the caller's request as given (kernel, device and
// the spec's fields with padding zeroed) -> handle.  A hit costs one hash and
// one compare of 15 words, takes no lock and writes no shared cache line.
// make_key is a pure function of exactly these inputs, so a front hit returns
// the handle the canonical cache would.  sj_cache_clear bumps g_epoch, which
// empties every thread's front cache at its next lookup.
struct RawKey {
    int32_t kernel, device, dtype, layout, variant, pad0;
    int64_t Z, G, D, NM, count;
    uint32_t class_mask;
    int32_t tile_n, tile_k, unroll, block;
    uint32_t flags;
    int32_t order, pad1;
    int64_t rows, inputs, width;
};
static_assert(sizeof(RawKey) % 8 == 0, "raw key is hashed as 64-bit words");

RawKey raw_key(sj_kernel k, const sj_spec *s, int device)
{
    RawKey r;
    std::memset(&r, 0, sizeof r);
    r.kernel = k;
    r.device = device;
    r.dtype = s->dtype;
    r.layout = s->layout;
    r.variant = s->variant;
    r.Z = s->Z;
    r.G = s->G;
    r.D = s->D;
    r.NM = s->NM;
    r.count = s->count;
    r.class_mask = s->class_mask;
    r.tile_n = s->tile_n;
    r.tile_k = s->tile_k;
    r.unroll = s->unroll;
    r.block = s->block;
    r.flags = s->flags;
    r.order = s->order;
    r.rows = s->rows;
    r.inputs = s->inputs;
    r.width = s->width;
    return r;
}

struct RawHashF {
    size_t operator()(const RawKey &k) const { return (size_t)hash_words(&k, sizeof k); }
};
struct RawEqF {
    bool operator()(const RawKey &a, const RawKey &b) const { return std::memcmp(&a, &b, sizeof a) == 0; }
};

struct FrontCounter {
    std::atomic<uint64_t> hits{0};   // written by its thread only; summed by sj_stats
};
std::mutex g_front_mu;
std::vector<FrontCounter *> g_front;   // one per thread that looked anything up; never freed
std::atomic<uint64_t> g_epoch{0};

struct FrontCache {
    uint64_t epoch = ~0ull;
    FrontCounter *counter = nullptr;
    std::unordered_map<RawKey, sj_handle_ *, RawHashF, RawEqF> map;
};
thread_local FrontCache t_front;

FrontCache &front()
{
    FrontCache &f = t_front;
    if (!f.counter) {
        f.counter = new FrontCounter;
        std::lock_guard<std::mutex> lk(g_front_mu);
        g_front.push_back(f.counter);
    }
    const uint64_t ep = g_epoch.load(std::memory_order_acquire);
    if (f.epoch != ep) {
        f.map.clear();
        f.epoch = ep;
    }
    return f;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

sj_status ensure_device(int *device, const char **arch)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SJ_ERR_NOT_INITIALIZED, "no HIP device is available");
    }
    if (dev < 0 || dev >= 64) return fail(SJ_ERR_UNSUPPORTED, "device ordinal beyond 63");
    if (g_dev[dev].ready.load(std::memory_order_acquire)) {
        *device = dev;
        *arch = g_dev[dev].arch.c_str();
        return SJ_OK;
    }
    sj_status s = (sj_status)sj_init(dev);
    if (s != SJ_OK) return s;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    *device = dev;
    *arch = g_dev[dev].arch.c_str();
    return SJ_OK;
}

// SJ_LOG=1 in the environment: one line per specialization built (or failed) on stderr.
static bool log_enabled()
{
    static const bool on = [] {
        const char *v = std::getenv("SJ_LOG");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

static void log_build(const sj_handle_ &h, sj_status s, bool precompiled)
{
    if (!log_enabled()) return;
    std::fprintf(stderr,
                 "sj: %s %s key=%016llx device=%d emit=%.3f ms compile=%.3f ms load=%.3f ms vgprs=%d lds=%d "
                 "scratch=%d code=%llu B%s\n",
                 s == SJ_OK ? "built" : "FAILED", h.kernel_name.c_str(), (unsigned long long)h.hash, h.key.device,
                 h.info.emit_ms, h.info.compile_ms, h.info.load_ms, h.info.vgprs, h.info.lds_bytes,
                 h.info.scratch_bytes, (unsigned long long)h.code.size(), precompiled ? " (adopted code object)" : "");
}

static sj_status build_handle_impl(const SpecKey &key, const std::vector<char> *precompiled, const double *values,
                                   sj_handle_ *h);

static sj_status build_handle(const SpecKey &key, const std::vector<char> *precompiled, const double *values,
                              sj_handle_ **out)
{
    auto h = std::make_unique<sj_handle_>();
    const sj_status s = build_handle_impl(key, precompiled, values, h.get());
    log_build(*h, s, precompiled != nullptr);
    if (s != SJ_OK) return s;
    *out = h.release();
    return SJ_OK;
}

static sj_status build_handle_impl(const SpecKey &key, const std::vector<char> *precompiled, const double *values,
                                   sj_handle_ *h)
{
    h->key = key;
    h->hash = key_hash(key);
    std::memset(&h->info, 0, sizeof h->info);
    h->info.struct_size = sizeof(sj_kernel_info);
    auto t0 = std::chrono::steady_clock::now();
    std::string src;
    sj_status s = emit_source(key, &src, &h->kernel_name, &h->kernel_name2, values);
    if (s != SJ_OK) return s;
    h->info.emit_ms = ms_since(t0);

    std::string log;
    if (precompiled) {
        h->code = *precompiled;     // compiled by another process; resource usage unknown here
        h->info.vgprs = h->info.agprs = h->info.sgprs = -1;
        h->info.lds_bytes = h->info.scratch_bytes = h->info.occupancy = -1;
    } else {
        t0 = std::chrono::steady_clock::now();
        s = rtc_compile(src, key.arch, h->kernel_name, &h->code, &log);
        h->info.compile_ms = ms_since(t0);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_stats.compiles++;
            g_stats.compile_ms_total += h->info.compile_ms;
            g_stats.emit_ms_total += h->info.emit_ms;
            if (s != SJ_OK) g_stats.compile_failures++;
        }
        if (s != SJ_OK) return s;
        parse_resource_usage(log, &h->info);
    }
    h->geom = key_geometry(key);
    h->info.block = (int32_t)h->geom.block;
    h->info.grid = h->geom.grid;
    h->info.variant = key.variant;
    h->info.tile_n = key.tile_n;
    h->info.tile_k = key.tile_k;
    h->info.unroll = key.unroll;
    h->info.code_bytes = h->code.size();
    h->info.key_hash = h->hash;
    std::snprintf(h->info.kernel_name, sizeof h->info.kernel_name, "%s", h->kernel_name.c_str());

    if (!(key.flags & SJ_FLAG_COMPILE_ONLY)) {
        t0 = std::chrono::steady_clock::now();
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != key.device) {
            if (hipSetDevice(key.device) != hipSuccess) return fail(SJ_ERR_HIP, "hipSetDevice failed");
        }
        hipError_t e = hipModuleLoadData(&h->module, h->code.data());
        if (e != hipSuccess) return fail(SJ_ERR_LOAD, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
        e = hipModuleGetFunction(&h->fn, h->module, h->kernel_name.c_str());
        if (e == hipSuccess && !h->kernel_name2.empty())
            e = hipModuleGetFunction(&h->fn2, h->module, h->kernel_name2.c_str());
        if (e != hipSuccess) {
            (void)hipModuleUnload(h->module);
            return fail(SJ_ERR_LOAD, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
        }
        h->info.load_ms = ms_since(t0);
        h->runnable = true;
        if (h->geom.persistent) {
            // persistent grid: the workgroups resident at once on this device
            int blocks = 0, cus = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, h->fn, (int)h->geom.block, 0) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, key.device) == hipSuccess &&
                blocks > 0 && cus > 0)
                h->geom.grid = (unsigned)std::min<int64_t>(h->geom.grid, (int64_t)blocks * cus);
            h->info.grid = h->geom.grid;
        }
        if (precompiled) {
            // resource usage of a code object compiled elsewhere, from the loaded function
            int v = 0;
            if (hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_NUM_REGS, h->fn) == hipSuccess) h->info.vgprs = v;
            if (hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, h->fn) == hipSuccess) h->info.lds_bytes = v;
            if (hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, h->fn) == hipSuccess) h->info.scratch_bytes = v;
            int blocks = 0;
            if (h->geom.block && hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, h->fn, (int)h->geom.block, 0) == hipSuccess)
                h->info.occupancy = (int32_t)std::min<int64_t>(8, (int64_t)blocks * (h->geom.block / 64) / 4);
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_stats.loads++;
        g_stats.load_ms_total += h->info.load_ms;
    }
    return SJ_OK;
}

sj_status get_or_build(const SpecKey &key, sj_handle_ **out, const std::vector<char> *precompiled = nullptr,
                       const double *values = nullptr)
{
    g_lookups.fetch_add(1, std::memory_order_relaxed);
    {   // hit: shared lock only
        std::shared_lock<std::shared_mutex> rl(g_rw);
        auto it = g_map.find(key);
        if (it != g_map.end() && it->second->state.load(std::memory_order_acquire) == kReady) {
            g_hits.fetch_add(1, std::memory_order_relaxed);
            *out = it->second->h;
            return SJ_OK;
        }
    }
    std::unique_lock<std::mutex> lk(g_mu);
    auto it = g_map.find(key);
    if (it != g_map.end()) {
        std::shared_ptr<Entry> e = it->second;
        if (e->state.load(std::memory_order_acquire) == kReady) {
            g_hits.fetch_add(1, std::memory_order_relaxed);
            *out = e->h;
            return SJ_OK;
        }
        g_stats.inflight_waits++;
        g_cv.wait(lk, [&] { return e->state.load(std::memory_order_acquire) != kBuilding; });
        if (e->state.load(std::memory_order_acquire) == kReady) {
            g_hits.fetch_add(1, std::memory_order_relaxed);
            *out = e->h;
            return SJ_OK;
        }
        return fail(e->err, e->msg);
    }
    g_stats.misses++;
    auto e = std::make_shared<Entry>();
    {
        std::unique_lock<std::shared_mutex> wl(g_rw);
        g_map.emplace(key, e);
    }
    lk.unlock();

    sj_handle_ *h = nullptr;
    sj_status s = build_handle(key, precompiled, values, &h);
    std::string msg = (s == SJ_OK) ? std::string() : std::string(sj_last_error());

    lk.lock();
    if (s == SJ_OK) {
        e->h = h;
        e->state.store(kReady, std::memory_order_release);
        g_stats.entries++;
    } else {
        e->err = s;
        e->msg = msg;
        e->state.store(kFailed, std::memory_order_release);
        std::unique_lock<std::shared_mutex> wl(g_rw);
        g_map.erase(key);
    }
    lk.unlock();
    g_cv.notify_all();
    if (s != SJ_OK) return fail(s, msg);
    *out = h;
    return SJ_OK;
}

static bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return na && nb && x < y + nb && y < x + na;
}

// Byte sizes of the run pointers of a contraction handle; the last one is the output.
static void contraction_bytes(const SpecKey &k, size_t *bytes)
{
    const size_t esz = (k.dtype == SJ_F64) ? 8 : 4;
    const size_t cols = (size_t)k.G * (size_t)k.Z;
    bytes[0] = (size_t)k.NM * (size_t)k.D * 8;
    if (k.kernel == SJ_LTIMES) {
        bytes[1] = (size_t)k.D * cols * esz;
        bytes[2] = (size_t)k.NM * cols * esz;
    } else {
        bytes[1] = (size_t)k.NM * cols * esz;
        bytes[2] = (size_t)k.D * cols * esz;
    }
}

sj_status launch_mlp_bwd(const sj_handle_ *h, void *th, void *X, void *t, void *g, void *loss, void *ws,
                         hipStream_t st)
{
    // per-row activations and deltas into ws, then one thread per parameter (and one for the
    // loss) summing over the rows; every workspace value is written before it is read
    const size_t P = (size_t)mlp_nparams(h->key.inputs, h->key.width);
    void *args1[] = {&th, &X, &t, &ws};
    hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0, st, args1, nullptr);
    if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    void *args2[] = {&X, &ws, &g, &loss};
    const unsigned grid2 = (unsigned)((P + 1 + 255) / 256);
    e = hipModuleLaunchKernel(h->fn2, grid2, 1, 1, 256, 1, 1, 0, st, args2, nullptr);
    if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    return SJ_OK;
}

sj_status check_ptrs(void *const *ptrs, int nptrs, int expect, const size_t *bytes, int first_out)
{
    if (!ptrs) return fail(SJ_ERR_INVALID_ARG, "null pointer array");
    if (nptrs != expect) return fail(SJ_ERR_INVALID_ARG, "wrong number of pointers");
    for (int i = 0; i < nptrs; ++i) {
        if (!ptrs[i]) return fail(SJ_ERR_INVALID_ARG, "null buffer pointer");
        if (((uintptr_t)ptrs[i]) & 15u) return fail(SJ_ERR_ALIGN, "buffer pointer not 16-byte aligned");
    }
    for (int o = first_out; o < nptrs; ++o)
        for (int i = 0; i < nptrs; ++i)
            if (i != o && ranges_overlap(ptrs[i], bytes[i], ptrs[o], bytes[o]))
                return fail(SJ_ERR_ALIAS, "an output buffer overlaps another buffer");
    return SJ_OK;
}

}  // namespace sj

using namespace sj;

extern "C" {

sj_status sj_init(int hip_device)
{
    clear_error();
    if (hip_device < 0 || hip_device >= 64) return fail(SJ_ERR_INVALID_ARG, "device ordinal out of range");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= hip_device) {
        (void)hipGetLastError();
        return fail(SJ_ERR_NOT_INITIALIZED, "HIP device not present");
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev[hip_device].ready.load(std::memory_order_acquire)) return SJ_OK;
    if (hipSetDevice(hip_device) != hipSuccess) return fail(SJ_ERR_HIP, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return fail(SJ_ERR_HIP, "hipGetDeviceProperties failed");
    g_dev[hip_device].arch = prop.gcnArchName;
    // the device address of this device's copy of the static MLP scratch (a failure is
    // reported by the entry point that needs it, not here)
    (void)noalloc_setup(hip_device);
    clear_error();
    g_dev[hip_device].ready.store(true, std::memory_order_release);
    return SJ_OK;
}

sj_status sj_layout_from_string(const char *name, int32_t *out)
{
    clear_error();
    if (!name || !out) return fail(SJ_ERR_INVALID_ARG, "null argument");
    static const char *names[6] = {"DGZ", "DZG", "GDZ", "GZD", "ZDG", "ZGD"};
    char up[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
        char c = name[i];
        if (i == 3) {
            if (c != '\0') return fail(SJ_ERR_INVALID_ARG, "layout name must have three letters");
            break;
        }
        if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
        up[i] = c;
        if (c == '\0') return fail(SJ_ERR_INVALID_ARG, "layout name must have three letters");
    }
    for (int i = 0; i < 6; ++i)
        if (std::strcmp(up, names[i]) == 0) {
            *out = i;
            return SJ_OK;
        }
    return fail(SJ_ERR_INVALID_ARG, std::string("unknown layout '") + name + "'");
}

sj_status sj_specialize(sj_kernel k, const sj_spec *spec, sj_handle *out)
{
    clear_error();
    if (!spec || !out) return fail(SJ_ERR_INVALID_ARG, "null spec or output handle");
    int device = -1;
    const char *arch = "gfx950";
    if (spec->struct_size == sizeof(sj_spec) && !(spec->flags & SJ_FLAG_COMPILE_ONLY)) {
        sj_status s = ensure_device(&device, &arch);
        if (s != SJ_OK) return s;
    }
    if (spec->struct_size != sizeof(sj_spec)) return fail(SJ_ERR_INVALID_ARG, "sj_spec.struct_size mismatch");
    FrontCache &f = front();
    const RawKey rk = raw_key(k, spec, device);
    auto fit = f.map.find(rk);
    if (fit != f.map.end()) {
        f.counter->hits.fetch_add(1, std::memory_order_relaxed);
        *out = fit->second;
        return SJ_OK;
    }
    SpecKey key;
    sj_status s = make_key(k, spec, device, arch, &key);
    if (s != SJ_OK) return s;
    sj_handle_ *h = nullptr;
    s = get_or_build(key, &h);
    if (s != SJ_OK) return s;
    if (f.map.size() >= 4096) f.map.clear();   // bounded: a thread cycling through many keys
    f.map.emplace(rk, h);
    *out = h;
    return SJ_OK;
}

sj_status sj_specialize_values(sj_kernel k, const sj_spec *spec, const double *weights, size_t count, sj_handle *out)
{
    clear_error();
    if (!spec || !out) return fail(SJ_ERR_INVALID_ARG, "null spec or output handle");
    if (spec->struct_size != sizeof(sj_spec)) return fail(SJ_ERR_INVALID_ARG, "sj_spec.struct_size mismatch");
    if (spec->variant != SJ_VAR_AUTO && spec->variant != SJ_VAR_DIRECT)
        return fail(SJ_ERR_UNSUPPORTED, "value specialization has the DIRECT structure only");
    if (spec->order == 2) return fail(SJ_ERR_INVALID_ARG, "value specialization needs order 1 (no run-time row rotation)");
    int device = -1;
    const char *arch = "gfx950";
    if (!(spec->flags & SJ_FLAG_COMPILE_ONLY)) {
        sj_status s = ensure_device(&device, &arch);
        if (s != SJ_OK) return s;
    }
    sj_spec t = *spec;
    t.variant = SJ_VAR_DIRECT;
    t.order = 1;
    SpecKey key;
    sj_status s = make_key(k, &t, device, arch, &key);
    if (s != SJ_OK) return s;
    s = make_values_key(weights, count, &key);
    if (s != SJ_OK) return s;
    sj_handle_ *h = nullptr;
    s = get_or_build(key, &h, nullptr, weights);
    if (s != SJ_OK) return s;
    *out = h;
    return SJ_OK;
}

sj_status sj_specialize_with_code(sj_kernel k, const sj_spec *spec, const void *code, size_t size, sj_handle *out)
{
    clear_error();
    if (!spec || !out || !code || size < 4) return fail(SJ_ERR_INVALID_ARG, "null spec, code or output handle");
    if (std::memcmp(code, "\x7f" "ELF", 4) != 0) return fail(SJ_ERR_LOAD, "code is not an ELF code object");
    if (spec->flags & SJ_FLAG_COMPILE_ONLY) return fail(SJ_ERR_INVALID_ARG, "adopting code needs a runnable spec");
    int device = -1;
    const char *arch = "gfx950";
    sj_status s = ensure_device(&device, &arch);
    if (s != SJ_OK) return s;
    SpecKey key;
    s = make_key(k, spec, device, arch, &key);
    if (s != SJ_OK) return s;
    std::vector<char> bytes((const char *)code, (const char *)code + size);
    sj_handle_ *h = nullptr;
    s = get_or_build(key, &h, &bytes);
    if (s != SJ_OK) return s;
    *out = h;
    return SJ_OK;
}

sj_status sj_emit_source(sj_kernel k, const sj_spec *spec, char *buf, size_t len, size_t *needed)
{
    clear_error();
    SpecKey key;
    sj_status s = make_key(k, spec, -1, "gfx950", &key);
    if (s != SJ_OK) return s;
    std::string src, name;
    s = emit_source(key, &src, &name);
    if (s != SJ_OK) return s;
    if (needed) *needed = src.size() + 1;
    if (buf && len) {
        size_t n = std::min(len - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
    }
    return SJ_OK;
}

sj_status sj_resolve(sj_kernel k, const sj_spec *spec, sj_spec *out)
{
    clear_error();
    if (!out) return fail(SJ_ERR_INVALID_ARG, "null output");
    SpecKey key;
    sj_status s = make_key(k, spec, -1, "gfx950", &key);
    if (s != SJ_OK) return s;
    sj_spec r;
    std::memset(&r, 0, sizeof r);
    r.struct_size = sizeof(sj_spec);
    r.dtype = key.dtype;
    r.layout = key.layout;
    r.variant = key.variant;
    r.Z = key.Z; r.G = key.G; r.D = key.D; r.NM = key.NM;
    r.count = spec->count;
    r.class_mask = key.class_mask;
    r.tile_n = key.tile_n; r.tile_k = key.tile_k; r.unroll = key.unroll; r.block = key.block;
    r.flags = key.flags | (key.index64 ? SJ_FLAG_INDEX64 : 0u);
    r.order = key.order;
    r.rows = key.rows; r.inputs = key.inputs; r.width = key.width;
    *out = r;
    return SJ_OK;
}

sj_status sj_run(sj_handle h, void *const *ptrs, int nptrs, void *stream)
{
    if (!h) return fail(SJ_ERR_INVALID_ARG, "null handle");
    if (!h->runnable) return fail(SJ_ERR_INVALID_ARG, "handle was compiled with SJ_FLAG_COMPILE_ONLY and cannot run");
    const SpecKey &k = h->key;
    if (k.kernel == SJ_LTIMES || k.kernel == SJ_LPLUSTIMES) {
        size_t bytes[3];
        contraction_bytes(k, bytes);
        sj_status s = check_ptrs(ptrs, nptrs, 3, bytes, 2);
        if (s != SJ_OK) return s;
        void *a0 = ptrs[0], *a1 = ptrs[1], *a2 = ptrs[2];
        void *args[] = {&a0, &a1, &a2};
        hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0,
                                             (hipStream_t)stream, args, nullptr);
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    if (k.kernel == SJ_LTIMES_LPLUS) {
        // {L, L+, psi, psi_out} or {L, L+, psi, psi_out, phi_out}
        const size_t cols = (size_t)k.G * (size_t)k.Z;
        const size_t bytes[5] = {(size_t)k.NM * (size_t)k.D * 8, (size_t)k.NM * (size_t)k.D * 8,
                                 (size_t)k.D * cols * 8, (size_t)k.D * cols * 8, (size_t)k.NM * cols * 8};
        const int n = (nptrs == 4) ? 4 : 5;
        sj_status s = check_ptrs(ptrs, nptrs, n, bytes, 3);
        if (s != SJ_OK) return s;
        void *a0 = ptrs[0], *a1 = ptrs[1], *a2 = ptrs[2], *a3 = ptrs[3], *a4 = (n == 5) ? ptrs[4] : nullptr;
        void *args[] = {&a0, &a1, &a2, &a3, &a4};
        hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0,
                                             (hipStream_t)stream, args, nullptr);
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    if (k.kernel == SJ_MASS) {
        // {B1, D, X, Y}
        size_t nd = 1, nq = 1;
        for (int64_t i = 0; i < k.inputs; ++i) { nd *= (size_t)k.D; nq *= (size_t)k.NM; }
        const size_t ne = (size_t)k.rows;
        const size_t bytes[4] = {(size_t)k.D * (size_t)k.NM * 8, ne * nq * 8, ne * nd * 8, ne * nd * 8};
        sj_status s = check_ptrs(ptrs, nptrs, 4, bytes, 3);
        if (s != SJ_OK) return s;
        void *a0 = ptrs[0], *a1 = ptrs[1], *a2 = ptrs[2], *a3 = ptrs[3];
        void *args[] = {&a0, &a1, &a2, &a3};
        hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0,
                                             (hipStream_t)stream, args, nullptr);
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    if (k.kernel == SJ_SCATTERING) {
        // {S, mat, phi, phi_out}
        size_t nl = 0;
        while ((nl + 1) * (nl + 1) <= (size_t)k.NM - 1) ++nl;
        nl += 1;
        const size_t line = (size_t)k.NM * (size_t)k.G * (size_t)k.Z * 8;
        const size_t bytes[4] = {(size_t)k.rows * nl * (size_t)k.G * (size_t)k.G * 8, (size_t)k.Z * 4, line, line};
        sj_status s = check_ptrs(ptrs, nptrs, 4, bytes, 3);
        if (s != SJ_OK) return s;
        void *a0 = ptrs[0], *a1 = ptrs[1], *a2 = ptrs[2], *a3 = ptrs[3];
        void *args[] = {&a0, &a1, &a2, &a3};
        hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0,
                                             (hipStream_t)stream, args, nullptr);
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    if (k.kernel == SJ_MLP_FWD || k.kernel == SJ_MLP_BWD) {
        const size_t R = (size_t)k.rows, F = (size_t)k.inputs, H = (size_t)k.width;
        const size_t P = (size_t)mlp_nparams(k.inputs, k.width);
        hipStream_t st = (hipStream_t)stream;
        if (k.kernel == SJ_MLP_FWD) {
            const size_t bytes[3] = {P * 4, R * F * 4, R * 4};
            sj_status s = check_ptrs(ptrs, nptrs, 3, bytes, 2);
            if (s != SJ_OK) return s;
            void *a0 = ptrs[0], *a1 = ptrs[1], *a2 = ptrs[2];
            void *args[] = {&a0, &a1, &a2};
            hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0, st, args, nullptr);
            if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
            return SJ_OK;
        }
        const size_t bytes[6] = {P * 4, R * F * 4, R * 4, P * 4, 4, R * (4 * H + 2) * 4};
        sj_status s = check_ptrs(ptrs, nptrs, 6, bytes, 3);
        if (s != SJ_OK) return s;
        return launch_mlp_bwd(h, ptrs[0], ptrs[1], ptrs[2], ptrs[3], ptrs[4], ptrs[5], st);
    }
    if (k.kernel == SJ_ADAM) return fail(SJ_ERR_INVALID_ARG, "Adam handles run through sj_run_adam");
    if (k.kernel == SJ_BGEMM) return fail(SJ_ERR_INVALID_ARG, "BGEMM handles run through sj_batch_plan / sj_batch_run");
    return fail(SJ_ERR_INVALID_ARG, "this handle is not launched through sj_run");
}

sj_status sj_time_run(sj_handle h, void *const *ptrs, int nptrs, int warmup, int reps, void *flush,
                      size_t flush_bytes, void *stream, float *times_ms)
{
    clear_error();
    if (!h || !times_ms || reps < 1 || warmup < 0) return fail(SJ_ERR_INVALID_ARG, "bad timing arguments");
    if (flush_bytes && !flush) return fail(SJ_ERR_INVALID_ARG, "flush_bytes > 0 needs a flush buffer");
    if (flush_bytes && ((uintptr_t)flush & 15u)) return fail(SJ_ERR_ALIGN, "flush buffer not 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < warmup; ++i) {
        sj_status s = sj_run(h, ptrs, nptrs, stream);
        if (s != SJ_OK) return s;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(SJ_ERR_HIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SJ_ERR_HIP, "hipEventCreate failed");
    }
    sj_status out = SJ_OK;
    for (int i = 0; i < reps && out == SJ_OK; ++i) {
        if (flush_bytes && launch_flush_read(flush, flush_bytes, st) != hipSuccess) {
            out = fail(SJ_ERR_HIP, "flush read failed");
            break;
        }
        (void)hipEventRecord(e0, st);
        out = sj_run(h, ptrs, nptrs, stream);
        (void)hipEventRecord(e1, st);
        if (out != SJ_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            out = fail(SJ_ERR_HIP, "hipEventSynchronize failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        times_ms[i] = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return out;
}

sj_status sj_run_adam(sj_handle h, void *const *ptrs, int nptrs, int64_t step, double lr, double b1, double b2,
                      double eps, void *stream)
{
    clear_error();
    if (!h) return fail(SJ_ERR_INVALID_ARG, "null handle");
    if (!h->runnable) return fail(SJ_ERR_INVALID_ARG, "handle was compiled with SJ_FLAG_COMPILE_ONLY and cannot run");
    if (h->key.kernel != SJ_ADAM) return fail(SJ_ERR_INVALID_ARG, "handle is not an SJ_ADAM specialization");
    if (step < 1) return fail(SJ_ERR_INVALID_ARG, "step must be >= 1");
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(SJ_ERR_INVALID_ARG, "need lr > 0, 0 <= b1, b2 < 1, eps > 0");
    const size_t n = (size_t)h->key.rows;
    const size_t bytes[4] = {n * 4, n * 4, n * 4, n * 4};
    // p, m, v are updated in place: each is an output; g is the only pure input.
    if (!ptrs || nptrs != 4) return fail(SJ_ERR_INVALID_ARG, "Adam takes {p, g, m, v}");
    sj_status s = check_ptrs(ptrs, nptrs, 4, bytes, 0);
    if (s != SJ_OK) return s;
    float flr = (float)lr, fb1 = (float)b1, fb2 = (float)b2, feps = (float)eps;
    float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
    void *p = ptrs[0], *g = ptrs[1], *m = ptrs[2], *v = ptrs[3];
    void *args[] = {&p, &g, &m, &v, &flr, &fb1, &fb2, &feps, &c1, &c2};
    hipError_t e = hipModuleLaunchKernel(h->fn, h->geom.grid, 1, 1, h->geom.block, 1, 1, 0, (hipStream_t)stream, args,
                                         nullptr);
    if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    return SJ_OK;
}

sj_status sj_handle_info(sj_handle h, sj_kernel_info *out)
{
    if (!h || !out) return fail(SJ_ERR_INVALID_ARG, "null argument");
    if (out->struct_size != sizeof(sj_kernel_info)) return fail(SJ_ERR_INVALID_ARG, "sj_kernel_info.struct_size mismatch");
    *out = h->info;
    return SJ_OK;
}

sj_status sj_handle_code(sj_handle h, const void **code, size_t *size)
{
    if (!h || !code || !size) return fail(SJ_ERR_INVALID_ARG, "null argument");
    *code = h->code.data();
    *size = h->code.size();
    return SJ_OK;
}

sj_status sj_stats(sj_stats_t *out)
{
    if (!out) return fail(SJ_ERR_INVALID_ARG, "null argument");
    if (out->struct_size != sizeof(sj_stats_t)) return fail(SJ_ERR_INVALID_ARG, "sj_stats_t.struct_size mismatch");
    std::lock_guard<std::mutex> lk(g_mu);
    *out = g_stats;
    uint64_t front_hits = 0;
    {
        std::lock_guard<std::mutex> fl(g_front_mu);
        for (FrontCounter *c : g_front) front_hits += c->hits.load(std::memory_order_relaxed);
    }
    out->lookups = g_lookups.load(std::memory_order_relaxed) + front_hits;
    out->hits = g_hits.load(std::memory_order_relaxed) + front_hits;
    out->struct_size = sizeof(sj_stats_t);
    return SJ_OK;
}

sj_status sj_cache_clear(void)
{
    std::unique_lock<std::mutex> lk(g_mu);
    std::unique_lock<std::shared_mutex> wl(g_rw);
    for (auto &kv : g_map)
        if (kv.second->state.load(std::memory_order_acquire) == kBuilding)
            return fail(SJ_ERR_INVALID_ARG, "a specialization is being compiled");
    for (auto &kv : g_map) {
        sj_handle_ *h = kv.second->h;
        if (h) {
            if (h->module) (void)hipModuleUnload(h->module);
            delete h;
        }
    }
    g_map.clear();
    g_stats.entries = 0;
    g_epoch.fetch_add(1, std::memory_order_acq_rel);   // every thread's front cache empties at its next lookup
    return SJ_OK;
}

const char *sj_status_string(sj_status s)
{
    switch (s) {
    case SJ_OK: return "SJ_OK";
    case SJ_ERR_INVALID_ARG: return "SJ_ERR_INVALID_ARG";
    case SJ_ERR_UNSUPPORTED: return "SJ_ERR_UNSUPPORTED";
    case SJ_ERR_COMPILE: return "SJ_ERR_COMPILE";
    case SJ_ERR_LOAD: return "SJ_ERR_LOAD";
    case SJ_ERR_LAUNCH: return "SJ_ERR_LAUNCH";
    case SJ_ERR_ALIGN: return "SJ_ERR_ALIGN";
    case SJ_ERR_ALIAS: return "SJ_ERR_ALIAS";
    case SJ_ERR_OOM: return "SJ_ERR_OOM";
    case SJ_ERR_HIP: return "SJ_ERR_HIP";
    case SJ_ERR_NOT_INITIALIZED: return "SJ_ERR_NOT_INITIALIZED";
    }
    return "unknown status";
}

}  // extern "C"
