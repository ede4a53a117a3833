// Internal declarations of the specialization library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sj.h"

struct sj_handle_;

namespace sj {

// Canonical, fully resolved specialization request.  Plain data; zero-filled
// before use so that hashing and comparison can work on the raw bytes.
struct SpecKey {
    int32_t kernel, dtype, layout, variant;
    int64_t Z, G, D, NM;
    int64_t B, I;            // contraction view: psi [B][D][I], phi [B][NM][I]
    int32_t tile_n, tile_k, unroll, block;
    int32_t index64, full_unroll;
    int32_t order, pad0;
    uint32_t class_mask;
    uint32_t flags;          // key-relevant flags only
    int64_t rows, inputs, width;
    int32_t device;          // -1 for compile-only keys
    int32_t lib_version;
    char arch[64];
    int32_t values, pad1;    // 1: the weights' values are constants of the specialization
    uint64_t vhash[2];       // two independent 64-bit hashes of those values (bit patterns)
};

bool key_equal(const SpecKey &a, const SpecKey &b);
uint64_t key_hash(const SpecKey &k);
uint64_t hash_words(const void *p, size_t bytes);   // bytes a multiple of 8

struct KeyHashF {
    size_t operator()(const SpecKey &k) const { return (size_t)key_hash(k); }
};
struct KeyEqF {
    bool operator()(const SpecKey &a, const SpecKey &b) const { return key_equal(a, b); }
};

// Thread-local error channel.
sj_status fail(sj_status s, const std::string &msg);
void clear_error();

// Validate `spec` for kernel `k` and fill the canonical key (defaults resolved).
// `device`/`arch` describe the target; device = -1 for compile-only requests.
sj_status make_key(sj_kernel k, const sj_spec *spec, int device, const char *arch, SpecKey *out);

// Source text (prologue + embedded template) and the kernel's symbol name.
sj_status emit_source(const SpecKey &key, std::string *src, std::string *kernel_name,
                      std::string *kernel_name2 = nullptr, const double *values = nullptr);

// Turn `key` (from make_key) into a value-specialized key for the `count`
// weights at `values` (host): checks, forced tiles, content hashes.
sj_status make_values_key(const double *values, size_t count, SpecKey *key);

// Number of parameters of the cost-model MLP with `inputs` features and width `width`.
inline int64_t mlp_nparams(int64_t inputs, int64_t width) { return width * inputs + width * width + 3 * width + 1; }

// Load and store forms of the streamed operands of a contraction key: 1 =
// nontemporal, 0 = ordinary; explicit SJ_FLAG_LOADS_* / SJ_FLAG_STORES_* flags,
// else the measured defaults.
void load_store_policy(const SpecKey &key, int *nt_load, int *nt_store);

// Whether a contraction key renumbers its workgroups so that each XCD takes a
// contiguous range (explicit SJ_FLAG_XCD_* flags, else the measured default).
bool xcd_contiguous(const SpecKey &key);

// Launch geometry of a resolved key.
struct Geometry {
    unsigned grid;
    unsigned block;
    int persistent;   // the kernel loops over its work: the grid is capped at load time to the resident workgroups
};
Geometry key_geometry(const SpecKey &key);

// hiprtc compile of `src` for `arch`; fills code and the compiler log.
sj_status rtc_compile(const std::string &src, const char *arch, const std::string &name,
                      std::vector<char> *code, std::string *log);

// Parse the resource-usage remarks of a compiler log into info.
void parse_resource_usage(const std::string &log, sj_kernel_info *info);

// Validate run pointers: non-null, 16-byte aligned, outputs (index >= first_out)
// overlapping no other buffer.
sj_status check_ptrs(void *const *ptrs, int nptrs, int expect, const size_t *bytes, int first_out);

// The two launches of the MLP backward pass of handle h (kernel SJ_MLP_BWD) with
// workspace ws of rows * (4 width + 2) floats; pointers already checked.
sj_status launch_mlp_bwd(const sj_handle_ *h, void *th, void *X, void *t, void *g, void *loss, void *ws,
                         hipStream_t st);

// Read `bytes` of `buf` on stream st (evicts L2 and the last-level cache with
// clean lines; used between timed launches).
hipError_t launch_flush_read(void *buf, size_t bytes, hipStream_t st);

// Resolve and keep the device address of `device`'s copy of the static MLP
// scratch array; `device` must be current.  Idempotent.
sj_status noalloc_setup(int device);

// Initialized device state.
sj_status ensure_device(int *device, const char **arch);

}  // namespace sj

struct sj_handle_ {
    sj::SpecKey key;
    uint64_t hash = 0;
    std::string kernel_name;
    std::vector<char> code;
    std::string kernel_name2;     // second kernel of the module (MLP backward), empty if none
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;
    hipFunction_t fn2 = nullptr;
    sj::Geometry geom{0, 0};
    sj_kernel_info info{};
    bool runnable = false;
};
