/*
 * sj.h -- runtime specialization of data-parallel kernels for AMD Instinct MI355X
 * (gfx950).  C ABI: plain host/device pointers, sizes and status codes.
 *
 * The problem statement follows ClangJIT (Finkel, Poliakoff & Richards, 2019):
 * a kernel whose sizes and data layout are known only at run time is
 * instantiated with those values on first request, compiled in-process, kept
 * in a program-global cache of instantiations and returned as a callable
 * handle (section 4, Algorithm 1: cache lookup, compile, store, return), with
 * no file-system access during the compile (section 1 and section 4: only data
 * from the running binary is used).  Explicitly specialized code stays ahead
 * of time (section 2); here that role is taken by the generic runtime-parameter
 * kernels behind sj_generic_run, which are also the fallback that the
 * paper's attribute-based design lacks (section 6, last list).
 *
 * Kernels:
 *  - SJ_LTIMES / SJ_LPLUSTIMES: the discrete-ordinates moment operators of the
 *    Kripke proxy application (section 5.2; the paper names the operators but
 *    does not write them down):
 *        phi[nm,g,z]  = sum_d  L[nm,d]  * psi[d,g,z]          (LTimes)
 *        psi'[d,g,z]  = sum_nm L+[d,nm] * phi[nm,g,z]         (LPlusTimes)
 *    over the six nestings of section 5.2's layout-dispatch listing, chosen at
 *    run time (by enum, or by name string as in section 5.2's JIT launcher).
 *  - SJ_BGEMM: batches of small square products C_i = A_i * B_i (section 5.1,
 *    RAJA small matrix multiply), one persistent launch per batch plan.
 *  - SJ_MLP_FWD / SJ_MLP_BWD / SJ_ADAM: the cost model that picks which
 *    specialization to compile, an instance of the profile-guided adaptive
 *    specialization and autotuning of section 6.
 *
 * Conventions (all entry points):
 *  - Every entry point returns sj_status.  On failure, sj_last_error() returns
 *    a thread-local message (for SJ_ERR_COMPILE it includes the compiler log).
 *  - Device buffers belong to the caller; the library never frees them.
 *  - Handles belong to the process-global cache; the same key always yields
 *    the same handle; a handle stays valid until sj_cache_clear() or exit.
 *    Each thread also keeps a private front cache of the requests it made, so
 *    a repeated sj_specialize takes no lock (measured on MI355X's host: about
 *    50 ns per hit from one thread and from each of eight).
 *    A handle is bound to the device that was current when it was created.
 *  - Plans belong to the caller (sj_plan_destroy).
 *  - Launches are asynchronous on `stream` (a hipStream_t; NULL is the null
 *    stream) and report launch-time errors only; faults surface at the
 *    caller's synchronization.
 *  - Outputs are overwritten (beta = 0).
 *  - Thread safety: sj_specialize compiles each key once even under concurrent
 *    calls; sj_run and the batch calls are reentrant.
 *  - Logging: with SJ_LOG=1 in the environment, every specialization the
 *    library builds (or fails to build) writes one line to stderr: kernel
 *    name, key hash, device, emit / compile / load milliseconds, VGPRs, LDS,
 *    scratch and code size.  Cache hits write nothing.
 */
#ifndef SJ_H
#define SJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SJ_VERSION 1

typedef enum sj_status {
    SJ_OK = 0,
    SJ_ERR_INVALID_ARG = 1,    /* bad size, enum, null pointer, struct_size */
    SJ_ERR_UNSUPPORTED = 2,    /* valid request this library does not implement */
    SJ_ERR_COMPILE = 3,        /* hiprtc rejected the emitted source; log in sj_last_error */
    SJ_ERR_LOAD = 4,           /* the code object did not load on the device */
    SJ_ERR_LAUNCH = 5,         /* kernel launch failed */
    SJ_ERR_ALIGN = 6,          /* a pointer is not 16-byte aligned */
    SJ_ERR_ALIAS = 7,          /* an input byte range overlaps an output byte range */
    SJ_ERR_OOM = 8,            /* host or device allocation failed */
    SJ_ERR_HIP = 9,            /* other HIP runtime error */
    SJ_ERR_NOT_INITIALIZED = 10 /* no GPU device could be initialized */
} sj_status;

typedef enum sj_kernel {
    SJ_LTIMES = 1,
    SJ_LPLUSTIMES = 2,
    SJ_BGEMM = 3,
    SJ_MLP_FWD = 4,
    SJ_MLP_BWD = 5,
    SJ_ADAM = 6,
    SJ_LTIMES_LPLUS = 7,   /* LTimes then LPlusTimes on the same columns in one pass (phi stays on chip) */
    SJ_SCATTERING = 8,     /* scattering source phi_out[nm,g,z] = sum_g' S[mat(z)][n(nm)][g][g'] phi[nm,g',z] */
    SJ_MASS = 9            /* tensor-product mass operator per element, y_e = B^T diag(D_e) B x_e (partial assembly) */
} sj_kernel;

/* Storage order of a psi-like array's three axes, rightmost fastest.  phi uses
 * the same order with D replaced by NM.  L is row-major [NM][D], L+ row-major
 * [D][NM], in every layout. */
typedef enum sj_layout {
    SJ_DGZ = 0, SJ_DZG = 1, SJ_GDZ = 2, SJ_GZD = 3, SJ_ZDG = 4, SJ_ZGD = 5
} sj_layout;

typedef enum sj_dtype {
    SJ_F64 = 0,     /* FP64 in, FP64 out, FP64 arithmetic */
    SJ_BF16 = 1,    /* LTimes: psi FP32 in, phi FP32 out; one BF16 product per term, FP32 accumulate (MFMA) */
    SJ_BF16X3 = 2,  /* as SJ_BF16 with split compensation: hi*hi + hi*lo + lo*hi per term */
    SJ_F32 = 3      /* MLP kernels */
} sj_dtype;

/* Kernel structure for LTimes / LPlusTimes.  AUTO picks DIRECT when the
 * innermost storage axis is a column axis (DGZ, DZG, GDZ, ZDG) and the FP64
 * matrix-core row kernel (MFMA) when it is D (GZD, ZGD); BF16 dtypes always
 * use MFMA.  FP64 MFMA with a column axis innermost is the matrix-core column
 * kernel (chosen explicitly, or by a tuner).  The fused SJ_LTIMES_LPLUS has
 * DIRECT and, for D innermost, the MFMA row structure (AUTO's choice there).
 * When AUTO's first choice declines a shape (register or LDS limits), the
 * next structure that accepts it is taken. */
typedef enum sj_variant {
    SJ_VAR_AUTO = 0,
    SJ_VAR_DIRECT = 1,   /* lanes along the contiguous column axis, direct HBM<->VGPR */
    SJ_VAR_STAGED = 2,   /* rows of contiguous D (or NM) values staged through LDS */
    SJ_VAR_MFMA = 3      /* matrix cores: BF16 dtypes; FP64 row kernel (D innermost) or column kernel;
                            SJ_SCATTERING: FP64 tiles of one moment and 16 zones (the default where
                            g or z is innermost; with nm innermost, 16-zone blocks staged in LDS) */
} sj_variant;

/* Flags. */
#define SJ_FLAG_COMPILE_ONLY      0x1u  /* compile to a code object, do not load: no GPU needed; the handle cannot run */
#define SJ_FLAG_INDEX64           0x2u  /* force 64-bit indexing (chosen automatically when an array has >= 2^31 elements) */
#define SJ_FLAG_LOADS_CACHED      0x4u  /* LTimes / LPlusTimes: ordinary loads of the streamed input */
#define SJ_FLAG_LOADS_NONTEMPORAL 0x8u  /* LTimes / LPlusTimes: nontemporal loads of the streamed input */
#define SJ_FLAG_STORES_CACHED     0x10u /* LTimes / LPlusTimes: ordinary stores of the output */
#define SJ_FLAG_STORES_NONTEMPORAL 0x20u /* LTimes / LPlusTimes: nontemporal stores of the output */
#define SJ_FLAG_ACCUMULATE        0x40u /* LTimes / LPlusTimes: add the result to the output's current values
                                           (phi += L psi, psi' += L+ phi: several direction sets summed into one
                                           output) instead of overwriting; the output is then also read */
/* Without a loads flag (stores flag) the default measured on MI355X applies:
 * nontemporal stores for every streamed output; nontemporal loads for LTimes'
 * column kernels, ordinary loads for LPlusTimes and for the FP64 MFMA row
 * kernel.  The two flags of a pair exclude each other; every policy flag is
 * part of the specialization key. */
#define SJ_FLAG_GENERIC_PER_LAYOUT 0x80u /* sj_generic_run, LTimes / LPlusTimes: the kernel compiled ahead of time
                                           for the spec's nesting (sizes still run-time arguments), Kripke's
                                           multiversioning; without it one kernel serves every nesting */
#define SJ_FLAG_DEBUG_FAIL_COMPILE 0x100u /* test hook: the emitted source contains a failing static_assert */
#define SJ_FLAG_XCD_CONTIGUOUS    0x200u /* LTimes / LPlusTimes / fused: workgroups are dispatched round-robin
                                           over the device's 8 XCDs (each with its own L2); the kernel renumbers
                                           them so that each XCD works through one contiguous range of the
                                           columns (or of each sweep of a persistent grid) */
#define SJ_FLAG_XCD_INTERLEAVED   0x400u /* LTimes / LPlusTimes / fused: workgroup b takes work item b (the
                                           hardware's round-robin order) */
/* Without an XCD flag the default measured on MI355X applies: contiguous for
 * the kernels whose column axis is innermost (DIRECT, FP64 MFMA columns,
 * BF16), interleaved for the row kernels (D innermost).  The two flags
 * exclude each other and are part of the specialization key. */

typedef struct sj_spec {
    uint32_t struct_size;   /* must be sizeof(sj_spec) */
    int32_t  dtype;         /* sj_dtype */
    int32_t  layout;        /* sj_layout (LTimes / LPlusTimes) */
    int32_t  variant;       /* sj_variant */
    int64_t  Z, G, D, NM;   /* LTimes / LPlusTimes: zones, groups, directions, moments; each in [1, 2^31-1] */
    int64_t  count;         /* BGEMM generic path: number of instances; SJ_SCATTERING: number of materials */
    uint32_t class_mask;    /* BGEMM: bit n set when size class n (1 <= n <= 16) occurs; 0 = all of 1..16 */
    int32_t  tile_n;        /* DIRECT: columns per thread (1, 2, 4); STAGED: rows per workgroup;
                               FP64 MFMA rows: 16-row tiles per wave (1..8); FP64 MFMA columns and
                               BF16: columns per lane (1, 2, 4 / 1, 4); BGEMM: window size, elements
                               per array staged in LDS (256..7168); SJ_SCATTERING, FP64 MFMA with g or
                               z innermost: tiles (one moment, 16 zones) per group of loads (1, 2, 4;
                               nm innermost takes 0 only); 0 = default */
    int32_t  tile_k;        /* STAGED: reduction values staged per step; 0 = default */
    int32_t  unroll;        /* DIRECT: reduction steps whose loads are issued before their FMAs;
                               FP64 MFMA columns: 4-deep reduction steps per group of loads in flight
                               (1..16); BGEMM: 16x16 MFMA tiles per work item (1, 2, 4, 8), each
                               holding floor(16/n) instances of size n; 0 = default */
    int32_t  block;         /* threads per workgroup (64..1024, multiple of 64); 0 = default */
    uint32_t flags;         /* SJ_FLAG_* */
    int32_t  order;         /* DIRECT and FP64 MFMA columns: 0 = default, 1 = every workgroup walks the reduction (LTimes) or
                               output (LPlusTimes) rows in ascending order, 2 = each workgroup starts at a
                               different row group (rotation), which spreads concurrent accesses over
                               DRAM channels when rows are megabytes apart.
                               FP64 MFMA rows (LTimes, LPlusTimes and the fused pair): 1 = each lane
                               reads its operand rows from HBM, 2 = a group's rows move as flat runs
                               through LDS (even D and NM); 0 = 2 where it fits.
                               SJ_SCATTERING, FP64 MFMA (the default where g or z is innermost and
                               G <= 32): 1 = tiles taken moments outer (a wave walks along z within a
                               moment), 2 = zone blocks outer (the tiles in flight together take the
                               moments of the same zones); 0 = the nesting's outer axis first (2 in
                               ZDG, else 1).
                               SJ_SCATTERING, DIRECT in the ZDG nesting: 0 or 1 = threads run along z
                               (whole wave on one moment: one matrix per wave where zones of a material
                               are contiguous), 2 = threads run along nm (several degrees per wave, the
                               material's matrices staged in LDS: faster when the material changes from
                               zone to zone); the other DIRECT nestings accept 0, 1 or 2 and ignore it */
    int64_t  rows, inputs, width;  /* MLP: batch rows, input features, hidden width */
} sj_spec;

typedef struct sj_handle_ *sj_handle;
typedef struct sj_plan_ *sj_plan;

typedef struct sj_kernel_info {
    uint32_t struct_size;   /* must be sizeof(sj_kernel_info) */
    int32_t  vgprs, agprs, sgprs;     /* from the compiler's resource-usage report (-1 if unknown); for a
                                         handle built by sj_specialize_with_code, VGPRs, LDS, scratch and
                                         occupancy are read from the loaded function and AGPRs, SGPRs are -1 */
    int32_t  lds_bytes, scratch_bytes, occupancy;  /* occupancy: waves per SIMD (-1 if unknown) */
    int32_t  block;         /* threads per workgroup the handle launches with */
    int64_t  grid;          /* workgroups per launch (LTimes/LPlusTimes/MLP), 0 if data-dependent */
    int32_t  variant;       /* resolved sj_variant */
    int32_t  tile_n, tile_k, unroll;  /* resolved tile parameters */
    double   emit_ms, compile_ms, load_ms;
    uint64_t code_bytes;
    uint64_t key_hash;
    char     kernel_name[64];
} sj_kernel_info;

typedef struct sj_stats_t {
    uint32_t struct_size;   /* must be sizeof(sj_stats_t) */
    uint64_t lookups, hits, misses, compiles, compile_failures, loads, inflight_waits, entries;
    double   emit_ms_total, compile_ms_total, load_ms_total;
} sj_stats_t;

/* Initialize for HIP device `hip_device` (makes it current on the calling
 * thread, reads its gcnArchName, turns comgr's on-disk cache off).
 * Idempotent.  SJ_ERR_NOT_INITIALIZED when the device is absent. */
sj_status sj_init(int hip_device);

/* Parse a layout name ("DGZ" .. "ZGD", case-insensitive) into *out.  The
 * analog of passing a type as a string (section 2, strings as types; section
 * 5.2, layout string from a configuration file). */
sj_status sj_layout_from_string(const char *name, int32_t *out);

/* Canonicalize `spec` for kernel `k` (defaults filled in, tile parameters
 * validated) and return the handle of that specialization, compiling it on a
 * miss: emit source from templates embedded in this library, compile with
 * hiprtc for the device's architecture, load the code object from memory.
 * Errors: SJ_ERR_INVALID_ARG (sizes, enums, tiles, struct_size),
 * SJ_ERR_UNSUPPORTED, SJ_ERR_COMPILE (no cache entry is kept, a retry
 * recompiles), SJ_ERR_LOAD, SJ_ERR_NOT_INITIALIZED. */
sj_status sj_specialize(sj_kernel k, const sj_spec *spec, sj_handle *out);

/* Specialization on values (constant matrix elements, named as future work in
 * ClangJIT section 6): like sj_specialize for SJ_LTIMES / SJ_LPLUSTIMES in FP64
 * with the DIRECT structure, with the weight matrix's values compiled into the
 * kernel.  `weights` is host memory holding the matrix the kernel would read
 * (L row-major [NM][D] for LTimes, L+ row-major [D][NM] for LPlusTimes),
 * `count` = NM * D doubles, all finite; it is read during the call only (the
 * caller keeps ownership).  Every coefficient becomes a constant of the
 * generated code and the reduction is fully unrolled; a term whose coefficient
 * is +0 or -0 is not generated, so an input row that only zero coefficients
 * reach is never read (a NaN or Inf in such a row no longer propagates).  The
 * key holds two independent 64-bit hashes of the values' bit patterns: equal
 * values return the same handle.  spec->variant must be AUTO or DIRECT and
 * spec->order 0 or 1 (the run-time row rotation of order 2 would make the
 * coefficients' positions unknown at compile time).  sj_run takes the plain
 * kernel's pointers; the weight pointer is checked like the others but not
 * read.  Errors: SJ_ERR_INVALID_ARG (null weights, count != NM * D, a
 * non-finite value, order 2), SJ_ERR_UNSUPPORTED (another kernel, structure
 * or dtype; D * NM * tile_n > 8192 products per thread). */
sj_status sj_specialize_values(sj_kernel k, const sj_spec *spec, const double *weights, size_t count,
                               sj_handle *out);

/* Like sj_specialize, but on a miss the handle is built from `code` instead of
 * being compiled: `code`/`size` must be the code object that sj_handle_code
 * returned for a SJ_FLAG_COMPILE_ONLY specialization of the same spec, made by
 * this library version in another process (the caller owns that buffer; it is
 * copied).  hiprtc serializes compiles within one process, so a tuner spreads
 * compiles over worker processes and adopts the results here.  A hit returns
 * the cached handle and ignores `code`.  SJ_ERR_LOAD when the code object does
 * not load or lacks the expected kernel. */
sj_status sj_specialize_with_code(sj_kernel k, const sj_spec *spec, const void *code, size_t size, sj_handle *out);

/* Launch a specialization.  No cache lookup happens here.  Pointers by kernel:
 *   SJ_LTIMES:     {L [NM*D] f64, psi [D*G*Z] (f64, or f32 for BF16 dtypes), phi [NM*G*Z] (same type as psi)}
 *   SJ_LPLUSTIMES: {L+ [D*NM] f64, phi [NM*G*Z] f64, psi_out [D*G*Z] f64}
 *   SJ_LTIMES_LPLUS: {L [NM*D], L+ [D*NM], psi [D*G*Z], psi_out [D*G*Z]} or the same with
 *                  phi [NM*G*Z] appended when the moments are wanted too (all f64); psi_out =
 *                  L+ (L psi) with the moments kept on chip (FP64; DIRECT structure, or
 *                  the matrix-core row structure when D is innermost)
 *   SJ_SCATTERING: {S [count*(n_max+1)*G*G] f64, mat [Z] int32, phi [NM*G*Z] f64, phi_out [NM*G*Z] f64}
 *                  with n_max = floor(sqrt(NM - 1)); S row-major [material][degree][g][g'] (row g receives
 *                  from group g'); phi and phi_out in the spec's nesting with D read as NM; the degree of
 *                  moment nm is floor(sqrt(nm)).  A zone whose material is outside [0, count) gets NaN
 *                  outputs (nothing is read out of range).  Overwrites phi_out.
 *   SJ_MASS:       {B1 [Q1D*D1D] f64, D [NE*Q1D^dim] f64, X [NE*D1D^dim] f64, Y [NE*D1D^dim] f64} with
 *                  spec->D = D1D (dofs per direction, 1..32), spec->NM = Q1D (points per direction, 1..32),
 *                  spec->inputs = dim (1, 2, 3), spec->count = NE (elements); B1 row-major [Q1D][D1D] (the
 *                  1-D basis at the points); per element the first index component is fastest; tile_n =
 *                  elements per wave (0 = default).  y_e = B^T diag(D_e) B x_e, B the dim-fold tensor
 *                  product of B1 (the Laghos-style partial-assembly mass action); overwrites Y.
 *   SJ_MLP_FWD:    {theta f32, X [rows*inputs] f32, y [rows] f32}
 *   SJ_MLP_BWD:    {theta f32, X [rows*inputs] f32, t [rows] f32, grad f32 (same packing as theta), loss [1] f32,
 *                  workspace [rows*(4*width+2)] f32}
 *   SJ_ADAM:       use sj_run_adam.
 * Checks: handle runnable, nptrs, pointers non-null and 16-byte aligned
 * (SJ_ERR_ALIGN), no overlap between an input and an output byte range
 * (SJ_ERR_ALIAS: the no-alias guarantee that section 2 derives from unique
 * objects).  SJ_BGEMM handles run through a plan instead. */
sj_status sj_run(sj_handle h, void *const *ptrs, int nptrs, void *stream);

/* Same math through the ahead-of-time generic kernels: sizes and strides are
 * kernel arguments, no compile.  Supports SJ_LTIMES / SJ_LPLUSTIMES in SJ_F64
 * (pointers as sj_run) and SJ_BGEMM with spec->count instances and pointers
 * {n [count] int32 (device), off [count] int64 (device, element offsets), A, B, C}. */
sj_status sj_generic_run(sj_kernel k, const sj_spec *spec, void *const *ptrs, int nptrs, void *stream);

/* Batched small products C_i = A_i * B_i, FP64, square n_i x n_i, row-major,
 * packed: instance i starts at element off_i = sum_{j<i} n_j^2 of each of A, B, C.
 * sj_batch_plan: h from sj_specialize(SJ_BGEMM, ...); n_host[count] with
 * 1 <= n_i <= 16 and class n_i present in the handle's class mask.  Sorts the
 * instances into size classes and uploads the work list (device memory owned
 * by the plan).  sj_batch_run: one persistent launch on `stream`.
 * sj_batch_graph_capture: records that launch into a HIP graph bound to A, B, C;
 * sj_batch_graph_launch replays it. */
sj_status sj_batch_plan(sj_handle h, const int32_t *n_host, int64_t count, sj_plan *out);
sj_status sj_batch_run(sj_plan p, const double *A, const double *B, double *C, void *stream);
sj_status sj_batch_graph_capture(sj_plan p, const double *A, const double *B, double *C, void *stream);
sj_status sj_batch_graph_launch(sj_plan p, void *stream);
/* Device arrays of the plan: n [count] int32 and off [count] int64 in the
 * caller's instance order (usable with sj_generic_run(SJ_BGEMM)), and the
 * total element count of each packed array. */
sj_status sj_batch_plan_arrays(sj_plan p, const int32_t **n_dev, const int64_t **off_dev, int64_t *total_elems);
sj_status sj_plan_destroy(sj_plan p);

/* One Adam step (Kingma & Ba 2015) on `n` FP32 parameters for a handle from
 * sj_specialize(SJ_ADAM, spec with rows = n):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * ptrs = {p, g, m, v}; step >= 1. */
sj_status sj_run_adam(sj_handle h, void *const *ptrs, int nptrs, int64_t step,
                      double lr, double b1, double b2, double eps, void *stream);

/* The MLP backward pass of an SJ_MLP_BWD handle, as sj_run computes it, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  ptrs = {theta, X, t, grad, loss}
 * as for sj_run without the workspace: the per-row activations and deltas go
 * to a static device array of 1,048,576 floats (4 MiB) that each device this
 * library runs on holds until the process ends.  Requires rows * (4 width + 2)
 * <= 1,048,576 (else SJ_ERR_INVALID_ARG, nothing launched).  Calls no
 * allocator.  Every call on one device shares that device's array: calls that
 * overlap on one device (different streams) race and must be ordered by the
 * caller.  Results equal sj_run's bit for bit (same kernels, same order).
 * Errors: as sj_run, plus SJ_ERR_HIP if the array's device address cannot be
 * resolved. */
sj_status sj_run_mlp_bwd_noalloc(sj_handle h, void *const *ptrs, int nptrs, void *stream);

/* Time a specialization (the measurement primitive of the autotuner): `warmup`
 * untimed launches, then `reps` launches, each bracketed by HIP events on
 * `stream`.  When flush_bytes > 0 the caller's scratch buffer `flush`
 * (16-byte aligned, else SJ_ERR_ALIGN) is read in full before every timed
 * launch (outside the bracket, with ordinary loads, which take over the lines
 * of L2 and of the 256 MB last-level cache) so the launch does not find its
 * operands there.  Reading, not writing: a written buffer would leave dirty
 * lines whose write-back falls into the timed launch.  A launch whose stores
 * stay in the caches (ordinary stores) leaves part of its own write-back for
 * after its end event; timing without a flush, launch after launch, counts it.
 * times_ms[reps] receives each launch's duration; the stream is synchronized
 * before returning.  Pointers as for sj_run. */
sj_status sj_time_run(sj_handle h, void *const *ptrs, int nptrs, int warmup, int reps, void *flush,
                      size_t flush_bytes, void *stream, float *times_ms);

/* The canonical request `spec` resolves to for kernel `k`, without compiling:
 * *out receives the spec with every default filled in (variant, tile_n,
 * tile_k, unroll, block, order) and the load and store forms of LTimes /
 * LPlusTimes / the fused kernel made explicit in flags (one of
 * SJ_FLAG_LOADS_CACHED / _NONTEMPORAL and one of SJ_FLAG_STORES_CACHED /
 * _NONTEMPORAL), plus SJ_FLAG_INDEX64 when 64-bit indexing is chosen.  Two
 * requests with equal resolutions name the same specialization (the same
 * handle).  Structure-internal fields are reported as the kernel uses them
 * (the FP64 matrix-core row structure: unroll 1 = weight fragments in
 * registers, 0 = in LDS; tile_k = reduction depth per step).  For a cost
 * model or tuner that must see what a request will run.  Errors as
 * sj_specialize's validation (no SJ_ERR_COMPILE / SJ_ERR_LOAD). */
sj_status sj_resolve(sj_kernel k, const sj_spec *spec, sj_spec *out);

/* The source text a spec compiles to (for inspection); `len` is the buffer
 * size, *needed receives the size including the terminating NUL. */
sj_status sj_emit_source(sj_kernel k, const sj_spec *spec, char *buf, size_t len, size_t *needed);

sj_status sj_handle_info(sj_handle h, sj_kernel_info *out);
/* Code object bytes of a handle (also valid for SJ_FLAG_COMPILE_ONLY handles). */
sj_status sj_handle_code(sj_handle h, const void **code, size_t *size);
sj_status sj_stats(sj_stats_t *out);
/* Drop every cache entry and unload its module.  No handle may be in use, and
 * no other call of this library may run concurrently (a lookup racing with the
 * clear could return a handle that is being freed).  Every thread's private
 * front cache is emptied at its next lookup. */
sj_status sj_cache_clear(void);
const char *sj_last_error(void);
const char *sj_status_string(sj_status s);

#ifdef __cplusplus
}
#endif
#endif /* SJ_H */
