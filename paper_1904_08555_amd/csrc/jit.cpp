// Specialization keys, source emission and in-process compilation.
//
// ClangJIT (section 4, Algorithm 1) turns (template, runtime values, type
// strings) into an instantiation and caches it program-wide.  Here the
// "template" is one of the kernel sources embedded in this library, the
// runtime values become compile-time constants in an emitted prologue, and
// hiprtc compiles the result for the device's architecture.  Nothing is read
// from disk: the kernel text is a string constant of this binary (the paper's
// fat-object idea, section 3, reduced to what a GPU kernel needs).
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <sstream>

#include "sj_internal.h"
#include "sj_templates.inc"  // generated at build time from csrc/kernels/*.hipk

namespace sj {

namespace {
thread_local std::string t_err;

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}


constexpr int64_t kMaxDim = 2147483647;  // each size <= 2^31 - 1

}  // namespace

sj_status fail(sj_status s, const std::string &msg)
{
    t_err = msg;
    return s;
}
void clear_error() { t_err.clear(); }

}  // namespace sj

extern "C" const char *sj_last_error(void) { return sj::t_err.c_str(); }

namespace sj {

bool key_equal(const SpecKey &a, const SpecKey &b) { return std::memcmp(&a, &b, sizeof(SpecKey)) == 0; }

uint64_t hash_words(const void *p, size_t bytes)
{
    // Two independent multiply-rotate chains over the 64-bit words, joined by
    // one final mix (the chains overlap in the pipeline; a single chained mix
    // per word was a third of a cache hit's time).
    const size_t n = bytes / 8;
    uint64_t a = 0x243F6A8885A308D3ull, b = 0x13198A2E03707344ull;
    size_t i = 0;
    for (; i + 1 < n; i += 2) {
        uint64_t w0, w1;
        std::memcpy(&w0, (const char *)p + 8 * i, 8);
        std::memcpy(&w1, (const char *)p + 8 * i + 8, 8);
        a = ((a ^ w0) * 0x9E3779B97F4A7C15ull);
        a = (a << 29) | (a >> 35);
        b = ((b ^ w1) * 0xC2B2AE3D27D4EB4Full);
        b = (b << 31) | (b >> 33);
    }
    if (i < n) {
        uint64_t w0;
        std::memcpy(&w0, (const char *)p + 8 * i, 8);
        a = ((a ^ w0) * 0x9E3779B97F4A7C15ull);
    }
    return mix64(a ^ ((b << 17) | (b >> 47)) ^ (uint64_t)bytes);
}

// FNV-1a over the bytes of 64-bit words, then a final avalanche: a hash
// independent of hash_words' multiply-rotate chains (both name a value set).
static uint64_t hash_fnv(const void *p, size_t bytes)
{
    const unsigned char *c = (const unsigned char *)p;
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    return h;
}

sj_status make_values_key(const double *values, size_t count, SpecKey *key)
{
    if (!values) return fail(SJ_ERR_INVALID_ARG, "null weights");
    if (key->kernel != SJ_LTIMES && key->kernel != SJ_LPLUSTIMES)
        return fail(SJ_ERR_UNSUPPORTED, "value specialization applies to LTimes and LPlusTimes");
    if (key->dtype != SJ_F64 || key->variant != SJ_VAR_DIRECT)
        return fail(SJ_ERR_UNSUPPORTED, "value specialization needs FP64 and the DIRECT structure");
    if (count != (size_t)(key->NM * key->D)) return fail(SJ_ERR_INVALID_ARG, "weight count must be NM * D");
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(values[i])) return fail(SJ_ERR_INVALID_ARG, "weights must be finite");
    // every coefficient must be a constant at its FMA: the whole reduction is unrolled
    if (key->D * key->NM * key->tile_n > 8192)
        return fail(SJ_ERR_UNSUPPORTED, "value specialization unrolls at most 8192 products per thread");
    key->full_unroll = 1;
    key->values = 1;
    key->vhash[0] = hash_words(values, count * sizeof(double));
    key->vhash[1] = hash_fnv(values, count * sizeof(double));
    return SJ_OK;
}

uint64_t key_hash(const SpecKey &k)
{
    static_assert(sizeof(SpecKey) % 8 == 0, "key is hashed as 64-bit words");
    return hash_words(&k, sizeof(SpecKey));
}

// ---------------------------------------------------------------- layouts

// Contraction view of a layout: psi [B][D][I], phi [B][NM][I].
static void layout_view(int layout, int64_t Z, int64_t G, int64_t *B, int64_t *I)
{
    switch (layout) {
    case SJ_DGZ:
    case SJ_DZG: *B = 1; *I = G * Z; break;
    case SJ_GDZ: *B = G; *I = Z; break;
    case SJ_ZDG: *B = Z; *I = G; break;
    default: /* GZD, ZGD */ *B = G * Z; *I = 1; break;
    }
}

static bool valid_block(int b) { return b >= 64 && b <= 1024 && b % 64 == 0; }

static sj_status make_key_one(sj_kernel k, const sj_spec *s, int device, const char *arch, SpecKey *out);

// SJ_VAR_AUTO on an FP64 contraction: the preferred structure for the layout,
// and when that one declines the shape (SJ_ERR_UNSUPPORTED: register, LDS or
// size limits) the next structure that accepts it, so that every valid shape
// has a default.  D innermost: MFMA rows, STAGED, DIRECT; a column axis
// innermost: DIRECT, MFMA columns.
// LDS bytes of the nm-innermost scattering MFMA form: 16 zones x G runs of NM moments, run pitch
// NM + 2 (NM + 1 when odd) doubles, zone pitch two doubles more than G runs
static int64_t scattering_block_lds(int64_t NM, int64_t G)
{
    const int64_t nmp = NM + (NM % 2 == 0 ? 2 : 1);
    return 16 * (G * nmp + 2) * 8;
}

sj_status make_key(sj_kernel k, const sj_spec *s, int device, const char *arch, SpecKey *out)
{
    if (!s || !out) return fail(SJ_ERR_INVALID_ARG, "null spec or output");
    if (s->struct_size != sizeof(sj_spec))
        return fail(SJ_ERR_INVALID_ARG, "sj_spec.struct_size does not match this library's sj_spec");
    if (!((k == SJ_LTIMES || k == SJ_LPLUSTIMES || k == SJ_LTIMES_LPLUS) && s->variant == SJ_VAR_AUTO &&
          s->dtype == SJ_F64))
        return make_key_one(k, s, device, arch, out);
    int64_t B = 0, I = 0;
    if (s->layout >= SJ_DGZ && s->layout <= SJ_ZGD && s->Z >= 1 && s->G >= 1) layout_view(s->layout, s->Z, s->G, &B, &I);
    static const int kRows[3] = {SJ_VAR_MFMA, SJ_VAR_STAGED, SJ_VAR_DIRECT};
    static const int kCols[2] = {SJ_VAR_DIRECT, SJ_VAR_MFMA};
    static const int kFusedRows[2] = {SJ_VAR_MFMA, SJ_VAR_DIRECT};
    static const int kFusedCols[1] = {SJ_VAR_DIRECT};
    const int *order = (I == 1) ? kRows : kCols;
    int n = (I == 1) ? 3 : 2;
    if (k == SJ_LTIMES_LPLUS) {
        order = (I == 1) ? kFusedRows : kFusedCols;
        n = (I == 1) ? 2 : 1;
    }
    sj_status st = SJ_ERR_UNSUPPORTED;
    for (int i = 0; i < n; ++i) {
        sj_spec t = *s;
        t.variant = order[i];
        st = make_key_one(k, &t, device, arch, out);
        if (st != SJ_ERR_UNSUPPORTED) return st;
    }
    return st;
}

static sj_status make_key_one(sj_kernel k, const sj_spec *s, int device, const char *arch, SpecKey *out)
{
    if (!s || !out) return fail(SJ_ERR_INVALID_ARG, "null spec or output");
    if (s->struct_size != sizeof(sj_spec))
        return fail(SJ_ERR_INVALID_ARG, "sj_spec.struct_size does not match this library's sj_spec");
    SpecKey key;
    std::memset(&key, 0, sizeof key);
    key.kernel = (int32_t)k;
    key.dtype = s->dtype;
    key.device = device;
    key.lib_version = SJ_VERSION;
    std::snprintf(key.arch, sizeof key.arch, "%s", arch ? arch : "");
    key.flags = s->flags & (SJ_FLAG_COMPILE_ONLY | SJ_FLAG_DEBUG_FAIL_COMPILE | SJ_FLAG_LOADS_CACHED |
                            SJ_FLAG_LOADS_NONTEMPORAL | SJ_FLAG_STORES_CACHED | SJ_FLAG_STORES_NONTEMPORAL |
                            SJ_FLAG_ACCUMULATE | SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED);
    if ((s->flags & SJ_FLAG_XCD_CONTIGUOUS) && (s->flags & SJ_FLAG_XCD_INTERLEAVED))
        return fail(SJ_ERR_INVALID_ARG, "SJ_FLAG_XCD_CONTIGUOUS and SJ_FLAG_XCD_INTERLEAVED exclude each other");
    if ((s->flags & (SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED)) && k != SJ_LTIMES && k != SJ_LPLUSTIMES &&
        k != SJ_LTIMES_LPLUS && k != SJ_SCATTERING)
        return fail(SJ_ERR_INVALID_ARG, "the XCD flags apply to LTimes, LPlusTimes, the fused kernel and scattering");
    if ((s->flags & SJ_FLAG_ACCUMULATE) && k != SJ_LTIMES && k != SJ_LPLUSTIMES)
        return fail(SJ_ERR_INVALID_ARG, "SJ_FLAG_ACCUMULATE applies to LTimes and LPlusTimes");
    if (k == SJ_LTIMES_LPLUS) {
        // LTimes then LPlusTimes in one pass: FP64; the DIRECT structure, or the FP64 matrix-core
        // row structure when D is innermost (GZD, ZGD)
        if (s->dtype != SJ_F64) return fail(SJ_ERR_UNSUPPORTED, "the fused kernel is FP64 only");
        if (s->variant == SJ_VAR_STAGED)
            return fail(SJ_ERR_UNSUPPORTED, "the fused kernel has the DIRECT and MFMA (D innermost) structures");
    }
    if ((s->flags & SJ_FLAG_LOADS_CACHED) && (s->flags & SJ_FLAG_LOADS_NONTEMPORAL))
        return fail(SJ_ERR_INVALID_ARG, "SJ_FLAG_LOADS_CACHED and SJ_FLAG_LOADS_NONTEMPORAL exclude each other");
    if ((s->flags & SJ_FLAG_STORES_CACHED) && (s->flags & SJ_FLAG_STORES_NONTEMPORAL))
        return fail(SJ_ERR_INVALID_ARG, "SJ_FLAG_STORES_CACHED and SJ_FLAG_STORES_NONTEMPORAL exclude each other");

    if (k == SJ_LTIMES || k == SJ_LPLUSTIMES || k == SJ_LTIMES_LPLUS) {
        if (s->layout < SJ_DGZ || s->layout > SJ_ZGD) return fail(SJ_ERR_INVALID_ARG, "layout out of range");
        const int64_t dims[4] = {s->Z, s->G, s->D, s->NM};
        for (int64_t v : dims)
            if (v < 1 || v > kMaxDim) return fail(SJ_ERR_INVALID_ARG, "sizes must be in [1, 2^31-1]");
        if (s->D > 4096 || s->NM > 4096) return fail(SJ_ERR_UNSUPPORTED, "D and NM are limited to 4096");
        // element counts (checked for overflow of int64 first)
        const int64_t cols = s->G * s->Z;  // < 2^62
        if (cols > (int64_t(1) << 50)) return fail(SJ_ERR_INVALID_ARG, "G*Z too large");
        const int64_t maxa = std::max(s->D, s->NM);
        if (cols > (INT64_MAX / 16) / maxa) return fail(SJ_ERR_INVALID_ARG, "array size overflows");
        if (s->dtype == SJ_F64) {
        } else if (s->dtype == SJ_BF16 || s->dtype == SJ_BF16X3) {
            if (k != SJ_LTIMES) return fail(SJ_ERR_UNSUPPORTED, "BF16 dtypes are implemented for LTimes only");
        } else {
            return fail(SJ_ERR_INVALID_ARG, "dtype must be SJ_F64, SJ_BF16 or SJ_BF16X3");
        }
        key.layout = s->layout;
        key.Z = s->Z; key.G = s->G; key.D = s->D; key.NM = s->NM;
        layout_view(s->layout, s->Z, s->G, &key.B, &key.I);
        const int64_t nelem = cols * maxa;
        key.index64 = (nelem >= (int64_t(1) << 31) || (s->flags & SJ_FLAG_INDEX64)) ? 1 : 0;

        int var = s->variant;
        if (var == SJ_VAR_AUTO) {
            if (s->dtype != SJ_F64) var = SJ_VAR_MFMA;
            else var = key.I == 1 ? SJ_VAR_MFMA : SJ_VAR_DIRECT;
        }
        if (s->dtype != SJ_F64 && var != SJ_VAR_MFMA)
            return fail(SJ_ERR_INVALID_ARG, "BF16 dtypes need the MFMA variant");
        if (var < SJ_VAR_DIRECT || var > SJ_VAR_MFMA) return fail(SJ_ERR_INVALID_ARG, "variant out of range");
        key.variant = var;
        const int64_t red = (k == SJ_LPLUSTIMES) ? s->NM : s->D;   // reduction length (first phase when fused)
        const int64_t outn = (k == SJ_LPLUSTIMES) ? s->D : s->NM;  // outputs per column (first phase when fused)
        if (var == SJ_VAR_DIRECT) {
            key.block = s->block ? s->block : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            int vec = s->tile_n;
            if (vec == 0) vec = (key.I % 2 == 0 && s->NM <= 16) ? 2 : 1;
            if (vec != 1 && vec != 2 && vec != 4) return fail(SJ_ERR_INVALID_ARG, "DIRECT tile_n (columns per thread) must be 1, 2 or 4");
            if (key.I % vec != 0) return fail(SJ_ERR_INVALID_ARG, "DIRECT tile_n must divide the contiguous column extent");
            key.tile_n = vec;
            int un = s->unroll ? s->unroll : 8;
            if (un < 1 || un > 64) return fail(SJ_ERR_INVALID_ARG, "unroll must be in [1, 64]");
            key.unroll = (int32_t)std::min<int64_t>(un, k == SJ_LTIMES ? s->D : s->D);
            // Accumulators (LTimes) or moments (LPlusTimes, both for the fused kernel) live in registers.
            const int64_t regs = s->NM * vec;
            if (regs > 128) return fail(SJ_ERR_UNSUPPORTED, "NM * tile_n > 128 FP64 values per thread");
            // Full unrolling while the straight-line body stays moderate (the fused kernel has two phases).
            key.full_unroll = (red * outn * vec * (k == SJ_LTIMES_LPLUS ? 2 : 1) <= 4096) ? 1 : 0;
            key.tile_k = 0;
            // Rotation pays when consecutive rows are >= 1 MiB apart (measured on MI355X:
            // 8 MiB row stride, 5.35 TB/s ascending vs 6.2 TB/s rotated).
            int order = s->order;
            if (order == 0) order = (key.I * 8 >= (int64_t(1) << 20)) ? 2 : 1;
            if (order != 1 && order != 2) return fail(SJ_ERR_INVALID_ARG, "order must be 0, 1 or 2");
            if ((k == SJ_LTIMES ? s->D : s->D) < 2 * key.unroll) order = 1;  // fewer than two row groups
            key.order = order;
        } else if (var == SJ_VAR_STAGED) {
            if (s->order != 0 && s->order != 1) return fail(SJ_ERR_INVALID_ARG, "this structure has no order 2");
            key.order = 1;
            if (key.I != 1) return fail(SJ_ERR_UNSUPPORTED, "STAGED needs a layout with D innermost (GZD, ZGD)");
            key.block = s->block ? s->block : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            key.tile_n = s->tile_n ? s->tile_n : key.block;
            if (key.tile_n % key.block != 0 || key.tile_n / key.block > 4)
                return fail(SJ_ERR_INVALID_ARG, "STAGED tile_n (rows per workgroup) must be block, 2*block, 3*block or 4*block");
            key.tile_k = s->tile_k ? s->tile_k : 16;
            if (key.tile_k < 1 || key.tile_k > 256) return fail(SJ_ERR_INVALID_ARG, "tile_k must be in [1, 256]");
            key.tile_k = (int32_t)std::min<int64_t>(key.tile_k, s->D);
            const int64_t rpt = key.tile_n / key.block;
            if (s->NM * rpt > 128) return fail(SJ_ERR_UNSUPPORTED, "NM * rows per thread > 128 FP64 values per thread");
            // STAGED unrolls every chunk of the reduction (or of the outputs) at compile time:
            // bound that work, or hiprtc's time grows without limit (D = 4096 took over half an
            // hour, D = 512 with NM = 16 eleven seconds)
            const int64_t nchunk = (s->D + key.tile_k - 1) / key.tile_k;
            if (nchunk > 16 || s->D * s->NM * rpt > 4096)
                return fail(SJ_ERR_UNSUPPORTED, "STAGED unrolls at most 16 chunks and 4096 products per row set");
            const int64_t lds = (int64_t)key.tile_n * std::max<int64_t>(key.tile_k + 1, s->NM + 1) * 8;
            if (lds > 160 * 1024) return fail(SJ_ERR_INVALID_ARG, "STAGED tile exceeds 160 KiB of LDS");
            key.unroll = 0;
            key.full_unroll = 1;
        } else if (k == SJ_LTIMES_LPLUS) {
            // Fused FP64 matrix-core row kernel (D innermost): tile_n = 16-row tiles per wave (per
            // group); both phases' weight fragments and per-wave tiles live in LDS.  order 1 = lanes
            // read psi rows directly, order 2 = contiguous runs of psi, phi and out staged in LDS.
            if (key.I != 1) return fail(SJ_ERR_UNSUPPORTED, "the fused MFMA kernel needs D innermost (GZD, ZGD)");
            if (s->order < 0 || s->order > 2) return fail(SJ_ERR_INVALID_ARG, "order must be 0, 1 or 2");
            if (s->unroll != 0) return fail(SJ_ERR_INVALID_ARG, "the fused MFMA kernel takes no unroll");
            key.block = s->block ? s->block : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            int rt = s->tile_n;
            if (rt == 0) rt = 1;   // measured on MI355X at D=96, NM=16: 336 us (1 tile) vs 347 us (2 tiles)
            if (rt < 1 || rt > 8) return fail(SJ_ERR_INVALID_ARG, "MFMA tile_n (16-row tiles per wave) must be in [1, 8]");
            const int64_t bd = (s->D + 15) / 16, bn = (s->NM + 15) / 16;
            if (rt * std::max(bd, bn) * 4 > 96) return fail(SJ_ERR_UNSUPPORTED, "MFMA accumulators exceed 96 FP64 values per lane");
            // registers per lane: the loads in flight, both phases' accumulators and about 20 more,
            // against 512 / (waves per SIMD the block needs)
            const int64_t budget = 512 / std::max(1, key.block / 256);
            const int64_t frags = 2 * bd * 4 * bn * 64 * 8;
            auto fits = [&](int order, const char **why) {
                const int64_t pf = std::min<int64_t>(std::max<int64_t>(12 / rt, 1), bd);
                const int64_t nj = (16 * rt * s->D / 2 + 63) / 64;
                const int64_t inflight = (order == 2) ? 2 * nj : pf * rt * 4;
                const int64_t tiles = (order == 2) ? 16 * rt * ((16 * bd + 2) + (16 * bn + 2)) * 8 : 16 * rt * (16 * bn + 2) * 8;
                if (order == 2 && (s->D % 2 != 0 || s->NM % 2 != 0)) return *why = "order 2 needs even D and NM", false;
                if (order == 2 && nj > 32) return *why = "order 2 holds at most 32 loads per lane", false;
                if (2 * (inflight + rt * bd * 4 + rt * bn * 4) + 20 > budget)
                    return *why = "fused MFMA registers exceed what the block size leaves per lane", false;
                if (frags + (int64_t)(key.block / 64) * tiles > 160 * 1024)
                    return *why = "fused MFMA fragments and tiles exceed 160 KiB of LDS", false;
                return true;
            };
            const char *why = "";
            int order = s->order;
            if (order == 0) order = fits(2, &why) ? 2 : 1;
            if (!fits(order, &why)) return fail(SJ_ERR_UNSUPPORTED, why);
            key.order = order;
            key.tile_n = rt;
            key.unroll = 0;
            key.tile_k = 16;
            key.full_unroll = 1;
        } else if (s->dtype == SJ_F64 && key.I > 1) {
            // FP64 matrix-core column contraction: tile_n = columns per lane (1, 2, 4),
            // unroll = 4-deep reduction steps per group of loads in flight, order 2 = rotated groups.
            key.block = s->block ? s->block : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            const int64_t ob = (outn + 15) / 16, ks = (red + 3) / 4;
            int t = s->tile_n;
            if (t == 0) {   // widest tile whose accumulators stay within 32 FP64 values per lane
                t = 1;
                for (int c = 4; c >= 2; c /= 2)
                    if (key.I % c == 0 && ob * 4 * c <= 32) { t = c; break; }
            }
            if (t != 1 && t != 2 && t != 4) return fail(SJ_ERR_INVALID_ARG, "MFMA tile_n (columns per lane) must be 1, 2 or 4");
            if (key.I % t != 0) return fail(SJ_ERR_INVALID_ARG, "MFMA tile_n must divide the contiguous column extent");
            if (ob * 4 * t > 128) return fail(SJ_ERR_UNSUPPORTED, "MFMA accumulators exceed 128 FP64 values per lane");
            int pf = s->unroll;
            if (pf == 0) pf = (int)std::max<int64_t>(1, std::min<int64_t>(16 / t, 32 / (ob * t)));
            if (pf < 1 || pf > 16) return fail(SJ_ERR_INVALID_ARG, "MFMA unroll (steps per group) must be in [1, 16]");
            key.unroll = (int32_t)std::min<int64_t>(pf, ks);
            if (ks * ob * 64 * 8 > 160 * 1024)
                return fail(SJ_ERR_UNSUPPORTED, "MFMA weight fragments exceed 160 KiB of LDS");
            int order = s->order;
            if (order == 0) order = (key.I * 8 >= (int64_t(1) << 20)) ? 2 : 1;
            if (order != 1 && order != 2) return fail(SJ_ERR_INVALID_ARG, "order must be 0, 1 or 2");
            if ((ks + key.unroll - 1) / key.unroll < 2) order = 1;   // a single group
            key.order = order;
            key.tile_n = t;
            key.tile_k = 4;
            key.full_unroll = 0;
        } else if (s->dtype == SJ_F64) {
            // FP64 matrix-core row contraction (D innermost): tile_n = 16-row tiles per wave (per
            // group); order 1 = every lane reads its operands from HBM, order 2 = a group's rows are
            // read and written as one contiguous run staged through LDS, persistent grid.
            if (s->order < 0 || s->order > 2) return fail(SJ_ERR_INVALID_ARG, "order must be 0, 1 or 2");
            if (s->block && !valid_block(s->block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            if (s->tile_n < 0 || s->tile_n > 8) return fail(SJ_ERR_INVALID_ARG, "MFMA tile_n (16-row tiles per wave) must be in [1, 8]");
            const int64_t ob = (outn + 15) / 16, kb = (red + 15) / 16;
            const int64_t nfrag = kb * 4 * ob;
            key.unroll = nfrag <= 32 ? 1 : 0;       // W fragments in registers (1) or LDS (0)
            if (!key.unroll && nfrag * 64 * 8 > 160 * 1024)
                return fail(SJ_ERR_UNSUPPORTED, "MFMA weight fragments exceed 160 KiB of LDS");
            // order 2: even row lengths, at most 32 16-byte loads per lane in flight, LDS within 160 KiB
            auto run_ok = [&](int64_t rt, int block, const char **why) {
                const int64_t pitch = std::max<int64_t>(16 * kb, outn) + 2;
                const int64_t lds = (int64_t)(block / 64) * 16 * rt * pitch * 8 + (key.unroll ? 0 : nfrag * 64 * 8);
                if (red % 2 != 0 || outn % 2 != 0) return *why = "order 2 needs even D and NM", false;
                if (rt * ob * 4 > 96) return *why = "MFMA accumulators exceed 96 FP64 values per lane", false;
                if ((16 * rt * red / 2 + 63) / 64 > 32) return *why = "order 2 holds at most 32 loads per lane", false;
                if (lds > 160 * 1024) return *why = "order 2 tiles exceed 160 KiB of LDS", false;
                return true;
            };
            int order = s->order, rt = s->tile_n, block = s->block;
            const char *why = "";
            if (order != 1) {
                // defaults measured on MI355X at D=96, NM=16 (ZGD): reduction-heavy rows (LTimes)
                // 2 tiles per wave in 256-thread workgroups, 163 us; output-heavy rows (LPlusTimes)
                // 1 tile in 64-thread workgroups, 153 us; the direct form takes 178 and 157 us
                static const int kTry[3][2] = {{2, 256}, {1, 256}, {1, 64}};
                int first = (red > outn || !key.unroll) ? 0 : 2;   // weights in LDS: share them over a wider block
                bool found = false;
                for (int i = first; i < 3 && !found; ++i) {
                    const int r = rt ? rt : kTry[i][0], b = block ? block : kTry[i][1];
                    if (run_ok(r, b, &why)) { rt = r; block = b; found = true; }
                }
                if (!found && order == 2) return fail(SJ_ERR_UNSUPPORTED, why);
                order = found ? 2 : 1;
            }
            if (order == 1) {
                if (rt == 0) rt = (2 * ob * 4 <= 96) ? 2 : 1;
                if (block == 0) block = 256;
                if (rt * ob * 4 > 96) return fail(SJ_ERR_UNSUPPORTED, "MFMA accumulators exceed 96 FP64 values per lane");
            }
            key.block = block;
            key.order = order;
            key.tile_n = rt;
            key.tile_k = 16;
            key.full_unroll = 1;
        } else {
            // BF16 matrix-core LTimes: column axis contiguous, a 32- or 128-column tile per wave; D
            // innermost (GZD, ZGD), a 16-row tile per wave (tile_n 1; D % 4 == 0 for 16-byte pieces).
            if (s->order != 0 && s->order != 1) return fail(SJ_ERR_INVALID_ARG, "this structure has no order 2");
            key.order = 1;
            key.block = s->block ? s->block : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            if (key.I == 1) {
                if (s->D % 4 != 0) return fail(SJ_ERR_UNSUPPORTED, "BF16 LTimes with D innermost needs D % 4 == 0");
                if (s->tile_n != 0 && s->tile_n != 1)
                    return fail(SJ_ERR_INVALID_ARG, "BF16 LTimes with D innermost takes tile_n 1 (16 rows per wave)");
            }
            // tile_n = columns per lane: 1 (4-byte loads, 32 columns per wave) or 4 (16-byte loads,
            // 128 columns per wave as four interleaved MFMA tiles; needs the column extent % 4 == 0).
            int cpl = s->tile_n;
            if (cpl == 0) cpl = (key.I > 1 && key.I % 4 == 0 && key.block <= 512) ? 4 : 1;
            if (cpl != 1 && cpl != 4) return fail(SJ_ERR_INVALID_ARG, "BF16 tile_n (columns per lane) must be 1 or 4");
            if (cpl == 4 && key.I % 4 != 0) return fail(SJ_ERR_INVALID_ARG, "BF16 tile_n 4 needs a column extent divisible by 4");
            // four columns per lane hold 128 FP32 accumulators: a 1024-thread block leaves 128 registers
            // per lane and the kernel spills (measured 21.9 ms against 2.38 ms at block 256)
            if (cpl == 4 && key.block > 512) return fail(SJ_ERR_UNSUPPORTED, "BF16 tile_n 4 needs a block of at most 512 threads");
            key.tile_n = cpl;
            // L's hi (and lo) fragments: 32x16 tiles in the column forms, 16x32 in the row form
            const int64_t frag_bytes = (key.I == 1 ? ((s->NM + 15) / 16) * ((s->D + 31) / 32)
                                                   : ((s->NM + 31) / 32) * ((s->D + 15) / 16)) * 64 * 16;
            if (frag_bytes * (s->dtype == SJ_BF16X3 ? 2 : 1) > 160 * 1024)
                return fail(SJ_ERR_UNSUPPORTED, "BF16 weight fragments exceed 160 KiB of LDS");
            if (s->D > 256) return fail(SJ_ERR_UNSUPPORTED, "BF16 LTimes keeps a column's D values in registers: D <= 256");
            key.tile_k = 16;
            if (s->unroll != 0) return fail(SJ_ERR_INVALID_ARG, "BF16 takes no unroll");
            key.unroll = 0;
            key.full_unroll = 1;
        }
        (void)outn;
        // the load and store forms become explicit, so that requests that resolve to the same
        // kernel (a policy flag equal to the default) share one key
        int ntl = 0, nts = 0;
        load_store_policy(key, &ntl, &nts);
        key.flags &= ~(SJ_FLAG_LOADS_CACHED | SJ_FLAG_LOADS_NONTEMPORAL | SJ_FLAG_STORES_CACHED |
                       SJ_FLAG_STORES_NONTEMPORAL);
        key.flags |= (ntl ? SJ_FLAG_LOADS_NONTEMPORAL : SJ_FLAG_LOADS_CACHED) |
                     (nts ? SJ_FLAG_STORES_NONTEMPORAL : SJ_FLAG_STORES_CACHED);
        const bool xcd = xcd_contiguous(key);
        key.flags &= ~(SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED);
        key.flags |= xcd ? SJ_FLAG_XCD_CONTIGUOUS : SJ_FLAG_XCD_INTERLEAVED;
        return (*out = key), SJ_OK;
    }
    if (k == SJ_MASS) {
        // tensor-product mass operator (partial assembly): D = D1D, NM = Q1D, inputs = dim, count = NE
        if (s->dtype != SJ_F64) return fail(SJ_ERR_INVALID_ARG, "the mass operator is FP64 (dtype SJ_F64)");
        if (s->inputs < 1 || s->inputs > 3) return fail(SJ_ERR_INVALID_ARG, "inputs (dimension) must be 1, 2 or 3");
        if (s->D < 1 || s->D > 32 || s->NM < 1 || s->NM > 32)
            return fail(SJ_ERR_INVALID_ARG, "D (dofs per direction) and NM (points per direction) must be in [1, 32]");
        if (s->count < 1 || s->count > (int64_t(1) << 31) - 1) return fail(SJ_ERR_INVALID_ARG, "count (elements) must be in [1, 2^31-1]");
        if (s->variant != SJ_VAR_AUTO && s->variant != SJ_VAR_DIRECT)
            return fail(SJ_ERR_UNSUPPORTED, "the mass operator has the DIRECT structure only");
        if (s->tile_k != 0 || s->unroll != 0 || s->order < 0 || s->order > 2 || (s->flags & SJ_FLAG_ACCUMULATE))
            return fail(SJ_ERR_INVALID_ARG, "the mass operator takes tile_n, block and order (0, 1, 2) only");
        // order 1: one group of elements per wave, x and D staged in LDS; order 2: persistent waves
        // that load the next group into registers while computing the current one (D stays in
        // registers)
        int order = s->order;
        const int64_t dim = s->inputs, D1D = s->D, Q1D = s->NM, mx = std::max(D1D, Q1D);
        int64_t nd = 1, nq = 1, ns = 1, mxlo = 1;
        for (int64_t i = 0; i < dim; ++i) { nd *= D1D; nq *= Q1D; ns *= mx; }
        for (int64_t i = 0; i + 1 < dim; ++i) mxlo *= mx;
        // elements per wave: measured on MI355X at D1D=4 Q1D=6, hexahedra 1 (441 us; 2: 550 us),
        // quadrilaterals 4 (276 us; 10: 335 us): about 24 pencils in the widest contraction
        // The pipelined form (order 2) holds a group's x and two groups' D values per lane in
        // registers: nlx + 2 nld doubles.  Defaults measured on MI355X (500,000 hexahedra and
        // 2,000,000 quadrilaterals, D1D=4 Q1D=6): pipelined with the largest group of at most 8
        // elements whose registers stay within 40 doubles (hexahedra 4: 274 us, 1: 368 us;
        // quadrilaterals 8: 209 us, 4: 242 us), 64-thread workgroups; where even one element
        // exceeds that, the staged form with about 24 pencils in the widest contraction (the
        // pipelined form spills beyond about 90 doubles).
        auto regs = [&](int64_t e) { return (e * nd + 63) / 64 + 2 * ((e * nq + 63) / 64); };
        int ew = s->tile_n;
        if (ew == 0) {
            if (order != 1 && regs(1) <= 40) {
                ew = 1;
                while (ew < 8 && regs(2 * ew) <= 40) ew *= 2;
                if (order == 0) order = 2;
            } else {
                ew = (int)std::max<int64_t>(1, std::min<int64_t>(32, 24 / mxlo));
            }
        }
        if (ew < 1 || ew > 64) return fail(SJ_ERR_INVALID_ARG, "tile_n (elements per wave) must be in [1, 64]");
        if (order == 0) order = (regs(ew) <= 40) ? 2 : 1;
        auto lds = [&](int block) { return (int64_t)(block / 64) * ew * (2 * ns + (order == 1 ? nq : 0)) * 8; };
        int block = s->block;
        if (block == 0) block = (order == 2) ? 64 : (lds(128) <= 64 * 1024) ? 128 : 64;
        if (!valid_block(block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
        if (lds(block) > 160 * 1024) return fail(SJ_ERR_UNSUPPORTED, "mass operator tiles exceed 160 KiB of LDS");
        if (s->count * std::max(nd, nq) > (int64_t(1) << 50)) return fail(SJ_ERR_INVALID_ARG, "arrays too large");
        key.D = D1D; key.NM = Q1D; key.inputs = dim; key.rows = s->count;
        key.tile_n = ew; key.block = block; key.variant = SJ_VAR_DIRECT; key.order = order;
        key.index64 = (s->count * std::max(nd, nq) >= (int64_t(1) << 31) || (s->flags & SJ_FLAG_INDEX64)) ? 1 : 0;
        return (*out = key), SJ_OK;
    }
    if (k == SJ_SCATTERING) {
        // scattering source over the six nestings of the moment arrays: one thread per (nm, z) line
        if (s->dtype != SJ_F64) return fail(SJ_ERR_INVALID_ARG, "scattering is FP64 (dtype SJ_F64)");
        if (s->layout < SJ_DGZ || s->layout > SJ_ZGD) return fail(SJ_ERR_INVALID_ARG, "layout out of range");
        const int64_t dims[3] = {s->Z, s->G, s->NM};
        for (int64_t v : dims)
            if (v < 1 || v > kMaxDim) return fail(SJ_ERR_INVALID_ARG, "sizes must be in [1, 2^31-1]");
        if (s->count < 1 || s->count > 65536) return fail(SJ_ERR_INVALID_ARG, "count (materials) must be in [1, 65536]");
        if (s->NM > 4096) return fail(SJ_ERR_UNSUPPORTED, "NM is limited to 4096");
        if (s->G > 64) return fail(SJ_ERR_UNSUPPORTED, "scattering keeps a line's G values in registers: G <= 64");
        if (s->variant != SJ_VAR_AUTO && s->variant != SJ_VAR_DIRECT && s->variant != SJ_VAR_MFMA)
            return fail(SJ_ERR_UNSUPPORTED, "scattering has the DIRECT and MFMA structures");
        if (s->tile_k != 0 || s->unroll != 0 || s->order < 0 || s->order > 2)
            return fail(SJ_ERR_INVALID_ARG, "scattering takes tile_n (MFMA only) and order 0, 1 or 2");
        if (s->flags & SJ_FLAG_ACCUMULATE) return fail(SJ_ERR_INVALID_ARG, "scattering overwrites its output");
        const int64_t lines = s->NM * s->Z;
        if (lines > (int64_t(1) << 40) || s->G * lines > (int64_t(1) << 50)) return fail(SJ_ERR_INVALID_ARG, "array size overflows");
        int64_t nl = 0;
        while ((nl + 1) * (nl + 1) <= s->NM - 1) ++nl;
        nl += 1;
        if (s->count * nl * s->G * s->G > (int64_t(1) << 40)) return fail(SJ_ERR_INVALID_ARG, "S too large");
        key.layout = s->layout;
        key.Z = s->Z; key.G = s->G; key.NM = s->NM;
        key.rows = s->count;   // materials
        key.variant = SJ_VAR_DIRECT;
        // LDS of the emitted kernel (see the emission): per-wave line tiles where g is innermost and
        // consecutive lines are contiguous, and the staged degree matrices where lanes run along nm
        int64_t snm = 0, sg = 0, sz = 0;
        const int64_t NMv = s->NM, Gv = s->G, Zv = s->Z;
        switch (s->layout) {
        case SJ_DGZ: snm = Gv * Zv; sg = Zv; sz = 1; break;
        case SJ_DZG: snm = Zv * Gv; sz = Gv; sg = 1; break;
        case SJ_GDZ: sg = NMv * Zv; snm = Zv; sz = 1; break;
        case SJ_GZD: sg = Zv * NMv; sz = NMv; snm = 1; break;
        case SJ_ZDG: sz = NMv * Gv; snm = Gv; sg = 1; break;
        default: sz = Gv * NMv; sg = NMv; snm = 1; break;
        }
        // the default structure: the FP64 matrix cores wherever g or z is innermost and G <= 32
        // (measured on MI355X at Z=32768 G=32 NM=16, four materials in zone regions, each launch
        // after a 1 GiB read that empties the last-level cache: DZG 60.4 us against 135-138 us,
        // ZDG 59.4 us against 148 us, DGZ 64.2 us against 76 us, GDZ 72.5 us against 80 us;
        // materials drawn per zone 142-252 us against 340-358 us)
        const bool mfma = (s->variant == SJ_VAR_MFMA) ||
                          (s->variant == SJ_VAR_AUTO && (sg == 1 || sz == 1) && Gv <= 32);
        if (mfma) {
            // FP64 matrix cores: tiles of one moment and 16 zones, tile_n tiles per group of loads,
            // persistent waves, the fragments of a matrix in registers; g innermost: the tile's
            // lines through LDS rows; z innermost: lanes along z, no LDS
            if (Gv > 32) return fail(SJ_ERR_UNSUPPORTED, "the scattering MFMA structure holds G <= 32");
            if (sg != 1 && sz != 1) {
                // nm innermost (GZD, ZGD): blocks of 16 zones staged whole in LDS, one tile per moment
                if (s->tile_n != 0) return fail(SJ_ERR_INVALID_ARG, "the nm-innermost MFMA form takes no tile_n");
                if (s->order > 1) return fail(SJ_ERR_INVALID_ARG, "the nm-innermost MFMA form has order 1 only");
                key.variant = SJ_VAR_MFMA;
                key.tile_n = 1;
                key.order = 1;
                // measured on MI355X at Z=32768 G=32 NM=16, zone regions: GZD 80 us at 512 threads against
                // 99 at 256; ZGD 68 us at 256 against 73 at 512
                key.block = s->block ? s->block : (sz < sg ? 512 : 256);
                if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
                if (scattering_block_lds(NMv, Gv) + 512 > 160 * 1024)
                    return fail(SJ_ERR_UNSUPPORTED, "a 16-zone block of the nm-innermost MFMA form exceeds 160 KiB of LDS");
                key.index64 = (s->G * lines >= (int64_t(1) << 31) || s->count * nl * s->G * s->G >= (int64_t(1) << 31) ||
                               (s->flags & SJ_FLAG_INDEX64)) ? 1 : 0;
                const bool xcd = (s->flags & SJ_FLAG_XCD_CONTIGUOUS) != 0;
                key.flags &= ~(SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED);
                key.flags |= xcd ? SJ_FLAG_XCD_CONTIGUOUS : SJ_FLAG_XCD_INTERLEAVED;
                return (*out = key), SJ_OK;
            }
            // order 1: moments outer (tiles in flight together run along z); order 2: zone blocks
            // outer (tiles in flight together take the moments of the same zones); default: the
            // nesting's outer axis first
            key.order = s->order ? s->order : (sz > snm ? 2 : 1);
            // defaults measured as above: one tile per group with zone blocks outer (ZDG), else two;
            // 512-thread workgroups for the column form (DGZ 64.2 us against 65.0 at 256, GDZ 72.5
            // against 75.9), 128 with zone blocks outer (ZDG 59.4 against 60.5), else 256
            const int rt = s->tile_n ? s->tile_n : (key.order == 2 ? 1 : 2);
            if (rt != 1 && rt != 2 && rt != 4) return fail(SJ_ERR_INVALID_ARG, "MFMA tile_n (tiles per group) must be 1, 2 or 4");
            key.variant = SJ_VAR_MFMA;
            key.tile_n = rt;
            key.block = s->block ? s->block : (sg != 1) ? 512 : (key.order == 2) ? 128 : 256;
            if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
            const int64_t tp = 16 * ((Gv + 15) / 16) + 2;   // LDS rows where g is innermost
            if (sg == 1 && (int64_t)(key.block / 64) * rt * 16 * tp * 8 + 512 > 160 * 1024)
                return fail(SJ_ERR_UNSUPPORTED, "scattering MFMA tiles exceed 160 KiB of LDS at this block size");
            key.index64 = (s->G * lines >= (int64_t(1) << 31) || s->count * nl * s->G * s->G >= (int64_t(1) << 31) ||
                        (s->flags & SJ_FLAG_INDEX64)) ? 1 : 0;
            const bool xcd = (s->flags & SJ_FLAG_XCD_CONTIGUOUS) != 0;
            key.flags &= ~(SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED);
            key.flags |= xcd ? SJ_FLAG_XCD_CONTIGUOUS : SJ_FLAG_XCD_INTERLEAVED;
            return (*out = key), SJ_OK;
        }
        if (s->tile_n != 0) return fail(SJ_ERR_INVALID_ARG, "tile_n is the MFMA structure's tiles per group");
        const bool run_lines = (sg == 1 && std::min(snm, sz) == Gv);
        // lanes along nm only where nm is the faster axis and g is not innermost, or on request
        // (order 2) in ZDG; measured on MI355X at Z=32768 G=32 NM=16 with four materials in zone
        // regions, ZDG with lanes along z 89.6 us against 103.5 us along nm; with a material drawn
        // per zone, 351 us against 218 us
        const bool zdg_nm = (sg == 1 && snm < sz && s->order == 2);
        const bool lane_nm = (snm < sz) && (sg != 1 || zdg_nm);
        const bool slds = (lane_nm && nl * (Gv * Gv + 2) * 8 <= 64 * 1024);
        const int64_t tp = Gv + (Gv % 2 == 0 ? 2 : 1);
        auto lds = [&](int block) {
            return (run_lines ? (int64_t)(block / 64) * 64 * tp * 8 : 0) + (slds ? nl * (Gv * Gv + 2) * 8 + 8 : 0);
        };
        // measured on MI355X at Z=32768 G=32 NM=16: line tiles and staged matrices (ZDG, lanes along
        // nm) 102.7 us at 384 threads against 116.9 us at 256; persistent line tiles alone (DZG, ZDG)
        // 66.9 and 77.7 us at 128 threads, 65.3 and 80.9 us at 256, 71.0 and 83.3 us at 64; staged
        // matrices with two zones per thread (GZD, ZGD) 60.6 and 60.0 us at 512 threads, 74.6 and
        // 74.8 us at 256 (the staging is shared by twice the zones); 256 for the other nestings
        // (512 bytes kept back for the compiler's alignment of the shared arrays)
        key.block = s->block ? s->block
                             : (run_lines && slds && lds(384) + 512 <= 160 * 1024) ? 384
                             : (run_lines && !slds)                                ? 128
                             : (!run_lines && slds)                                ? 512
                                                                                   : 256;
        if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
        if (lds(key.block) + 512 > 160 * 1024)
            return fail(SJ_ERR_UNSUPPORTED, "scattering line tiles exceed 160 KiB of LDS at this block size");
        key.index64 = (s->G * lines >= (int64_t(1) << 31) || s->count * nl * s->G * s->G >= (int64_t(1) << 31) ||
                        (s->flags & SJ_FLAG_INDEX64)) ? 1 : 0;
        key.order = zdg_nm ? 2 : 1;
        // workgroup order over the XCDs: explicit flag, else the hardware's round-robin order
        const bool xcd = (s->flags & SJ_FLAG_XCD_CONTIGUOUS) != 0;
        key.flags &= ~(SJ_FLAG_XCD_CONTIGUOUS | SJ_FLAG_XCD_INTERLEAVED);
        key.flags |= xcd ? SJ_FLAG_XCD_CONTIGUOUS : SJ_FLAG_XCD_INTERLEAVED;
        return (*out = key), SJ_OK;
    }
    if (k == SJ_MLP_FWD || k == SJ_MLP_BWD || k == SJ_ADAM) {
        if (s->dtype != SJ_F32) return fail(SJ_ERR_INVALID_ARG, "the MLP kernels are FP32 (dtype SJ_F32)");
        if (s->rows < 1 || s->rows > (int64_t(1) << 24)) return fail(SJ_ERR_INVALID_ARG, "rows must be in [1, 2^24]");
        key.rows = s->rows;
        if (k != SJ_ADAM) {
            if (s->inputs < 1 || s->inputs > 64) return fail(SJ_ERR_INVALID_ARG, "inputs must be in [1, 64]");
            if (s->width < 1 || s->width > 128) return fail(SJ_ERR_INVALID_ARG, "width must be in [1, 128]");
            if (mlp_nparams(s->inputs, s->width) * 4 > 64 * 1024)
                return fail(SJ_ERR_UNSUPPORTED, "MLP parameters exceed 64 KiB of LDS");
            // the kernels index the rows * (4 width + 2) workspace and the rows * inputs
            // features with 32-bit offsets
            if (s->rows * (4 * s->width + 2) >= (int64_t(1) << 31) || s->rows * s->inputs >= (int64_t(1) << 31))
                return fail(SJ_ERR_INVALID_ARG, "rows * (4 width + 2) and rows * inputs must be below 2^31");
            key.inputs = s->inputs;
            key.width = s->width;
        }
        key.block = s->block ? s->block : (k == SJ_ADAM ? 256 : 64);
        if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
        key.order = 1;
        return (*out = key), SJ_OK;
    }
    if (k == SJ_BGEMM) {
        if (s->dtype != SJ_F64) return fail(SJ_ERR_INVALID_ARG, "BGEMM is FP64 (dtype SJ_F64)");
        uint32_t mask = s->class_mask ? s->class_mask : 0x1FFFEu;   // bits 1..16
        if (mask & ~0x1FFFEu) return fail(SJ_ERR_INVALID_ARG, "class_mask may only set bits 1..16");
        key.class_mask = mask;
        // variant: MFMA (or AUTO) = workgroup form, the waves of a workgroup share a window and the
        // grid is persistent; DIRECT = wave form, each wave owns a window copied global -> LDS directly.
        int var = s->variant ? s->variant : SJ_VAR_MFMA;
        if (var != SJ_VAR_MFMA && var != SJ_VAR_DIRECT)
            return fail(SJ_ERR_INVALID_ARG, "BGEMM variant must be SJ_VAR_MFMA (workgroup form) or SJ_VAR_DIRECT (wave form)");
        key.variant = var;
        const bool wave_form = (var == SJ_VAR_DIRECT);
        // defaults measured on MI355X at 200,000 products with n ~ U{3..16}
        key.block = s->block ? s->block : (wave_form ? 256 : 1024);
        if (!valid_block(key.block)) return fail(SJ_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
        const int u = s->unroll ? s->unroll : 1;
        if (u != 1 && u != 2 && u != 4 && u != 8)
            return fail(SJ_ERR_INVALID_ARG, "BGEMM unroll (16x16 tiles per work item) must be 1, 2, 4 or 8");
        key.unroll = u;
        const int win = s->tile_n ? s->tile_n : (wave_form ? 256 : 2048);
        if (win < 256 || win > 7168)
            return fail(SJ_ERR_INVALID_ARG, "BGEMM tile_n (window elements per array, LDS) must be in [256, 7168]");
        key.tile_n = win;
        // LDS per workgroup: A and B windows (16 bytes per element) + metadata (at most 6 bytes per
        // element); the wave form holds one window per wave.
        const int64_t mmax = win + (win + 1) / 2;
        const int64_t lds = wave_form ? (int64_t)(key.block / 64) * (2 * ((win + 31) / 32) * 32 * 8 + ((mmax + 63) / 64) * 64 * 4)
                                      : (int64_t)win * 16 + mmax * 4;
        if (lds > 160 * 1024) return fail(SJ_ERR_INVALID_ARG, "BGEMM window and block exceed 160 KiB of LDS");
        if (s->tile_k != 0) return fail(SJ_ERR_INVALID_ARG, "BGEMM takes no tile_k");
        // order (workgroup form): 1 = the next window is loaded after the current one is written
        // back; d + 1 (d = 1..3) = the loads of the next d windows are in flight in registers,
        // issued before the current window's products (prefetch depth d)
        const int order = s->order ? s->order : (wave_form ? 1 : 2);
        if (order < 1 || order > 4) return fail(SJ_ERR_INVALID_ARG, "BGEMM order must be 0 .. 4");
        if (wave_form && order != 1) return fail(SJ_ERR_INVALID_ARG, "the BGEMM wave form has no prefetch order");
        key.order = order;
        // streamed elements: nontemporal loads and stores unless asked for ordinary ones (workgroup
        // form; the wave form's direct-to-LDS loads and its stores keep the hint)
        const bool ntl = wave_form || !(s->flags & SJ_FLAG_LOADS_CACHED);
        const bool nts = wave_form || !(s->flags & SJ_FLAG_STORES_CACHED);
        key.flags &= ~(SJ_FLAG_LOADS_CACHED | SJ_FLAG_LOADS_NONTEMPORAL | SJ_FLAG_STORES_CACHED |
                       SJ_FLAG_STORES_NONTEMPORAL);
        key.flags |= (ntl ? SJ_FLAG_LOADS_NONTEMPORAL : SJ_FLAG_LOADS_CACHED) |
                     (nts ? SJ_FLAG_STORES_NONTEMPORAL : SJ_FLAG_STORES_CACHED);
        return (*out = key), SJ_OK;
    }
    return fail(SJ_ERR_UNSUPPORTED, "kernel not supported by sj_specialize");
}

// scattering with threads along nm, g not innermost and the degree matrices staged in LDS:
// two zones per thread (measured on MI355X at Z=32768 G=32 NM=16, zone regions, 512-thread
// workgroups: GZD 60.6 us against 65.0 us, ZGD 60.0 us against 71.3 us, bit-identical)
static bool scattering_pairs(const SpecKey &k)
{
    const bool nm_fastest = (k.layout == SJ_GZD || k.layout == SJ_ZGD);
    int64_t nl = 0;
    while ((nl + 1) * (nl + 1) <= k.NM - 1) ++nl;
    nl += 1;
    return nm_fastest && nl * (k.G * k.G + 2) * 8 <= 64 * 1024;
}

// scattering nestings with nm innermost (GZD, ZGD); with NM = 1 another axis is innermost too
static bool scattering_nm_inner(const SpecKey &k)
{
    return (k.layout == SJ_GZD || k.layout == SJ_ZGD) && k.NM > 1;
}

// scattering with G innermost and no staged matrices (threads along z): persistent waves that
// load their next 64 lines during the current ones (measured on MI355X at Z=32768 G=32 NM=16,
// zone regions: DZG 66.9 us against 73.7 us, ZDG 77.7 us against 89.2 us, bit-identical)
static bool scattering_persistent(const SpecKey &k)
{
    const bool sg1 = (k.layout == SJ_DZG || k.layout == SJ_ZDG);
    return sg1 && k.order != 2;
}

Geometry key_geometry(const SpecKey &k)
{
    Geometry g{0, (unsigned)k.block, 0};
    if (k.kernel == SJ_MLP_FWD || k.kernel == SJ_MLP_BWD || k.kernel == SJ_ADAM)
        g.grid = (unsigned)((k.rows + k.block - 1) / k.block);
    if (k.kernel == SJ_SCATTERING && k.variant == SJ_VAR_MFMA && scattering_nm_inner(k)) {
        g.grid = (unsigned)std::min<int64_t>((k.Z + 15) / 16, 8192);   // one 16-zone block per workgroup
        g.persistent = 1;
    } else if (k.kernel == SJ_SCATTERING && k.variant == SJ_VAR_MFMA) {
        const int64_t groups = (k.NM * ((k.Z + 15) / 16) + k.tile_n - 1) / k.tile_n, waves = k.block / 64;
        g.grid = (unsigned)std::min<int64_t>((groups + waves - 1) / waves, 8192);
        g.persistent = 1;
    } else if (k.kernel == SJ_SCATTERING) {
        g.grid = (unsigned)((k.NM * k.Z + k.block - 1) / k.block);
        if (scattering_pairs(k)) g.grid = (unsigned)((k.NM * ((k.Z + 1) / 2) + k.block - 1) / k.block);
        if (scattering_persistent(k)) {
            const int64_t groups = (k.NM * k.Z + 63) / 64, waves = k.block / 64;
            g.grid = (unsigned)std::min<int64_t>((groups + waves - 1) / waves, 8192);
            g.persistent = 1;
        }
    }
    if (k.kernel == SJ_MASS) {
        const int64_t per_block = (int64_t)(k.block / 64) * k.tile_n;
        g.grid = (unsigned)((k.rows + per_block - 1) / per_block);
        if (k.order == 2) {   // persistent: capped at load time to the workgroups the device holds at once
            g.grid = (unsigned)std::min<int64_t>(g.grid, 65536);
            g.persistent = 1;
        }
    }
    if (k.kernel == SJ_LTIMES || k.kernel == SJ_LPLUSTIMES || k.kernel == SJ_LTIMES_LPLUS) {
        if (k.variant == SJ_VAR_DIRECT) {
            const int64_t nv = k.B * (k.I / k.tile_n);
            g.grid = (unsigned)((nv + k.block - 1) / k.block);
        } else if (k.variant == SJ_VAR_STAGED) {
            g.grid = (unsigned)((k.B + k.tile_n - 1) / k.tile_n);
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.I > 1) {
            const int64_t tiles = k.B * ((k.I + 16 * k.tile_n - 1) / (16 * k.tile_n));
            const int64_t waves = k.block / 64;
            g.grid = (unsigned)std::min<int64_t>((tiles + waves - 1) / waves, 2048);
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.kernel == SJ_LTIMES_LPLUS) {
            // persistent: at most one group of tiles per wave; capped at load time to the
            // workgroups the device holds at once
            const int64_t groups = (k.B + 16 * k.tile_n - 1) / (16 * k.tile_n);
            const int64_t waves = k.block / 64;
            g.grid = (unsigned)std::min<int64_t>((groups + waves - 1) / waves, 8192);
            g.persistent = 1;
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.order == 2) {
            const int64_t groups = (k.B + 16 * k.tile_n - 1) / (16 * k.tile_n);
            const int64_t waves = k.block / 64;
            g.grid = (unsigned)std::min<int64_t>((groups + waves - 1) / waves, 8192);
            g.persistent = 1;
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64) {
            const int64_t rows_per_block = (int64_t)(k.block / 64) * 16 * k.tile_n;
            g.grid = (unsigned)((k.B + rows_per_block - 1) / rows_per_block);
        } else if (k.variant == SJ_VAR_MFMA) {
            const int64_t cols = k.tile_n == 4 ? 128 : 32;
            const int64_t tiles = k.I == 1 ? (k.B + 15) / 16 : k.B * ((k.I + cols - 1) / cols);
            const int64_t waves = k.block / 64;
            g.grid = (unsigned)std::min<int64_t>((tiles + waves - 1) / waves, 2048);
        }
    }
    return g;
}

// ---------------------------------------------------------------- emission

// contraction kernels: the workgroup renumbering for XCD-contiguous work
static const char *kXcdHelper =
    "// Workgroups are dispatched round-robin over the XCDs (each with its own L2).  With SJ_XCD > 1,\n"
    "// workgroup b works as logical block sj_block_id(): XCD x = b mod SJ_XCD takes one contiguous\n"
    "// range of logical blocks (a bijection of [0, gridDim.x) for any grid size).\n"
    "__device__ __forceinline__ unsigned sj_block_id()\n"
    "{\n"
    "#if SJ_XCD > 1\n"
    "    const unsigned b = blockIdx.x, n = gridDim.x;\n"
    "    const unsigned x = b % SJ_XCD, q = n / SJ_XCD, r = n % SJ_XCD;\n"
    "    return x * q + (x < r ? x : r) + b / SJ_XCD;\n"
    "#else\n"
    "    return blockIdx.x;\n"
    "#endif\n"
    "}\n";

static const char *kCommonPrologue =
    "// emitted by the sj specializer\n"
    "#if SJ_NT_LOAD\n"
    "#define SJ_LOAD(p) __builtin_nontemporal_load(p)\n"
    "#else\n"
    "#define SJ_LOAD(p) (*(p))\n"
    "#endif\n"
    "#if SJ_NT_STORE\n"
    "#define SJ_STORE_RAW(v, p) __builtin_nontemporal_store((v), (p))\n"
    "#else\n"
    "#define SJ_STORE_RAW(v, p) (*(p) = (v))\n"
    "#endif\n"
    "#if SJ_ACCUM\n"
    "#define SJ_STORE(v, p) SJ_STORE_RAW((v) + *(p), (p))\n"
    "#else\n"
    "#define SJ_STORE(v, p) SJ_STORE_RAW((v), (p))\n"
    "#endif\n";

void load_store_policy(const SpecKey &k, int *nt_load, int *nt_store)
{
    // streaming hint: skip cache retention when every fetched line is used at once.
    // Explicit flags, else the default measured on MI355X at Z=32768 G=32 D=96 NM=16:
    // nontemporal stores for every streamed output; nontemporal loads for LTimes' column
    // kernels (LTimes DGZ 166 us vs 177 us with ordinary loads) and its LDS-staged row kernel
    // (163 us vs 174 us); ordinary loads for LPlusTimes (DGZ 151 us vs 186 us nontemporal) and
    // for the direct row kernels, whose lanes read each 128-byte line in two halves (171 us vs
    // 199 us).
    // The BF16 row form reads and writes every 128-byte line in two 64-byte halves from two
    // instructions: with nontemporal hints the halves travel separately (measured by the HBM
    // counters at Z=262144 G=64 D=128 NM=64: 10.2 GB read and 4.7 GB written against 8.6 and
    // 4.3), so it takes ordinary loads and stores (BF16 2.49 ms against 2.78, BF16x3 2.41
    // against 2.54).
    const bool direct_rows = (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.I == 1 && k.order != 2);
    const bool bf16_rows = (k.dtype != SJ_F64 && k.I == 1);
    const bool streamed = (k.variant != SJ_VAR_DIRECT) || k.I * (k.tile_n ? k.tile_n : 1) >= 16;
    int ntl = ((k.kernel == SJ_LTIMES || k.kernel == SJ_LTIMES_LPLUS) && streamed && !direct_rows && !bf16_rows) ? 1 : 0;
    int nts = (streamed && !bf16_rows) ? 1 : 0;
    if (k.flags & SJ_FLAG_LOADS_CACHED) ntl = 0;
    if (k.flags & SJ_FLAG_LOADS_NONTEMPORAL) ntl = 1;
    if (k.flags & SJ_FLAG_STORES_CACHED) nts = 0;
    if (k.flags & SJ_FLAG_STORES_NONTEMPORAL) nts = 1;
    *nt_load = ntl;
    *nt_store = nts;
}

bool xcd_contiguous(const SpecKey &k)
{
    // explicit flags, else the default measured on MI355X at Z=32768 G=32 D=96 NM=16 with an
    // access-pattern probe of the column kernels (96 rows 8 MiB apart, two columns per thread):
    // 197 us in the hardware's round-robin order, 157 us with each XCD on a contiguous column range
    if (k.flags & SJ_FLAG_XCD_CONTIGUOUS) return true;
    if (k.flags & SJ_FLAG_XCD_INTERLEAVED) return false;
    return k.I > 1 && k.variant != SJ_VAR_STAGED;
}

// The templates name their kernel through this macro.
static const char *base_name_macro(const SpecKey &) { return "SJ_KERNEL_NAME"; }

sj_status emit_source(const SpecKey &k, std::string *src, std::string *name, std::string *name2, const double *values)
{
    if (k.values && !values) return fail(SJ_ERR_INVALID_ARG, "a value-specialized key needs its weights to emit");
    if (name2) name2->clear();
    std::ostringstream o;
    const char *body = nullptr;
    const char *bgemm_common = nullptr;   // shared class bodies of the two batched-product forms
    o << "// kernel " << k.kernel << " dtype " << k.dtype << " layout " << k.layout << " variant " << k.variant << "\n";
    o << "typedef " << (k.index64 ? "long long" : "int") << " sj_index_t;\n";
    const char *sfx = k.index64 ? "LL" : "";
    if (k.kernel == SJ_LTIMES || k.kernel == SJ_LPLUSTIMES || k.kernel == SJ_LTIMES_LPLUS) {
        o << "#define SJ_D " << k.D << "\n#define SJ_NM " << k.NM << "\n";
        o << "#define SJ_B " << k.B << sfx << "\n#define SJ_I " << k.I << sfx << "\n";
        o << "#define SJ_BLOCK " << k.block << "\n";
        int ntl = 0, nts = 0;
        load_store_policy(k, &ntl, &nts);
        o << "#define SJ_NT_LOAD " << ntl << "\n#define SJ_NT_STORE " << nts << "\n#define SJ_ACCUM "
          << ((k.flags & SJ_FLAG_ACCUMULATE) ? 1 : 0) << "\n#define SJ_XCD " << (xcd_contiguous(k) ? 8 : 0) << "\n"
          << kXcdHelper;
        if (k.variant == SJ_VAR_DIRECT) {
            o << "#define SJ_VEC " << k.tile_n << "\n#define SJ_UNROLL " << k.unroll << "\n#define SJ_FULL_UNROLL "
              << k.full_unroll << "\n#define SJ_ROTATE " << (k.order == 2 ? 1 : 0) << "\n";
            if (k.kernel == SJ_LTIMES_LPLUS) {
                body = kTpl_fused_direct;
                *name = "sj_ltimes_lplus_direct";
            } else {
                body = (k.kernel == SJ_LTIMES) ? kTpl_ltimes_direct : kTpl_lplustimes_direct;
                *name = (k.kernel == SJ_LTIMES) ? "sj_ltimes_direct" : "sj_lplustimes_direct";
                if (k.values) {
                    // the weights as exact hexadecimal literals, row-major like the run-time matrix
                    *name += "_values";
                    o << "#define SJ_WVAL 1\nstatic __device__ constexpr double sj_wv[" << k.NM * k.D << "] = {";
                    char buf[40];
                    for (int64_t i = 0; i < k.NM * k.D; ++i) {
                        std::snprintf(buf, sizeof buf, "%a", values[i]);
                        o << (i % 8 == 0 ? "\n    " : " ") << buf << ",";
                    }
                    o << "\n};\n";
                }
            }
        } else if (k.variant == SJ_VAR_STAGED) {
            o << "#define SJ_TILE_N " << k.tile_n << "\n#define SJ_TILE_K " << k.tile_k << "\n";
            body = (k.kernel == SJ_LTIMES) ? kTpl_ltimes_staged : kTpl_lplustimes_staged;
            *name = (k.kernel == SJ_LTIMES) ? "sj_ltimes_staged" : "sj_lplustimes_staged";
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.I > 1) {
            const bool lt = (k.kernel == SJ_LTIMES);
            o << "#define SJ_K " << (lt ? k.D : k.NM) << "\n#define SJ_NOUT " << (lt ? k.NM : k.D) << "\n#define SJ_T "
              << k.tile_n << "\n#define SJ_PF " << k.unroll << "\n#define SJ_ROTATE " << (k.order == 2 ? 1 : 0) << "\n";
            *name = lt ? "sj_ltimes_cols_mfma" : "sj_lplustimes_cols_mfma";
            body = kTpl_cols_mfma64;
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64 && k.kernel == SJ_LTIMES_LPLUS) {
            o << "#define SJ_ROWS " << k.B << sfx << "\n#define SJ_RT " << k.tile_n << "\n";
            *name = (k.order == 2) ? "sj_ltimes_lplus_rows_mfma_lds" : "sj_ltimes_lplus_rows_mfma";
            body = (k.order == 2) ? kTpl_fused_rows_lds_mfma64 : kTpl_fused_rows_mfma64;
        } else if (k.variant == SJ_VAR_MFMA && k.dtype == SJ_F64) {
            const bool lt = (k.kernel == SJ_LTIMES);
            o << "#define SJ_ROWS " << k.B << sfx << "\n#define SJ_K " << (lt ? k.D : k.NM) << "\n#define SJ_NOUT "
              << (lt ? k.NM : k.D) << "\n#define SJ_RT " << k.tile_n << "\n#define SJ_WREG " << k.unroll << "\n";
            if (k.order == 2) {
                *name = lt ? "sj_ltimes_rows_mfma_lds" : "sj_lplustimes_rows_mfma_lds";
                body = kTpl_rows_lds_mfma64;
            } else {
                *name = lt ? "sj_ltimes_rows_mfma" : "sj_lplustimes_rows_mfma";
                body = kTpl_rows_mfma64;
            }
        } else if (k.variant == SJ_VAR_MFMA) {
            *name = (k.dtype == SJ_BF16X3) ? "sj_ltimes_bf16x3" : "sj_ltimes_bf16";
            if (k.I == 1) *name += "_rows";
            else if (k.tile_n == 4) *name += "w";
            o << "#define SJ_X3 " << (k.dtype == SJ_BF16X3 ? 1 : 0) << "\n";
            body = (k.I == 1) ? kTpl_ltimes_bf16_rows : (k.tile_n == 4) ? kTpl_ltimes_bf16w : kTpl_ltimes_bf16;
        }
    }
    if (k.kernel == SJ_MASS) {
        o << "#define SJ_DIM " << k.inputs << "\n#define SJ_D1D " << k.D << "\n#define SJ_Q1D " << k.NM << "\n#define SJ_NE "
          << k.rows << sfx << "\n#define SJ_EW " << k.tile_n << "\n#define SJ_BLOCK " << k.block << "\n#define SJ_NT_LOAD "
          << ((k.flags & SJ_FLAG_LOADS_CACHED) ? 0 : 1) << "\n#define SJ_NT_STORE " << ((k.flags & SJ_FLAG_STORES_CACHED) ? 0 : 1)
          << "\n#define SJ_ACCUM 0\n";
        body = (k.order == 2) ? kTpl_mass_pa_pipe : kTpl_mass_pa;
        *name = std::string(k.order == 2 ? "sj_mass_pa_pipe_" : "sj_mass_pa_") + std::to_string(k.inputs) + "d_d" +
                std::to_string(k.D) + "_q" + std::to_string(k.NM);
        o << "#define SJ_KERNEL_NAME " << *name << "\n";
    }
    if (k.kernel == SJ_SCATTERING) {
        // strides of the (nm, g, z) axes in the nesting, rightmost fastest
        const int64_t NM = k.NM, G = k.G, Z = k.Z;
        int64_t snm = 0, sg = 0, sz = 0;
        switch (k.layout) {
        case SJ_DGZ: snm = G * Z; sg = Z; sz = 1; break;
        case SJ_DZG: snm = Z * G; sz = G; sg = 1; break;
        case SJ_GDZ: sg = NM * Z; snm = Z; sz = 1; break;
        case SJ_GZD: sg = Z * NM; sz = NM; snm = 1; break;
        case SJ_ZDG: sz = NM * G; snm = G; sg = 1; break;
        default: /* ZGD */ sz = G * NM; sg = NM; snm = 1; break;
        }
        int64_t nl = 0;
        while ((nl + 1) * (nl + 1) <= NM - 1) ++nl;
        nl += 1;
        const bool lane_nm = (snm < sz) && (sg != 1 || k.order == 2);   // as in the key
        static const char *lay[6] = {"dgz", "dzg", "gdz", "gzd", "zdg", "zgd"};
        if (k.variant == SJ_VAR_MFMA) {
            int ntl = 1, nts = 1;
            if (k.flags & SJ_FLAG_LOADS_CACHED) ntl = 0;
            if (k.flags & SJ_FLAG_STORES_CACHED) nts = 0;
            o << "#define SJ_NM " << NM << "\n#define SJ_G " << G << "\n#define SJ_Z " << Z << sfx << "\n#define SJ_NMAT "
              << k.rows << "\n#define SJ_NL " << nl << "\n#define SJ_SNM " << snm << sfx << "\n#define SJ_SZ " << sz << sfx
              << "\n#define SJ_SG " << sg << sfx << "\n#define SJ_RT " << k.tile_n << "\n#define SJ_ZMAJOR " << (k.order == 2 ? 1 : 0)
              << "\n#define SJ_BLOCK " << k.block << "\n#define SJ_NT_LOAD " << ntl
              << "\n#define SJ_NT_STORE " << nts << "\n#define SJ_ACCUM 0\n"
              << "#define SJ_XCD " << ((k.flags & SJ_FLAG_XCD_CONTIGUOUS) ? 8 : 0) << "\n" << kXcdHelper;
            body = (sg == 1) ? kTpl_scattering_mfma_rows : (sz == 1) ? kTpl_scattering_mfma_cols : kTpl_scattering_mfma_blocks;
            if (sg != 1 && sz != 1) o << "#define SJ_ZOUTER " << (sz > sg ? 1 : 0) << "\n";
            *name = std::string("sj_scattering_mfma_") + lay[k.layout];
            o << "#define SJ_KERNEL_NAME " << *name << "\n";
        } else {
        o << "#define SJ_PERSIST " << (scattering_persistent(k) ? 1 : 0) << "\n#define SJ_PAIR "
          << (scattering_pairs(k) ? 1 : 0) << "\n";
        int ntl = 1, nts = 1;   // phi is read once and phi_out written once: streamed
        if (k.flags & SJ_FLAG_LOADS_CACHED) ntl = 0;
        if (k.flags & SJ_FLAG_STORES_CACHED) nts = 0;
        o << "#define SJ_NM " << NM << "\n#define SJ_G " << G << "\n#define SJ_Z " << Z << sfx << "\n#define SJ_NMAT "
          << k.rows << "\n#define SJ_NL " << nl << "\n#define SJ_SNM " << snm << sfx << "\n#define SJ_SG " << sg << sfx
          << "\n#define SJ_SZ " << sz << sfx << "\n#define SJ_LANE_NM " << (lane_nm ? 1 : 0) << "\n#define SJ_RUN_LINES "
          << ((sg == 1 && std::min(snm, sz) == G) ? 1 : 0) << "\n#define SJ_SLDS "
          << ((lane_nm && nl * (G * G + 2) * 8 <= 64 * 1024) ? 1 : 0) << "\n#define SJ_BLOCK "
          << k.block << "\n#define SJ_NT_LOAD " << ntl << "\n#define SJ_NT_STORE " << nts << "\n#define SJ_ACCUM 0\n"
          << "#define SJ_XCD " << ((k.flags & SJ_FLAG_XCD_CONTIGUOUS) ? 8 : 0) << "\n" << kXcdHelper;
        body = kTpl_scattering_direct;
        *name = std::string("sj_scattering_direct_") + lay[k.layout];
        o << "#define SJ_KERNEL_NAME " << *name << "\n";
        }
    }
    if (k.kernel == SJ_MLP_FWD || k.kernel == SJ_MLP_BWD || k.kernel == SJ_ADAM) {
        o << "#define SJ_R " << k.rows << "\n#define SJ_F " << (k.inputs ? k.inputs : 1) << "\n#define SJ_H "
          << (k.width ? k.width : 1) << "\n#define SJ_BLOCK " << k.block << "\n#define SJ_NT_LOAD 0\n#define SJ_NT_STORE 0\n#define SJ_ACCUM 0\n"
          << "#define SJ_WANT_FWD " << (k.kernel == SJ_MLP_FWD) << "\n#define SJ_WANT_BWD " << (k.kernel == SJ_MLP_BWD)
          << "\n#define SJ_WANT_ADAM " << (k.kernel == SJ_ADAM) << "\n";
        body = kTpl_mlp;
        if (k.kernel == SJ_MLP_FWD) {
            *name = "sj_mlp_fwd";
        } else if (k.kernel == SJ_MLP_BWD) {
            *name = "sj_mlp_bwd_rows";
            if (name2) *name2 = "sj_mlp_bwd_params";
        } else {
            *name = "sj_adam";
        }
    }
    if (k.kernel == SJ_BGEMM) {
        const bool wave_form = (k.variant == SJ_VAR_DIRECT);
        o << "#define SJ_BLOCK " << k.block << "\n#define SJ_U " << k.unroll << "\n#define SJ_WMAX " << k.tile_n
          << "\n#define SJ_ITEM_STEP " << (wave_form ? 1 : k.block / 64) << "\n#define SJ_CLASS_CASES";
        for (int n = 1; n <= 16; ++n)
            if (k.class_mask & (1u << n))
                o << " case " << n << ": it = sj_bgemm_class<" << n << ">(Ms, Ls, it, nitems, As, Bs); break;";
        o << "\n#define SJ_PREFETCH " << (k.order >= 2 ? k.order - 1 : 0) << "\n#define SJ_NT_LOAD "
          << ((k.flags & SJ_FLAG_LOADS_NONTEMPORAL) ? 1 : 0) << "\n#define SJ_NT_STORE "
          << ((k.flags & SJ_FLAG_STORES_NONTEMPORAL) ? 1 : 0) << "\n#define SJ_ACCUM 0\n";
        bgemm_common = kTpl_bgemm_common;
        body = wave_form ? kTpl_bgemm_wave : kTpl_bgemm;
        *name = wave_form ? "sj_bgemm_waves" : "sj_bgemm_persistent";
    }
    if (!body) return fail(SJ_ERR_UNSUPPORTED, "no kernel template for this key");
    if (k.kernel == SJ_LTIMES || k.kernel == SJ_LPLUSTIMES || k.kernel == SJ_LTIMES_LPLUS) {
        // one symbol per nesting, so profiles tell the layouts apart
        static const char *lay[6] = {"dgz", "dzg", "gdz", "gzd", "zdg", "zgd"};
        *name += std::string("_") + lay[k.layout];
        o << "#define " << base_name_macro(k) << " " << *name << "\n";
    }
    o << kCommonPrologue;
    if (k.flags & SJ_FLAG_DEBUG_FAIL_COMPILE)
        o << "static_assert(SJ_BLOCK < 0, \"compile failure requested by SJ_FLAG_DEBUG_FAIL_COMPILE\");\n";
    if (bgemm_common) o << bgemm_common;
    o << body;
    *src = o.str();
    return SJ_OK;
}

// ---------------------------------------------------------------- hiprtc

static std::once_flag g_env_once;

static void disable_disk_cache()
{
    // comgr keeps an on-disk cache of compilations unless AMD_COMGR_CACHE=0;
    // the specializer must not depend on or leave files (ClangJIT section 1).
    std::call_once(g_env_once, [] { setenv("AMD_COMGR_CACHE", "0", 1); });
}

sj_status rtc_compile(const std::string &src, const char *arch, const std::string &name, std::vector<char> *code,
                      std::string *log)
{
    disable_disk_cache();
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr);
    if (r != HIPRTC_SUCCESS) return fail(SJ_ERR_COMPILE, std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r));
    const std::string archopt = std::string("--offload-arch=") + arch;
    const char *opts[] = {archopt.c_str(), "-O3", "-std=c++17", "-ffp-contract=fast",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-Rpass-analysis=kernel-resource-usage"};
    r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string lg(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &lg[0]);
    while (!lg.empty() && lg.back() == '\0') lg.pop_back();
    if (log) *log = lg;
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return fail(SJ_ERR_COMPILE, std::string("hiprtc compile failed (") + hiprtcGetErrorString(r) + "):\n" + lg);
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code->resize(cs);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return SJ_OK;
}

static int remark_value(const std::string &log, const char *label)
{
    size_t p = log.find(label);
    if (p == std::string::npos) return -1;
    p += std::strlen(label);
    while (p < log.size() && (log[p] == ' ' || log[p] == ':')) ++p;
    return std::atoi(log.c_str() + p);
}

void parse_resource_usage(const std::string &log, sj_kernel_info *info)
{
    info->vgprs = remark_value(log, "remark:     VGPRs:");
    info->agprs = remark_value(log, "remark:     AGPRs:");
    info->sgprs = remark_value(log, "remark:     TotalSGPRs:");
    info->scratch_bytes = remark_value(log, "ScratchSize [bytes/lane]:");
    info->occupancy = remark_value(log, "Occupancy [waves/SIMD]:");
    info->lds_bytes = remark_value(log, "LDS Size [bytes/block]:");
}

}  // namespace sj
