// Ahead-of-time generic kernels: the same operations with every size and
// stride a kernel argument.  They are the baseline that runtime specialization
// is measured against (the paper's "AoT generic" variants, section 5) and the
// fallback when a specialization cannot be compiled (section 6 notes that the
// attribute-based design has no fallback path).
//
// What a generic kernel cannot do: keep a runtime-sized set of accumulators in
// registers.  So the moments are processed in register chunks of 16 with the
// reduction loop re-run per chunk (LTimes re-reads psi once per chunk of 16
// moments; LPlusTimes adds each chunk's contribution into psi'), loop bounds
// are runtime values, and addresses come from runtime strides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "sj_internal.h"

namespace {

constexpr int kChunk = 16;
constexpr int kBlock = 256;

struct Strides {
    long long Z, G, D, NM;
    long long ad, ag, az;   // input offsets per unit of (reduction index, g, z)
    long long bd, bg, bz;   // output offsets per unit of (output index, g, z)
    int z_fast;             // 1: consecutive threads take consecutive z
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); like the
// specialized column kernels, the generic ones renumber them so that XCD x = b mod 8 takes one
// contiguous range of columns (a bijection of the grid), so the comparison between the two does
// not measure this launch order.
__device__ __forceinline__ long long xcd_block()
{
    const unsigned b = blockIdx.x, n = gridDim.x;
    const unsigned x = b % 8u, q = n / 8u, r = n % 8u;
    return (long long)(x * q + (x < r ? x : r) + b / 8u);
}

__device__ __forceinline__ void ltimes_body(const double *__restrict__ L, const double *__restrict__ psi,
                                            double *__restrict__ phi, const Strides &s)
{
    const long long t = xcd_block() * kBlock + threadIdx.x;
    if (t >= s.G * s.Z) return;
    long long g, z;
    if (s.z_fast) { g = t / s.Z; z = t - g * s.Z; }
    else { z = t / s.G; g = t - z * s.G; }
    const double *p = psi + g * s.ag + z * s.az;
    double *q = phi + g * s.bg + z * s.bz;
    for (long long nm0 = 0; nm0 < s.NM; nm0 += kChunk) {
        double acc[kChunk];
        const double *Lr[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            acc[j] = 0.0;
            Lr[j] = L + std::min(nm0 + j, s.NM - 1) * s.D;   // rows past NM repeat the last one; never stored
        }
        for (long long d = 0; d < s.D; ++d) {
            const double x = p[d * s.ad];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) acc[j] = __builtin_fma(Lr[j][d], x, acc[j]);
        }
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            if (nm0 + j < s.NM) q[(nm0 + j) * s.bd] = acc[j];
    }
}

__device__ __forceinline__ void lplustimes_body(const double *__restrict__ Lp, const double *__restrict__ phi,
                                                double *__restrict__ out, const Strides &s)
{
    const long long t = xcd_block() * kBlock + threadIdx.x;
    if (t >= s.G * s.Z) return;
    long long g, z;
    if (s.z_fast) { g = t / s.Z; z = t - g * s.Z; }
    else { z = t / s.G; g = t - z * s.G; }
    const double *p = phi + g * s.ag + z * s.az;
    double *q = out + g * s.bg + z * s.bz;
    for (long long nm0 = 0; nm0 < s.NM; nm0 += kChunk) {
        double x[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) x[j] = (nm0 + j < s.NM) ? p[(nm0 + j) * s.ad] : 0.0;
        const long long jmax = std::min<long long>(kChunk, s.NM - nm0);
        for (long long d = 0; d < s.D; ++d) {
            const double *l = Lp + d * s.NM + nm0;
            double o = 0.0;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) o = __builtin_fma(j < jmax ? l[j] : 0.0, x[j], o);
            if (nm0 == 0) q[d * s.bd] = o;
            else q[d * s.bd] += o;
        }
    }
}

// Reduction axis innermost (GZD, ZGD): every column is a contiguous row of
// `red` input values and a contiguous row of `outn` outputs, so N columns are
// one [N][red] and one [N][outn] row-major matrix, W is [outn][red] row-major
// (L for LTimes, L+ for LPlusTimes).  A workgroup takes `tr` consecutive rows
// (tr chosen on the host so that the tiles fit in dynamic LDS): it reads them
// as one contiguous run (consecutive threads, consecutive addresses) into LDS
// with a row pitch of red + 1, W into LDS beside them when it fits (else W is
// read through the caches), each thread then forms outputs of one row in
// register chunks of 16 (outputs j, j + kBlock/tr, ...), and the [tr][outn]
// results leave through LDS as one contiguous run.  Only the loop bounds and
// addresses are run-time values; the access pattern is the coalesced one a
// specialization uses, so the comparison measures what compile-time sizes buy.
template <bool WLDS>
__global__ void __launch_bounds__(kBlock)
generic_rows(const double *__restrict__ W, const double *__restrict__ in, double *__restrict__ out, long long N,
             long long red, long long outn, int tr)
{
    extern __shared__ double lds[];
    double *xin = lds;                                   // [tr][red + 1]
    double *yout = lds + (long long)tr * (red + 1);      // [tr][outn + 1]
    double *wl = yout + (long long)tr * (outn + 1);      // [outn][red] when WLDS
    const long long r0 = (long long)blockIdx.x * tr;
    const int rows = (int)(N - r0 < tr ? N - r0 : tr);
    // tile-local indices fit in 32 bits (the tiles are within 64 KiB); element e = row r, column c is
    // advanced by kBlock without a division per element
    const int ired = (int)red, iout = (int)outn;
    const int nin = rows * ired, nout = rows * iout;
    const double *src = in + r0 * red;
    {
        // eight loads in flight per thread before their LDS writes
        constexpr int U = 8;
        int r = (int)threadIdx.x / ired, c = (int)threadIdx.x % ired;
        const int dr = kBlock / ired, dc = kBlock % ired;
        for (int e0 = threadIdx.x; e0 < nin; e0 += U * kBlock) {
            double v[U];
            int at[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * kBlock;
                at[u] = r * (ired + 1) + c;
                v[u] = e < nin ? src[e] : 0.0;
                r += dr;
                c += dc;
                if (c >= ired) { c -= ired; ++r; }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + u * kBlock < nin) xin[at[u]] = v[u];
        }
    }
    if (WLDS)
        for (int e = threadIdx.x; e < iout * ired; e += kBlock) wl[e] = W[e];
    __syncthreads();
    const double *Wr = WLDS ? wl : W;
    const int per = kBlock / tr;                         // threads per row
    const int r = threadIdx.x % tr, j0 = threadIdx.x / tr;
    if (r < rows && j0 < per) {
        const double *x = xin + r * (ired + 1);
        for (int o0 = j0; o0 < iout; o0 += per * kChunk) {
            double acc[kChunk];
            const double *wr[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                acc[c] = 0.0;
                const int o = o0 + c * per;
                wr[c] = Wr + (long long)(o < iout ? o : iout - 1) * red;   // past outn: repeat the last row, never stored
            }
            for (int k = 0; k < ired; ++k) {
                const double xv = x[k];
#pragma unroll
                for (int c = 0; c < kChunk; ++c) acc[c] = __builtin_fma(wr[c][k], xv, acc[c]);
            }
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const int o = o0 + c * per;
                if (o < iout) yout[r * (iout + 1) + o] = acc[c];
            }
        }
    }
    __syncthreads();
    double *dst = out + r0 * outn;
    {
        int rr = (int)threadIdx.x / iout, c = (int)threadIdx.x % iout;
        const int dr = kBlock / iout, dc = kBlock % iout;
        for (int e = threadIdx.x; e < nout; e += kBlock) {
            dst[e] = yout[rr * (iout + 1) + c];
            rr += dr;
            c += dc;
            if (c >= iout) { c -= iout; ++rr; }
        }
    }
}

// The same row contraction on the FP64 matrix cores with run-time sizes:
// v_mfma_f64_16x16x4f64 (A lane l holds A[l%16][l/16], B lane l holds
// B[l/16][l%16], C register i of lane l holds C[4i + l/16][l%16]).  A wave
// takes 16-row tiles grid-stride: the tile's rows arrive as one contiguous run
// into a per-wave LDS tile (row pitch red + 1), and for every 16-output block a
// run-time loop over 4-deep reduction steps feeds the MFMAs with A = the rows
// and B = W (staged in LDS once per workgroup), two accumulators in turn; each
// block's outputs are stored from the C registers (sixteen lanes write sixteen
// consecutive outputs of a row).
constexpr int kRowWaves = 4;

__global__ void __launch_bounds__(kRowWaves * 64)
generic_rows_mfma(const double *__restrict__ W, const double *__restrict__ in, double *__restrict__ out, long long N,
                  int red, int outn)
{
    typedef double d4 __attribute__((ext_vector_type(4)));
    extern __shared__ double lds[];
    const int pitch = red + 1;
    double *wl = lds;                                                  // [outn][red]
    double *tile = lds + (long long)outn * red + (threadIdx.x >> 6) * (16 * pitch);
    const int lane = threadIdx.x & 63, m = lane & 15, q = lane >> 4;
    for (int e = threadIdx.x; e < outn * red; e += kRowWaves * 64) wl[e] = W[e];
    __syncthreads();
    const long long tiles = (N + 15) / 16;
    for (long long t = (long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6); t < tiles;
         t += (long long)gridDim.x * kRowWaves) {
        const long long r0 = t * 16;
        const int rows = (int)(N - r0 < 16 ? N - r0 : 16);
        const int nin = rows * red;
        const double *src = in + r0 * red;
        {   // eight loads in flight per lane before their LDS writes
            constexpr int U = 8;
            int r = lane / red, c = lane % red;
            const int dr = 64 / red, dc = 64 % red;
            for (int e0 = lane; e0 < nin; e0 += U * 64) {
                double v[U];
                int at[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * 64;
                    at[u] = r * pitch + c;
                    v[u] = e < nin ? src[e] : 0.0;
                    r += dr;
                    c += dc;
                    if (c >= red) { c -= red; ++r; }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (e0 + u * 64 < nin) tile[at[u]] = v[u];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // rows past the tile's end read row 0 (their results are not stored)
        const double *arow = tile + (m < rows ? m : 0) * pitch;
        const int nob = (outn + 15) / 16, nkb = (red + 3) / 4;
        double *dst = out + r0 * outn;
        for (int ob = 0; ob < nob; ++ob) {
            const int o = ob * 16 + m;
            const double *wrow = wl + (long long)(o < outn ? o : 0) * red;
            d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            int kb = 0;
            for (; kb + 1 < nkb; kb += 2) {
                const int k0 = 4 * kb + q, k1 = k0 + 4;
                const double a0 = k0 < red ? arow[k0] : 0.0, a1 = k1 < red ? arow[k1] : 0.0;
                const double b0 = (o < outn && k0 < red) ? wrow[k0] : 0.0;
                const double b1 = (o < outn && k1 < red) ? wrow[k1] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
            }
            if (kb < nkb) {
                const int k0 = 4 * kb + q;
                const double a0 = k0 < red ? arow[k0] : 0.0;
                const double b0 = (o < outn && k0 < red) ? wrow[k0] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
            }
            // C register i of lane l: row 4i + l/16, output o; sixteen lanes write 16 consecutive
            // outputs of one row
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * i + q < rows && o < outn) dst[(long long)(4 * i + q) * outn + o] = acc0[i] + acc1[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");   // A reads done before the next tile's run
    }
}

// Rows per workgroup of generic_rows: the row tiles (and W, when it is staged)
// within 64 KiB of LDS.
inline int generic_rows_tile(long long red, long long outn, bool wlds)
{
    const long long room = 8192 - (wlds ? outn * red : 0);
    const long long t = room / (red + outn + 2);
    return (int)std::max<long long>(1, std::min<long long>(kBlock, t));
}

__global__ void __launch_bounds__(kBlock)
generic_ltimes(const double *__restrict__ L, const double *__restrict__ psi, double *__restrict__ phi, Strides s)
{
    ltimes_body(L, psi, phi, s);
}

__global__ void __launch_bounds__(kBlock)
generic_lplustimes(const double *__restrict__ Lp, const double *__restrict__ phi, double *__restrict__ out, Strides s)
{
    lplustimes_body(Lp, phi, out, s);
}

// Offsets of logical (a, g, z) for an (A, G, Z) array stored in nesting LAYOUT,
// the nesting known at compile time and the sizes at run time.
template <int LAYOUT>
__device__ __forceinline__ void layout_strides_ct(long long A, long long G, long long Z, long long &sa, long long &sg,
                                                  long long &sz)
{
    if constexpr (LAYOUT == SJ_DGZ) { sa = G * Z; sg = Z; sz = 1; }
    else if constexpr (LAYOUT == SJ_DZG) { sa = Z * G; sz = G; sg = 1; }
    else if constexpr (LAYOUT == SJ_GDZ) { sg = A * Z; sa = Z; sz = 1; }
    else if constexpr (LAYOUT == SJ_GZD) { sg = Z * A; sz = A; sa = 1; }
    else if constexpr (LAYOUT == SJ_ZDG) { sz = A * G; sa = G; sg = 1; }
    else { sz = G * A; sg = A; sa = 1; }
}

// Ahead-of-time kernels per nesting with run-time sizes: Kripke's own
// multiversioning (ClangJIT section 5.2, layout-dispatch listing), the middle
// baseline between the generic kernels (nesting and sizes at run time) and the
// specializations (both at compile time).  The same loops as the generic
// kernels; only the stride pattern and the thread order are constants.
template <int LAYOUT, bool LT>
__global__ void __launch_bounds__(kBlock)
aot_layout_kernel(const double *__restrict__ W, const double *__restrict__ in, double *__restrict__ out, long long Z,
                  long long G, long long D, long long NM)
{
    Strides s;
    s.Z = Z; s.G = G; s.D = D; s.NM = NM;
    layout_strides_ct<LAYOUT>(LT ? D : NM, G, Z, s.ad, s.ag, s.az);
    layout_strides_ct<LAYOUT>(LT ? NM : D, G, Z, s.bd, s.bg, s.bz);
    s.z_fast = (LAYOUT == SJ_DGZ || LAYOUT == SJ_GDZ || LAYOUT == SJ_GZD) ? 1 : 0;
    if constexpr (LT) ltimes_body(W, in, out, s);
    else lplustimes_body(W, in, out, s);
}

template <bool LT>
hipError_t launch_aot(int layout, unsigned nblk, hipStream_t st, const double *W, const double *in, double *out,
                      long long Z, long long G, long long D, long long NM)
{
    switch (layout) {
    case SJ_DGZ: hipLaunchKernelGGL((aot_layout_kernel<SJ_DGZ, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    case SJ_DZG: hipLaunchKernelGGL((aot_layout_kernel<SJ_DZG, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    case SJ_GDZ: hipLaunchKernelGGL((aot_layout_kernel<SJ_GDZ, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    case SJ_GZD: hipLaunchKernelGGL((aot_layout_kernel<SJ_GZD, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    case SJ_ZDG: hipLaunchKernelGGL((aot_layout_kernel<SJ_ZDG, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    default: hipLaunchKernelGGL((aot_layout_kernel<SJ_ZGD, LT>), dim3(nblk), dim3(kBlock), 0, st, W, in, out, Z, G, D, NM); break;
    }
    return hipGetLastError();
}

// One workgroup (one wave) per instance, runtime n; A and B staged in LDS.
__global__ void __launch_bounds__(64)
generic_bgemm(const int *__restrict__ n, const long long *__restrict__ off, const double *__restrict__ A,
              const double *__restrict__ B, double *__restrict__ C, long long count)
{
    __shared__ double a[256], b[256];
    for (long long i = blockIdx.x; i < count; i += gridDim.x) {
        const int s = n[i];
        const long long o = off[i];
        const int ss = s * s;
        for (int e = threadIdx.x; e < ss; e += 64) {
            a[e] = A[o + e];
            b[e] = B[o + e];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ss; e += 64) {
            const int r = e / s, c = e - (e / s) * s;
            double acc = 0.0;
            for (int k = 0; k < s; ++k) acc = __builtin_fma(a[r * s + k], b[k * s + c], acc);
            C[o + e] = acc;
        }
        __syncthreads();
    }
}

// Reads `bytes` of the buffer at p (16-byte pieces, grid-stride) so that earlier
// contents of L2 and the last-level cache are evicted by clean lines; the only
// store is conditional on a value the XOR of real data practically never
// reaches, which keeps the loads.
typedef unsigned int sj_u4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) flush_read(sj_u4 *p, size_t n16, size_t tail, const unsigned char *tail_p)
{
    sj_u4 acc = {0u, 0u, 0u, 0u};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
        acc ^= p[i];   // ordinary loads: they take the last-level cache's lines (nontemporal ones did not evict it)
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (size_t i = 0; i < tail; ++i) acc.x ^= tail_p[i];
    if (n16 > 0 && acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xf39cc060u && acc.w == 0x5cedc834u)
        p[0] = acc;
}

// Offsets of logical (a, g, z) for an (A, G, Z) array stored in `layout` order.
void layout_strides(int layout, long long A, long long G, long long Z, long long *sa, long long *sg, long long *sz)
{
    switch (layout) {
    case SJ_DGZ: *sa = G * Z; *sg = Z; *sz = 1; break;
    case SJ_DZG: *sa = Z * G; *sz = G; *sg = 1; break;
    case SJ_GDZ: *sg = A * Z; *sa = Z; *sz = 1; break;
    case SJ_GZD: *sg = Z * A; *sz = A; *sa = 1; break;
    case SJ_ZDG: *sz = A * G; *sa = G; *sg = 1; break;
    default: /* ZGD */ *sz = G * A; *sg = A; *sa = 1; break;
    }
}

}  // namespace

namespace sj {

hipError_t launch_flush_read(void *buf, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16;
    const unsigned grid = (unsigned)std::max<size_t>(1, std::min<size_t>((n16 + 255) / 256, 8192));
    hipLaunchKernelGGL(flush_read, dim3(grid), dim3(256), 0, st, (sj_u4 *)buf, n16, bytes % 16,
                       (const unsigned char *)buf + n16 * 16);
    return hipGetLastError();
}

}  // namespace sj

extern "C" sj_status sj_generic_run(sj_kernel k, const sj_spec *spec, void *const *ptrs, int nptrs, void *stream)
{
    using namespace sj;
    clear_error();
    if (!spec) return fail(SJ_ERR_INVALID_ARG, "null spec");
    if (spec->struct_size != sizeof(sj_spec)) return fail(SJ_ERR_INVALID_ARG, "sj_spec.struct_size mismatch");
    hipStream_t st = (hipStream_t)stream;
    if (k == SJ_LTIMES || k == SJ_LPLUSTIMES) {
        if (spec->dtype != SJ_F64) return fail(SJ_ERR_UNSUPPORTED, "generic kernels are FP64 only");
        if (spec->flags & SJ_FLAG_ACCUMULATE) return fail(SJ_ERR_UNSUPPORTED, "generic kernels overwrite their output");
        if (spec->layout < SJ_DGZ || spec->layout > SJ_ZGD) return fail(SJ_ERR_INVALID_ARG, "layout out of range");
        const long long Z = spec->Z, G = spec->G, D = spec->D, NM = spec->NM;
        if (Z < 1 || G < 1 || D < 1 || NM < 1 || Z > 2147483647LL || G > 2147483647LL || D > 2147483647LL ||
            NM > 2147483647LL)
            return fail(SJ_ERR_INVALID_ARG, "sizes must be in [1, 2^31-1]");
        const size_t cols = (size_t)G * (size_t)Z;
        size_t bytes[3];
        bytes[0] = (size_t)NM * (size_t)D * 8;
        bytes[1] = (k == SJ_LTIMES ? (size_t)D : (size_t)NM) * cols * 8;
        bytes[2] = (k == SJ_LTIMES ? (size_t)NM : (size_t)D) * cols * 8;
        sj_status s = check_ptrs(ptrs, nptrs, 3, bytes, 2);
        if (s != SJ_OK) return s;
        Strides st_{};
        st_.Z = Z; st_.G = G; st_.D = D; st_.NM = NM;
        const long long A_in = (k == SJ_LTIMES) ? D : NM, A_out = (k == SJ_LTIMES) ? NM : D;
        layout_strides(spec->layout, A_in, G, Z, &st_.ad, &st_.ag, &st_.az);
        layout_strides(spec->layout, A_out, G, Z, &st_.bd, &st_.bg, &st_.bz);
        st_.z_fast = (st_.az <= st_.ag) ? 1 : 0;
        const long long nblk = ((long long)cols + kBlock - 1) / kBlock;
        if (nblk > 2147483647LL) return fail(SJ_ERR_UNSUPPORTED, "too many columns for one launch");
        const double *L = (const double *)ptrs[0];
        const double *in = (const double *)ptrs[1];
        double *outp = (double *)ptrs[2];
        if (st_.ad == 1 && st_.bd == 1 && A_in * A_out + 64 * (A_in + 1) <= 8192) {
            // the reduction axis is innermost in both arrays, W and four 16-row tiles fit in 64 KiB
            // of LDS: the matrix-core row kernel with run-time sizes
            const long long tiles = ((long long)cols + 15) / 16;
            const unsigned grid = (unsigned)std::min<long long>((tiles + kRowWaves - 1) / kRowWaves, 8192);
            const size_t shm = ((size_t)(A_in * A_out) + 64 * (size_t)(A_in + 1)) * 8;
            hipLaunchKernelGGL(generic_rows_mfma, dim3(grid), dim3(kRowWaves * 64), shm, st, L, in, outp,
                               (long long)cols, (int)A_in, (int)A_out);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("generic launch: ") + hipGetErrorString(e));
            return SJ_OK;
        }
        if (st_.ad == 1 && st_.bd == 1 && A_in + A_out + 2 <= 8192) {
            // the reduction axis is innermost in both arrays: rows staged through LDS (serves the
            // generic call and the per-nesting one alike: the access pattern is the nesting's); W
            // is staged too when that still leaves room for 32 rows
            const bool wlds = A_in * A_out + 32 * (A_in + A_out + 2) <= 8192;
            const int tr = generic_rows_tile(A_in, A_out, wlds);
            const long long nrow = ((long long)cols + tr - 1) / tr;
            if (nrow > 2147483647LL) return fail(SJ_ERR_UNSUPPORTED, "too many columns for one launch");
            const size_t shm = ((size_t)tr * (size_t)(A_in + A_out + 2) + (wlds ? (size_t)(A_in * A_out) : 0)) * 8;
            if (wlds)
                hipLaunchKernelGGL(generic_rows<true>, dim3((unsigned)nrow), dim3(kBlock), shm, st, L, in, outp,
                                   (long long)cols, A_in, A_out, tr);
            else
                hipLaunchKernelGGL(generic_rows<false>, dim3((unsigned)nrow), dim3(kBlock), shm, st, L, in, outp,
                                   (long long)cols, A_in, A_out, tr);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("generic launch: ") + hipGetErrorString(e));
            return SJ_OK;
        }
        if (spec->flags & SJ_FLAG_GENERIC_PER_LAYOUT) {
            hipError_t e = (k == SJ_LTIMES) ? launch_aot<true>(spec->layout, (unsigned)nblk, st, L, in, outp, Z, G, D, NM)
                                            : launch_aot<false>(spec->layout, (unsigned)nblk, st, L, in, outp, Z, G, D, NM);
            if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("generic launch: ") + hipGetErrorString(e));
            return SJ_OK;
        }
        if (k == SJ_LTIMES)
            hipLaunchKernelGGL(generic_ltimes, dim3((unsigned)nblk), dim3(kBlock), 0, st, L, in, outp, st_);
        else
            hipLaunchKernelGGL(generic_lplustimes, dim3((unsigned)nblk), dim3(kBlock), 0, st, L, in, outp, st_);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("generic launch: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    if (k == SJ_BGEMM) {
        if (!ptrs || nptrs != 5) return fail(SJ_ERR_INVALID_ARG, "BGEMM takes {n, off, A, B, C}");
        for (int i = 0; i < 5; ++i) {
            if (!ptrs[i]) return fail(SJ_ERR_INVALID_ARG, "null buffer pointer");
            if (((uintptr_t)ptrs[i]) & 7u) return fail(SJ_ERR_ALIGN, "buffer pointer not 8-byte aligned");
        }
        const long long count = spec->count;
        if (count < 0) return fail(SJ_ERR_INVALID_ARG, "count must be >= 0");
        if (count == 0) return SJ_OK;
        const unsigned grid = (unsigned)std::min<long long>(count, 1 << 20);
        hipLaunchKernelGGL(generic_bgemm, dim3(grid), dim3(64), 0, st, (const int *)ptrs[0],
                           (const long long *)ptrs[1], (const double *)ptrs[2], (const double *)ptrs[3],
                           (double *)ptrs[4], count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(SJ_ERR_LAUNCH, std::string("generic launch: ") + hipGetErrorString(e));
        return SJ_OK;
    }
    return fail(SJ_ERR_UNSUPPORTED, "no generic kernel for this kernel id");
}
