// GPU side of the counter-based input generator (see __init__.py for the
// definition): SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) evaluated at the
// logical index of every stored element, so a device buffer is filled with
// exactly the values the host generator gives for the same (seed, array id,
// logical index).  Uniform values only: the integer mix and the scaling by a
// power of two are exact on both sides.  Holds no arithmetic of the kernels
// under test.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// dist: 0 = U[0,1) with 53 bits, 1 = U[-1,1) (2u-1), 2 = U[0,1) with 24 bits
__device__ inline double value(uint64_t key, uint64_t i, int dist)
{
    const uint64_t b = mix64(key + (i + 1) * kGamma);
    if (dist == 2) return (double)(b >> 40) * 0x1p-24;
    const double u = (double)(b >> 11) * 0x1p-53;
    return dist == 1 ? 2.0 * u - 1.0 : u;
}

// Storage position p of an (A, G, Z) array in `layout` order -> logical
// D-G-Z index (a*G + g)*Z + z.  layout < 0: the array is plain (index = p).
__device__ inline uint64_t logical_index(int64_t p, int layout, int64_t A, int64_t G, int64_t Z)
{
    if (layout < 0) return (uint64_t)p;
    int64_t n0, n1, n2;  // storage extents, slowest first
    switch (layout) {
    case 0: n0 = A; n1 = G; n2 = Z; break;   // DGZ
    case 1: n0 = A; n1 = Z; n2 = G; break;   // DZG
    case 2: n0 = G; n1 = A; n2 = Z; break;   // GDZ
    case 3: n0 = G; n1 = Z; n2 = A; break;   // GZD
    case 4: n0 = Z; n1 = A; n2 = G; break;   // ZDG
    default: n0 = Z; n1 = G; n2 = A; break;  // ZGD
    }
    (void)n0;
    const int64_t x2 = p % n2, q = p / n2, x1 = q % n1, x0 = q / n1;
    int64_t a, g, z;
    switch (layout) {
    case 0: a = x0; g = x1; z = x2; break;
    case 1: a = x0; z = x1; g = x2; break;
    case 2: g = x0; a = x1; z = x2; break;
    case 3: g = x0; z = x1; a = x2; break;
    case 4: z = x0; a = x1; g = x2; break;
    default: z = x0; g = x1; a = x2; break;
    }
    return (uint64_t)((a * G + g) * Z + z);
}

template <typename T>
__global__ void __launch_bounds__(256) fill_kernel(T *out, int64_t n, uint64_t key, int dist, int layout, int64_t A,
                                                   int64_t G, int64_t Z)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
        out[p] = (T)value(key, logical_index(p, layout, A, G, Z), dist);
}

}  // namespace

extern "C" {

// Fill `n` elements of `out` (dtype 0: double, 1: float).  For layout >= 0 the
// array is an (A, G, Z) array stored in that order and n must equal A*G*Z.
// Returns 0 on success, 1 for bad arguments, 2 for a launch error.
int sjgen_fill(void *out, int dtype, int dist, uint64_t seed, int arr, int layout, int64_t n, int64_t A, int64_t G,
               int64_t Z, void *stream)
{
    if (!out || n < 0 || dist < 0 || dist > 2 || dtype < 0 || dtype > 1 || layout > 5) return 1;
    if (layout >= 0 && (A < 1 || G < 1 || Z < 1 || A * G * Z != n)) return 1;
    if (n == 0) return 0;
    const uint64_t key = mix64(seed + (uint64_t)arr * kGamma);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dtype == 0)
        hipLaunchKernelGGL(fill_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                           (double *)out, n, key, dist, layout, A, G, Z);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                           (float *)out, n, key, dist, layout, A, G, Z);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
