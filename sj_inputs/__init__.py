"""Seeded, counter-based synthetic input generator.

This module is the one piece of code that both the CPU oracle side and the GPU
side use: it produces input values only and holds none of the arithmetic of the
moment contractions, the batched products or the cost model.

Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  A SplitMix64 stream seeded with
``s`` returns, as its k-th output (k = 1, 2, ...), ``mix64(s + k * GAMMA)``.
That closed form makes the generator counter-based: element ``i`` of array
``arr`` under seed ``seed`` is

    key   = mix64(seed + arr * GAMMA)          # the arr-th output of SplitMix64(seed)
    bits  = mix64(key + (i + 1) * GAMMA)       # the (i+1)-th output of SplitMix64(key)

with all arithmetic modulo 2^64.  Derived values:

* ``u01``   : (bits >> 11) * 2^-53, uniform on [0, 1) with 53 random bits;
* ``u01_24``: (bits >> 40) * 2^-24, uniform on [0, 1) with 24 random bits
  (exactly representable in float32, used where the GPU input is float32);
* ``sym``   : 2*u - 1, uniform on [-1, 1) (exact in binary64);
* ``normal``: Box-Muller on (1 - u01(2i), u01(2i+1)) -> sqrt(-2 ln u1) cos(2 pi u2)
  (host only: libm results of log/cos are not bit-reproducible on the GPU);
* ``n in {lo..hi}``: lo + floor(u01 * (hi - lo + 1)).

The index ``i`` is always a *logical* index, so that the same logical element has
the same value whatever storage layout it is written in.  For psi-like arrays
the logical order is D-G-Z (d slowest, z fastest): ``i = (d*G + g)*Z + z``.

Array ids used by the tests and the benchmark: psi = 1, L = 2, L+ = 3, A = 4,
B = 5, n = 6, phi = 7, MLP data = 8...
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

ARR_PSI = 1
ARR_L = 2
ARR_LPLUS = 3
ARR_A = 4
ARR_B = 5
ARR_N = 6
ARR_PHI = 7
ARR_MLP = 8

# Storage layouts of a psi-like array with axes (A, G, Z), A standing for D
# (psi) or NM (phi).  The letters give the storage order, rightmost fastest.
LAYOUTS = ("DGZ", "DZG", "GDZ", "GZD", "ZDG", "ZGD")


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea & Flood 2014), on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, arr: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + np.uint64(arr) * GAMMA
    return mix64(np.array([s], dtype=np.uint64))[0]


def bits(seed: int, arr: int, idx) -> np.ndarray:
    """Raw 64-bit outputs for logical indices ``idx`` (any integer array)."""
    key = stream_key(seed, arr)
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + (i + np.uint64(1)) * GAMMA
    return mix64(z)


def u01(seed: int, arr: int, idx) -> np.ndarray:
    return (bits(seed, arr, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def u01_24(seed: int, arr: int, idx) -> np.ndarray:
    return (bits(seed, arr, idx) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def sym(seed: int, arr: int, idx) -> np.ndarray:
    return 2.0 * u01(seed, arr, idx) - 1.0


def normal(seed: int, arr: int, idx) -> np.ndarray:
    i = np.asarray(idx, dtype=np.uint64)
    u1 = 1.0 - u01(seed, arr, 2 * i)
    u2 = u01(seed, arr, 2 * i + 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def int_range(seed: int, arr: int, idx, lo: int, hi: int) -> np.ndarray:
    u = u01(seed, arr, idx)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


# ---------------------------------------------------------------------------
# Layout helpers (pure index bookkeeping, no arithmetic of the method).

def layout_shape(layout: str, A: int, G: int, Z: int) -> tuple:
    dims = {"D": A, "G": G, "Z": Z}
    return tuple(dims[c] for c in layout)


def to_layout(logical: np.ndarray, layout: str) -> np.ndarray:
    """Logical (A, G, Z) array -> contiguous array stored in ``layout`` order."""
    perm = tuple("DGZ".index(c) for c in layout)
    return np.ascontiguousarray(np.transpose(logical, perm))


def from_layout(stored: np.ndarray, layout: str, A: int, G: int, Z: int) -> np.ndarray:
    """Flat or shaped array stored in ``layout`` order -> logical (A, G, Z) array."""
    x = np.asarray(stored).reshape(layout_shape(layout, A, G, Z))
    perm = tuple(layout.index(c) for c in "DGZ")
    return np.ascontiguousarray(np.transpose(x, perm))


def psi_logical(seed: int, D: int, G: int, Z: int, arr: int = ARR_PSI, bits24: bool = False) -> np.ndarray:
    """psi[d, g, z] ~ U[0, 1) as a logical (D, G, Z) float64 array."""
    n = D * G * Z
    gen = u01_24 if bits24 else u01
    return gen(seed, arr, np.arange(n, dtype=np.uint64)).reshape(D, G, Z)


def psi_columns(seed: int, D: int, G: int, Z: int, g, z, arr: int = ARR_PSI, bits24: bool = False) -> np.ndarray:
    """psi[:, g_j, z_j] for sampled columns j, shape (D, len(g)); logical indexing
    of the full (D, G, Z) problem, so samples agree with the full array."""
    g = np.asarray(g, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    d = np.arange(D, dtype=np.uint64)[:, None]
    idx = (d * np.uint64(G) + g[None, :]) * np.uint64(Z) + z[None, :]
    gen = u01_24 if bits24 else u01
    return gen(seed, arr, idx)


def matrix_sym(seed: int, arr: int, rows: int, cols: int) -> np.ndarray:
    """Row-major rows x cols matrix ~ U[-1, 1)."""
    return sym(seed, arr, np.arange(rows * cols, dtype=np.uint64)).reshape(rows, cols)


def batch_sizes(seed: int, count: int, lo: int = 3, hi: int = 16) -> np.ndarray:
    return int_range(seed, ARR_N, np.arange(count, dtype=np.uint64), lo, hi).astype(np.int32)


def batch_offsets(n: np.ndarray) -> np.ndarray:
    """off_i = sum_{j<i} n_j^2 (int64), plus the total as the last entry."""
    sq = np.asarray(n, dtype=np.int64) ** 2
    off = np.zeros(len(sq) + 1, dtype=np.int64)
    np.cumsum(sq, out=off[1:])
    return off


def batch_normal(seed: int, arr: int, total: int) -> np.ndarray:
    return normal(seed, arr, np.arange(total, dtype=np.uint64))
