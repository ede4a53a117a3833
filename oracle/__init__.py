"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product library never does.

``build()`` compiles ``oracle.c`` with gcc (-O2 -ffp-contract=off -fopenmp)
into ``liboracle.so`` next to this file.  The wrappers below take numpy arrays
and call the C functions unchanged; they hold no arithmetic of their own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LAYOUTS = ("DGZ", "DZG", "GDZ", "GZD", "ZDG", "ZGD")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle.  Always recompiles when ``force``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = i32
        for name in ("orc_ltimes", "orc_lplustimes", "orc_ltimes_absscale"):
            f = getattr(L, name)
            f.argtypes = [i32, i64, i64, i64, i64, vp, vp, vp]
            f.restype = i32
        L.orc_bgemm.argtypes = [i64, vp, vp, vp, vp, vp]
        for f in (L.orc_mass, L.orc_mass_absscale):
            f.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp]
        for f in (L.orc_scattering, L.orc_scattering_absscale):
            f.argtypes = [i32, i64, i64, i64, i64, vp, vp, vp, vp]
        L.orc_bgemm.restype = i32
        L.orc_bf16_round.argtypes = [d]
        L.orc_bf16_round.restype = d
        L.orc_ltimes_bf16_emul.argtypes = [i32, i32, i64, i64, i64, i64, vp, vp, vp]
        L.orc_ltimes_bf16_emul.restype = i32
        L.orc_mlp_nparams.argtypes = [i64, i64]
        L.orc_mlp_nparams.restype = i64
        L.orc_mlp_forward.argtypes = [i64, i64, i64, vp, vp, vp]
        L.orc_mlp_forward.restype = i32
        L.orc_mlp_loss_grad.argtypes = [i64, i64, i64, vp, vp, vp, vp]
        L.orc_mlp_loss_grad.restype = d
        L.orc_adam.argtypes = [i64, vp, vp, vp, vp, i64, d, d, d, d]
        L.orc_adam.restype = i32
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _layout_id(layout) -> int:
    return LAYOUTS.index(layout) if isinstance(layout, str) else int(layout)


def set_threads(n: int) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count in use."""
    return lib().orc_set_threads(int(n))


def ltimes(layout, Z, G, D, NM, L, psi) -> np.ndarray:
    """phi (flat, stored in ``layout`` order with D -> NM) from psi (flat, ``layout`` order)."""
    L = _f64(L).reshape(-1)
    psi = _f64(psi).reshape(-1)
    assert L.size == NM * D and psi.size == D * G * Z
    phi = np.empty(NM * G * Z, dtype=np.float64)
    rc = lib().orc_ltimes(_layout_id(layout), Z, G, D, NM, _ptr(L), _ptr(psi), _ptr(phi))
    if rc != 0:
        raise ValueError("orc_ltimes failed")
    return phi


def lplustimes(layout, Z, G, D, NM, Lplus, phi) -> np.ndarray:
    Lplus = _f64(Lplus).reshape(-1)
    phi = _f64(phi).reshape(-1)
    assert Lplus.size == D * NM and phi.size == NM * G * Z
    out = np.empty(D * G * Z, dtype=np.float64)
    rc = lib().orc_lplustimes(_layout_id(layout), Z, G, D, NM, _ptr(Lplus), _ptr(phi), _ptr(out))
    if rc != 0:
        raise ValueError("orc_lplustimes failed")
    return out


def ltimes_absscale(layout, Z, G, D, NM, L, psi) -> np.ndarray:
    L = _f64(L).reshape(-1)
    psi = _f64(psi).reshape(-1)
    out = np.empty(NM * G * Z, dtype=np.float64)
    rc = lib().orc_ltimes_absscale(_layout_id(layout), Z, G, D, NM, _ptr(L), _ptr(psi), _ptr(out))
    if rc != 0:
        raise ValueError("orc_ltimes_absscale failed")
    return out


def scattering(layout, Z, G, NM, S, mat, phi, absolute=False) -> np.ndarray:
    """phi_out (flat, ``layout`` order with D -> NM) = the scattering source of
    phi: S is [nmat][n_max + 1][G][G], mat [Z] int32 material of each zone.
    ``absolute`` returns the error scale sum |S| |phi| instead."""
    S = _f64(S).reshape(-1)
    phi = _f64(phi).reshape(-1)
    mat = np.ascontiguousarray(np.asarray(mat, dtype=np.int32).reshape(-1))
    import math
    nl = math.isqrt(NM - 1) + 1          # degrees 0 .. floor(sqrt(NM - 1))
    assert S.size % (nl * G * G) == 0 and phi.size == NM * G * Z and mat.size == Z
    nmat = S.size // (nl * G * G)
    out = np.empty(NM * G * Z, dtype=np.float64)
    f = lib().orc_scattering_absscale if absolute else lib().orc_scattering
    rc = f(_layout_id(layout), Z, G, NM, nmat, _ptr(S), mat.ctypes.data, _ptr(phi), _ptr(out))
    if rc != 0:
        raise ValueError("orc_scattering failed (%d)" % rc)
    return out


def mass(dim, D1D, Q1D, B1, Dq, X, absolute=False) -> np.ndarray:
    """Tensor-product mass operator per element: Y[e] = B^T diag(Dq[e]) B X[e];
    B1 [Q1D][D1D], Dq [NE][Q1D^dim], X [NE][D1D^dim] (first index fastest).
    ``absolute`` returns the error scale |B|^T |Dq| |B| |X| instead."""
    B1 = _f64(B1).reshape(-1)
    nd, nq = D1D ** dim, Q1D ** dim
    X = _f64(X).reshape(-1)
    Dq = _f64(Dq).reshape(-1)
    assert B1.size == Q1D * D1D and X.size % nd == 0 and Dq.size == (X.size // nd) * nq
    NE = X.size // nd
    Y = np.empty(NE * nd, dtype=np.float64)
    f = lib().orc_mass_absscale if absolute else lib().orc_mass
    rc = f(dim, D1D, Q1D, NE, _ptr(B1), _ptr(Dq), _ptr(X), _ptr(Y))
    if rc != 0:
        raise ValueError("orc_mass failed (%d)" % rc)
    return Y


def bgemm(n, off, A, B) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.int64)
    A = _f64(A)
    B = _f64(B)
    C = np.empty_like(A)
    lib().orc_bgemm(len(n), _ptr(n), _ptr(off), _ptr(A), _ptr(B), _ptr(C))
    return C


def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))


def ltimes_bf16_emul(mode, layout, Z, G, D, NM, L, psi) -> np.ndarray:
    L = _f64(L).reshape(-1)
    psi = _f64(psi).reshape(-1)
    phi = np.empty(NM * G * Z, dtype=np.float64)
    rc = lib().orc_ltimes_bf16_emul(int(mode), _layout_id(layout), Z, G, D, NM, _ptr(L), _ptr(psi), _ptr(phi))
    if rc != 0:
        raise ValueError("orc_ltimes_bf16_emul failed")
    return phi


def mlp_nparams(F, H) -> int:
    return int(lib().orc_mlp_nparams(F, H))


def mlp_forward(F, H, theta, X) -> np.ndarray:
    theta = _f64(theta)
    X = _f64(X).reshape(-1, F)
    y = np.empty(X.shape[0], dtype=np.float64)
    rc = lib().orc_mlp_forward(X.shape[0], F, H, _ptr(theta), _ptr(X), _ptr(y))
    if rc != 0:
        raise ValueError("orc_mlp_forward failed")
    return y


def mlp_loss_grad(F, H, theta, X, t):
    theta = _f64(theta)
    X = _f64(X).reshape(-1, F)
    t = _f64(t)
    g = np.empty_like(theta)
    loss = lib().orc_mlp_loss_grad(X.shape[0], F, H, _ptr(theta), _ptr(X), _ptr(t), _ptr(g))
    return float(loss), g


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays p, m, v given gradient g."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    rc = lib().orc_adam(p.size, _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(step), lr, b1, b2, eps)
    if rc != 0:
        raise ValueError("orc_adam failed")
