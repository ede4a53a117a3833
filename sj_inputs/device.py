"""ctypes access to the generator's device fill kernel (libsjfill.so)."""
from __future__ import annotations

import ctypes
import os

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsjfill.so")
_lib = None

DIST_U01 = 0
DIST_SYM = 1
DIST_U01_24 = 2


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is missing: build it with `python -m paper_1904_08555_amd.build`")
        L = ctypes.CDLL(_LIB)
        L.sjgen_fill.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p]
        L.sjgen_fill.restype = ctypes.c_int
        _lib = L
    return _lib


def fill(tensor, seed: int, arr: int, dist: int = DIST_U01, layout: int = -1, dims=(0, 0, 0), stream=None):
    """Fill a CUDA float64/float32 tensor in place with generator values.
    ``layout`` >= 0: the tensor holds an (A, G, Z) array stored in that layout
    order (dims = (A, G, Z)) and values follow its logical D-G-Z index."""
    import torch
    if tensor.dtype == torch.float64:
        dt = 0
    elif tensor.dtype == torch.float32:
        dt = 1
    else:
        raise TypeError("fill supports float64 and float32 tensors")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    A, G, Z = dims
    rc = lib().sjgen_fill(tensor.data_ptr(), dt, dist, seed & (2 ** 64 - 1), arr, layout, tensor.numel(), A, G, Z,
                          stream)
    if rc != 0:
        raise RuntimeError(f"sjgen_fill failed with code {rc}")
    return tensor
