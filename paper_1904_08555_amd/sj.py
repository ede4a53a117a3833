"""ctypes binding of ``libsj.so`` (declared in ``include/sj.h``).

Argument marshalling only: every function forwards to the C entry point of the
same name.  Buffers may be given as torch tensors (their ``data_ptr()`` is
passed) or as integer device addresses; ``stream`` defaults to torch's current
stream when torch has a GPU, else the null stream.  Errors raise ``SJError``
carrying the status and the library's message.  The library must have been
built (``python -m paper_1904_08555_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsj.so")

# sj_status
SJ_OK = 0
SJ_ERR_INVALID_ARG = 1
SJ_ERR_UNSUPPORTED = 2
SJ_ERR_COMPILE = 3
SJ_ERR_LOAD = 4
SJ_ERR_LAUNCH = 5
SJ_ERR_ALIGN = 6
SJ_ERR_ALIAS = 7
SJ_ERR_OOM = 8
SJ_ERR_HIP = 9
SJ_ERR_NOT_INITIALIZED = 10
# sj_kernel
SJ_LTIMES = 1
SJ_LPLUSTIMES = 2
SJ_BGEMM = 3
SJ_MLP_FWD = 4
SJ_MLP_BWD = 5
SJ_ADAM = 6
SJ_LTIMES_LPLUS = 7
SJ_SCATTERING = 8
SJ_MASS = 9
# sj_layout
LAYOUTS = ("DGZ", "DZG", "GDZ", "GZD", "ZDG", "ZGD")
SJ_DGZ, SJ_DZG, SJ_GDZ, SJ_GZD, SJ_ZDG, SJ_ZGD = range(6)
# sj_dtype
SJ_F64 = 0
SJ_BF16 = 1
SJ_BF16X3 = 2
SJ_F32 = 3
# sj_variant
SJ_VAR_AUTO = 0
SJ_VAR_DIRECT = 1
SJ_VAR_STAGED = 2
SJ_VAR_MFMA = 3
# flags
SJ_FLAG_COMPILE_ONLY = 0x1
SJ_FLAG_INDEX64 = 0x2
SJ_FLAG_LOADS_CACHED = 0x4
SJ_FLAG_LOADS_NONTEMPORAL = 0x8
SJ_FLAG_STORES_CACHED = 0x10
SJ_FLAG_STORES_NONTEMPORAL = 0x20
SJ_FLAG_ACCUMULATE = 0x40
SJ_FLAG_GENERIC_PER_LAYOUT = 0x80
SJ_FLAG_DEBUG_FAIL_COMPILE = 0x100
SJ_FLAG_XCD_CONTIGUOUS = 0x200
SJ_FLAG_XCD_INTERLEAVED = 0x400

EXPORTED = (
    "sj_init", "sj_layout_from_string", "sj_specialize", "sj_specialize_values", "sj_specialize_with_code", "sj_run", "sj_generic_run", "sj_batch_plan",
    "sj_batch_run", "sj_batch_graph_capture", "sj_batch_graph_launch", "sj_batch_plan_arrays", "sj_plan_destroy",
    "sj_run_adam", "sj_run_mlp_bwd_noalloc", "sj_time_run", "sj_resolve", "sj_emit_source", "sj_handle_info", "sj_handle_code", "sj_stats", "sj_cache_clear",
    "sj_last_error", "sj_status_string",
)


class sj_spec(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("Z", ctypes.c_int64), ("G", ctypes.c_int64), ("D", ctypes.c_int64), ("NM", ctypes.c_int64),
        ("count", ctypes.c_int64), ("class_mask", ctypes.c_uint32),
        ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32), ("unroll", ctypes.c_int32),
        ("block", ctypes.c_int32), ("flags", ctypes.c_uint32), ("order", ctypes.c_int32),
        ("rows", ctypes.c_int64), ("inputs", ctypes.c_int64), ("width", ctypes.c_int64),
    ]


class sj_kernel_info(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("vgprs", ctypes.c_int32), ("agprs", ctypes.c_int32),
        ("sgprs", ctypes.c_int32), ("lds_bytes", ctypes.c_int32), ("scratch_bytes", ctypes.c_int32),
        ("occupancy", ctypes.c_int32), ("block", ctypes.c_int32), ("grid", ctypes.c_int64),
        ("variant", ctypes.c_int32), ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32),
        ("unroll", ctypes.c_int32), ("emit_ms", ctypes.c_double), ("compile_ms", ctypes.c_double),
        ("load_ms", ctypes.c_double), ("code_bytes", ctypes.c_uint64), ("key_hash", ctypes.c_uint64),
        ("kernel_name", ctypes.c_char * 64),
    ]


class sj_stats_t(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("lookups", ctypes.c_uint64), ("hits", ctypes.c_uint64),
        ("misses", ctypes.c_uint64), ("compiles", ctypes.c_uint64), ("compile_failures", ctypes.c_uint64),
        ("loads", ctypes.c_uint64), ("inflight_waits", ctypes.c_uint64), ("entries", ctypes.c_uint64),
        ("emit_ms_total", ctypes.c_double), ("compile_ms_total", ctypes.c_double), ("load_ms_total", ctypes.c_double),
    ]


class SJError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.message = message
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")


_STATUS_NAMES = {
    0: "SJ_OK", 1: "SJ_ERR_INVALID_ARG", 2: "SJ_ERR_UNSUPPORTED", 3: "SJ_ERR_COMPILE", 4: "SJ_ERR_LOAD",
    5: "SJ_ERR_LAUNCH", 6: "SJ_ERR_ALIGN", 7: "SJ_ERR_ALIAS", 8: "SJ_ERR_OOM", 9: "SJ_ERR_HIP",
    10: "SJ_ERR_NOT_INITIALIZED",
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libsj.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1904_08555_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "sj_init": [ctypes.c_int],
        "sj_layout_from_string": [ctypes.c_char_p, P(i32)],
        "sj_specialize": [ctypes.c_int, P(sj_spec), P(vp)],
        "sj_specialize_with_code": [ctypes.c_int, P(sj_spec), ctypes.c_char_p, ctypes.c_size_t, P(vp)],
        "sj_specialize_values": [ctypes.c_int, P(sj_spec), P(d), ctypes.c_size_t, P(vp)],
        "sj_run": [vp, P(vp), ctypes.c_int, vp],
        "sj_generic_run": [ctypes.c_int, P(sj_spec), P(vp), ctypes.c_int, vp],
        "sj_batch_plan": [vp, vp, i64, P(vp)],
        "sj_batch_run": [vp, vp, vp, vp, vp],
        "sj_batch_graph_capture": [vp, vp, vp, vp, vp],
        "sj_batch_graph_launch": [vp, vp],
        "sj_batch_plan_arrays": [vp, P(vp), P(vp), P(i64)],
        "sj_plan_destroy": [vp],
        "sj_run_adam": [vp, P(vp), ctypes.c_int, i64, d, d, d, d, vp],
        "sj_run_mlp_bwd_noalloc": [vp, P(vp), ctypes.c_int, vp],
        "sj_time_run": [vp, P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp,
                        P(ctypes.c_float)],
        "sj_resolve": [ctypes.c_int, P(sj_spec), P(sj_spec)],
        "sj_emit_source": [ctypes.c_int, P(sj_spec), ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_size_t)],
        "sj_handle_info": [vp, P(sj_kernel_info)],
        "sj_handle_code": [vp, P(vp), P(ctypes.c_size_t)],
        "sj_stats": [P(sj_stats_t)],
        "sj_cache_clear": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.sj_last_error.argtypes = []
    L.sj_last_error.restype = ctypes.c_char_p
    L.sj_status_string.argtypes = [ctypes.c_int]
    L.sj_status_string.restype = ctypes.c_char_p
    del u32
    _lib = L
    return L


def _check(status: int):
    if status != SJ_OK:
        msg = lib().sj_last_error()
        raise SJError(status, msg.decode(errors="replace") if msg else "")


def _addr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    raise TypeError(f"cannot take a device address of {type(x)!r}")


def _stream(stream):
    if stream is not None:
        if isinstance(stream, int):
            return stream
        return int(getattr(stream, "cuda_stream", stream))
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return 0


def _layout(layout) -> int:
    if isinstance(layout, str):
        return sj_layout_from_string(layout)
    return int(layout)


def make_spec(**kw) -> sj_spec:
    s = sj_spec()
    s.struct_size = ctypes.sizeof(sj_spec)
    for k, v in kw.items():
        if k == "layout":
            v = _layout(v)
        if not hasattr(s, k):
            raise TypeError(f"sj_spec has no field {k!r}")
        setattr(s, k, int(v))
    return s


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[_addr(p) for p in ptrs])
    return arr


# ------------------------------------------------------------- entry points

def sj_init(device: int = 0) -> None:
    _check(lib().sj_init(int(device)))


def sj_layout_from_string(name: str) -> int:
    out = ctypes.c_int32()
    _check(lib().sj_layout_from_string(name.encode(), ctypes.byref(out)))
    return out.value


class Handle:
    """A specialization handle (owned by the library's cache)."""

    def __init__(self, ptr: int, kernel: int):
        self.ptr = ptr
        self.kernel = kernel

    def __int__(self):
        return self.ptr

    def __eq__(self, other):
        return isinstance(other, Handle) and other.ptr == self.ptr

    def __hash__(self):
        return hash(self.ptr)

    def __repr__(self):
        return f"Handle(0x{self.ptr:x}, kernel={self.kernel})"


def sj_specialize(kernel: int, spec: sj_spec | None = None, **kw) -> Handle:
    if spec is None:
        spec = make_spec(**kw)
    out = ctypes.c_void_p()
    _check(lib().sj_specialize(int(kernel), ctypes.byref(spec), ctypes.byref(out)))
    return Handle(out.value, int(kernel))


def sj_specialize_values(kernel: int, weights, spec: sj_spec | None = None, **kw) -> Handle:
    """Value specialization: `weights` (the L or L+ matrix the kernel would read, host,
    any array-like of NM * D floats) compiled into the kernel as constants."""
    import numpy as np
    if spec is None:
        spec = make_spec(**kw)
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    out = ctypes.c_void_p()
    _check(lib().sj_specialize_values(int(kernel), ctypes.byref(spec), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      w.size, ctypes.byref(out)))
    return Handle(out.value, int(kernel))


def sj_specialize_with_code(kernel: int, code: bytes, spec: sj_spec | None = None, **kw) -> Handle:
    if spec is None:
        spec = make_spec(**kw)
    out = ctypes.c_void_p()
    _check(lib().sj_specialize_with_code(int(kernel), ctypes.byref(spec), code, len(code), ctypes.byref(out)))
    return Handle(out.value, int(kernel))


def sj_run(handle: Handle, ptrs, stream=None) -> None:
    arr = _ptr_array(ptrs)
    _check(lib().sj_run(handle.ptr, arr, len(ptrs), _stream(stream)))


def sj_run_mlp_bwd_noalloc(handle: Handle, ptrs, stream=None) -> None:
    """ptrs = {theta, X, t, grad, loss}: the backward pass with the library's
    static scratch as workspace (see include/sj.h)."""
    arr = _ptr_array(ptrs)
    _check(lib().sj_run_mlp_bwd_noalloc(handle.ptr, arr, len(ptrs), _stream(stream)))


def sj_generic_run(kernel: int, ptrs, spec: sj_spec | None = None, stream=None, **kw) -> None:
    if spec is None:
        spec = make_spec(**kw)
    arr = _ptr_array(ptrs)
    _check(lib().sj_generic_run(int(kernel), ctypes.byref(spec), arr, len(ptrs), _stream(stream)))


def sj_time_run(handle: Handle, ptrs, warmup: int = 2, reps: int = 10, flush=None, stream=None):
    """Per-launch durations in ms (list of floats); see include/sj.h."""
    arr = _ptr_array(ptrs)
    out = (ctypes.c_float * reps)()
    fbytes = 0 if flush is None else int(flush.numel() * flush.element_size())
    _check(lib().sj_time_run(handle.ptr, arr, len(ptrs), int(warmup), int(reps), _addr(flush), fbytes,
                             _stream(stream), out))
    return list(out)


def sj_resolve(kernel: int, spec: sj_spec | None = None, **kw) -> dict:
    """The canonical request a spec resolves to (defaults filled in, load and
    store forms explicit in ``flags``), as a dict of the sj_spec fields."""
    if spec is None:
        spec = make_spec(**kw)
    out = sj_spec()
    _check(lib().sj_resolve(int(kernel), ctypes.byref(spec), ctypes.byref(out)))
    return {name: getattr(out, name) for name, _ in sj_spec._fields_ if name != "struct_size"}


def sj_emit_source(kernel: int, spec: sj_spec | None = None, **kw) -> str:
    if spec is None:
        spec = make_spec(**kw)
    need = ctypes.c_size_t()
    _check(lib().sj_emit_source(int(kernel), ctypes.byref(spec), None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().sj_emit_source(int(kernel), ctypes.byref(spec), buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def sj_handle_info(handle: Handle) -> dict:
    info = sj_kernel_info()
    info.struct_size = ctypes.sizeof(sj_kernel_info)
    _check(lib().sj_handle_info(handle.ptr, ctypes.byref(info)))
    out = {name: getattr(info, name) for name, _ in sj_kernel_info._fields_ if name != "struct_size"}
    out["kernel_name"] = info.kernel_name.decode()
    return out


def sj_handle_code(handle: Handle) -> bytes:
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _check(lib().sj_handle_code(handle.ptr, ctypes.byref(p), ctypes.byref(n)))
    return ctypes.string_at(p.value, n.value)


def sj_stats() -> dict:
    st = sj_stats_t()
    st.struct_size = ctypes.sizeof(sj_stats_t)
    _check(lib().sj_stats(ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in sj_stats_t._fields_ if name != "struct_size"}


def sj_cache_clear() -> None:
    _check(lib().sj_cache_clear())


def sj_last_error() -> str:
    m = lib().sj_last_error()
    return m.decode(errors="replace") if m else ""


def sj_status_string(status: int) -> str:
    return lib().sj_status_string(int(status)).decode()


class Plan:
    def __init__(self, ptr: int, count: int):
        self.ptr = ptr
        self.count = count

    def __repr__(self):
        return f"Plan(0x{self.ptr:x}, count={self.count})"


def sj_batch_plan(handle: Handle, n_host) -> Plan:
    import numpy as np
    n = np.ascontiguousarray(n_host, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib().sj_batch_plan(handle.ptr, n.ctypes.data, len(n), ctypes.byref(out)))
    return Plan(out.value, len(n))


def sj_batch_run(plan: Plan, A, B, C, stream=None) -> None:
    _check(lib().sj_batch_run(plan.ptr, _addr(A), _addr(B), _addr(C), _stream(stream)))


def sj_batch_graph_capture(plan: Plan, A, B, C, stream=None) -> None:
    _check(lib().sj_batch_graph_capture(plan.ptr, _addr(A), _addr(B), _addr(C), _stream(stream)))


def sj_batch_graph_launch(plan: Plan, stream=None) -> None:
    _check(lib().sj_batch_graph_launch(plan.ptr, _stream(stream)))


def sj_batch_plan_arrays(plan: Plan):
    n = ctypes.c_void_p()
    off = ctypes.c_void_p()
    tot = ctypes.c_int64()
    _check(lib().sj_batch_plan_arrays(plan.ptr, ctypes.byref(n), ctypes.byref(off), ctypes.byref(tot)))
    return n.value, off.value, tot.value


def sj_plan_destroy(plan: Plan) -> None:
    _check(lib().sj_plan_destroy(plan.ptr))
    plan.ptr = 0


def sj_run_adam(handle: Handle, ptrs, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None) -> None:
    arr = _ptr_array(ptrs)
    _check(lib().sj_run_adam(handle.ptr, arr, len(ptrs), int(step), float(lr), float(b1), float(b2), float(eps),
                             _stream(stream)))
