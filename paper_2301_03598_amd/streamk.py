"""Thin ctypes binding of the Stream-K C ABI (include/streamk.h).

Argument marshalling only: every step of the GEMM runs in libstreamk.so.
The functions carry the C names; ``check`` turns a status into an exception.
If the library is not built, importing the compute entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_float, c_int32, c_int64, c_uint64, c_void_p, c_char_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("STREAMK_LIB") or os.path.join(_HERE, "libstreamk.so")

# status codes
SK_OK, SK_ERR_INVALID_VALUE, SK_ERR_UNSUPPORTED, SK_ERR_WORKSPACE_TOO_SMALL, \
    SK_ERR_MISALIGNED, SK_ERR_HIP, SK_ERR_TIMEOUT = range(7)
# dtypes / orders / schedules
SK_F64, SK_F32, SK_F16, SK_BF16, SK_F8_E4M3 = range(5)
SK_ROW_MAJOR, SK_COL_MAJOR = 0, 1
SK_SCHED_AUTO, SK_SCHED_DP, SK_SCHED_SK, SK_SCHED_DP_1TILE_SK, SK_SCHED_2TILE_SK_DP, SK_SCHED_FIXED_SPLIT = range(6)
SK_FLAG_NO_XCD_REMAP = 0x1
SK_FLAG_ROW_MAJOR_TILES = 0x2
SK_FLAG_STATIC_DP_TILES = 0x4
SK_MAX_GRID, SK_MAX_PEERS = 1024, 64
SK_FIXUP_AUTO, SK_FIXUP_SERIAL, SK_FIXUP_SPREAD = 0, 1, 2
FIXUP = {"auto": SK_FIXUP_AUTO, "serial": SK_FIXUP_SERIAL, "spread": SK_FIXUP_SPREAD}
FIXUP_NAME = {v: k for k, v in FIXUP.items()}

DTYPE = {"f64": SK_F64, "f32": SK_F32, "f16": SK_F16, "bf16": SK_BF16, "f8e4m3": SK_F8_E4M3}
ORDER = {"row": SK_ROW_MAJOR, "col": SK_COL_MAJOR}
SCHED = {"auto": SK_SCHED_AUTO, "dp": SK_SCHED_DP, "sk": SK_SCHED_SK,
         "dp1sk": SK_SCHED_DP_1TILE_SK, "2tsk": SK_SCHED_2TILE_SK_DP, "fs": SK_SCHED_FIXED_SPLIT}
SCHED_NAME = {v: k for k, v in SCHED.items()}

SK_NOALLOC_SCRATCH_BYTES = 80 << 20

EXPORTS = ["sk_plan", "sk_workspace_size", "sk_gemm", "sk_gemm_noalloc", "sk_gemm_grouped",
           "sk_workspace_check", "sk_status_string"]


class sk_gemm_desc_t(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("k", c_int64),
                ("alpha", c_double), ("beta", c_double),
                ("ab_type", c_int32), ("c_type", c_int32),
                ("a_order", c_int32), ("b_order", c_int32), ("c_order", c_int32),
                ("reserved0", c_int32),
                ("lda", c_int64), ("ldb", c_int64), ("ldc", c_int64),
                ("A", c_void_p), ("B", c_void_p), ("C", c_void_p),
                ("a_scale", c_float), ("b_scale", c_float)]


class sk_config_t(ctypes.Structure):
    _fields_ = [("sched", c_int32), ("blk_m", c_int32), ("blk_n", c_int32), ("blk_k", c_int32),
                ("grid", c_int32), ("wg_slots", c_int32), ("sk_threshold_waves", c_int32),
                ("flags", c_int32),
                ("model_a", c_double), ("model_b", c_double), ("model_c", c_double),
                ("model_d", c_double),
                ("trace", c_void_p), ("trace_capacity", c_int64),
                ("wait_limit_us", c_int32), ("fixup", c_int32), ("model_bw", c_double),
                ("split", c_int32)]


class sk_plan_t(ctypes.Structure):
    _fields_ = [("sched", c_int32), ("blk_m", c_int32), ("blk_n", c_int32), ("blk_k", c_int32),
                ("grid", c_int32), ("wg_slots", c_int32), ("dp_first", c_int32),
                ("xcd_remap", c_int32),
                ("tiles", c_int64), ("iters_total", c_int64),
                ("sk_tile_begin", c_int64), ("sk_tile_end", c_int64),
                ("sk_iter_begin", c_int64), ("sk_iters", c_int64),
                ("dp_tiles", c_int64), ("workspace_bytes", c_uint64),
                ("fixup", c_int32), ("max_peers", c_int32), ("split", c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SkError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {sk_status_string(status)}")


_lib = None


def lib():
    """Load libstreamk.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2301_03598_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.sk_plan.argtypes = [P(sk_gemm_desc_t), c_int32, P(sk_config_t), P(sk_plan_t)]
        L.sk_workspace_size.argtypes = [P(sk_gemm_desc_t), c_int32, P(sk_config_t),
                                        P(ctypes.c_size_t)]
        L.sk_gemm.argtypes = [P(sk_gemm_desc_t), P(sk_config_t), c_void_p, ctypes.c_size_t, c_void_p]
        L.sk_gemm_noalloc.argtypes = [P(sk_gemm_desc_t), P(sk_config_t), c_void_p, c_void_p]
        L.sk_gemm_grouped.argtypes = [P(sk_gemm_desc_t), c_int32, P(sk_config_t), c_void_p,
                                      ctypes.c_size_t, c_void_p]
        L.sk_workspace_check.argtypes = [c_void_p, ctypes.c_size_t, c_void_p]
        L.sk_status_string.argtypes = [c_int32]
        L.sk_status_string.restype = c_char_p
        for f in EXPORTS[:-1]:
            getattr(L, f).restype = c_int32
        _lib = L
    return _lib


def _cfg_ptr(cfg):
    return ctypes.byref(cfg) if cfg is not None else None


# ---- the C entry points, same names -------------------------------------

def sk_status_string(status: int) -> str:
    return lib().sk_status_string(int(status)).decode()


def sk_plan(descs, cfg=None):
    arr, n = _desc_array(descs)
    out = sk_plan_t()
    st = lib().sk_plan(arr, n, _cfg_ptr(cfg), ctypes.byref(out))
    return st, out


def sk_workspace_size(descs, cfg=None):
    arr, n = _desc_array(descs)
    size = ctypes.c_size_t(0)
    st = lib().sk_workspace_size(arr, n, _cfg_ptr(cfg), ctypes.byref(size))
    return st, size.value


def sk_gemm(desc, cfg, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    return lib().sk_gemm(ctypes.byref(desc), _cfg_ptr(cfg), c_void_p(workspace_ptr or None),
                         ws_bytes, c_void_p(stream or None))


def sk_gemm_noalloc(desc, cfg, wait_error_ptr: int, stream: int) -> int:
    return lib().sk_gemm_noalloc(ctypes.byref(desc), _cfg_ptr(cfg), c_void_p(wait_error_ptr or None),
                                 c_void_p(stream or None))


def sk_gemm_grouped(descs, cfg, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    """``descs`` may be a ctypes array or a host address (int) of ``count``
    packed descriptors together with a count: (address, count)."""
    if isinstance(descs, tuple):
        addr, n = descs
        arr = ctypes.cast(c_void_p(addr), ctypes.POINTER(sk_gemm_desc_t))
    else:
        arr, n = _desc_array(descs)
    return lib().sk_gemm_grouped(arr, n, _cfg_ptr(cfg), c_void_p(workspace_ptr or None), ws_bytes,
                                 c_void_p(stream or None))


def sk_workspace_check(workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    return lib().sk_workspace_check(c_void_p(workspace_ptr or None), ws_bytes,
                                    c_void_p(stream or None))


# ---- marshalling helpers -------------------------------------------------

def _desc_array(descs):
    if isinstance(descs, sk_gemm_desc_t):
        return ctypes.pointer(descs), 1
    if isinstance(descs, ctypes.Array):
        return ctypes.cast(descs, ctypes.POINTER(sk_gemm_desc_t)), len(descs)
    arr = (sk_gemm_desc_t * len(descs))(*descs)
    return ctypes.cast(arr, ctypes.POINTER(sk_gemm_desc_t)), len(descs)


def check(status: int, where: str = "") -> None:
    if status != SK_OK:
        raise SkError(status, where)


def make_desc(m, n, k, A, B, C, *, ab_type, c_type, a_order="row", b_order="row",
              c_order="row", lda=0, ldb=0, ldc=0, alpha=1.0, beta=0.0,
              a_scale=1.0, b_scale=1.0) -> sk_gemm_desc_t:
    """Build a descriptor; A, B, C are device addresses (ints) or objects
    with data_ptr()."""
    def addr(x):
        if x is None:
            return None
        return x.data_ptr() if hasattr(x, "data_ptr") else int(x)
    d = sk_gemm_desc_t()
    d.m, d.n, d.k = int(m), int(n), int(k)
    d.alpha, d.beta = float(alpha), float(beta)
    d.ab_type = DTYPE[ab_type] if isinstance(ab_type, str) else int(ab_type)
    d.c_type = DTYPE[c_type] if isinstance(c_type, str) else int(c_type)
    d.a_order = ORDER[a_order] if isinstance(a_order, str) else int(a_order)
    d.b_order = ORDER[b_order] if isinstance(b_order, str) else int(b_order)
    d.c_order = ORDER[c_order] if isinstance(c_order, str) else int(c_order)
    d.lda, d.ldb, d.ldc = int(lda), int(ldb), int(ldc)
    d.A, d.B, d.C = addr(A), addr(B), addr(C)
    d.a_scale, d.b_scale = float(a_scale), float(b_scale)
    return d


def make_config(sched="auto", blk=None, grid=0, wg_slots=0, threshold=0, flags=0,
                model=None, trace_ptr=0, trace_capacity=0, fixup="auto",
                wait_limit_us=0, split=0) -> sk_config_t:
    c = sk_config_t()
    c.split = int(split)
    c.fixup = FIXUP[fixup] if isinstance(fixup, str) else int(fixup)
    c.wait_limit_us = int(wait_limit_us)
    c.sched = SCHED[sched] if isinstance(sched, str) else int(sched)
    if blk is not None:
        c.blk_m, c.blk_n = int(blk[0]), int(blk[1])
        c.blk_k = int(blk[2]) if len(blk) > 2 else 0
    c.grid, c.wg_slots, c.sk_threshold_waves, c.flags = int(grid), int(wg_slots), int(threshold), int(flags)
    if model is not None:
        c.model_a, c.model_b, c.model_c, c.model_d = (float(v) for v in model)
    c.trace = trace_ptr or None
    c.trace_capacity = int(trace_capacity)
    return c
