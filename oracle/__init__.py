"""CPU oracle for the Stream-K GEMM path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the HIP path.

Two independent oracles live here:

* ``gemm`` (numeric): C = alpha*A*B + beta*C in IEEE double by the paper's
  sequential cache-blocked loop nest (section 3.1, Algorithm 1), on the exact
  decoded values of the stored inputs.  Implemented in plain C
  (``oracle_gemm.c``), built with gcc.
* ``schedule`` (pure integer): which workgroup performs which MAC-loop
  iterations of which output tile, and who reconciles partial sums
  (section 4, Algorithm 5; section 5.2 hybrids; appendix A.1 grid model).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_gemm.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DT = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f8e4m3": 4}
ORD = {"row": 0, "col": 1}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        i64, f64, i32, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.oracle_gemm_f64.restype = i32
        L.oracle_gemm_f64.argtypes = [i64, i64, i64, f64, f64, i32, i32, i32, i32, i32,
                                      i64, i64, i64, vp, vp, vp, f64, f64, vp,
                                      i64, i64, i64, i32]
        L.oracle_gemm_elem.restype = f64
        L.oracle_gemm_elem.argtypes = [i64, i64, i64, f64, f64, i32, i32, i32, i32, i32,
                                       i64, i64, i64, vp, vp, vp, f64, f64]
        L.oracle_round.restype = i32
        L.oracle_round.argtypes = [vp, i64, i32, vp]
        L.oracle_decode_vec.restype = i32
        L.oracle_decode_vec.argtypes = [vp, i32, i64, vp]
        L.oracle_decode.restype = i32
        L.oracle_decode.argtypes = [vp, i32, i32, i64, i64, i64, f64, vp]
        _lib = L
    return _lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr() if hasattr(t, "data_ptr") else t.ctypes.data


def _cpu(op):
    """An Operand-like (tensor, ld, dtype, order, scale) on the CPU."""
    t = op.tensor
    if hasattr(t, "device") and t.device.type != "cpu":
        t = t.cpu()
    return t.contiguous()


def gemm(m, n, k, A, B, C=None, alpha=1.0, beta=0.0, c_type="f32",
         blk=(64, 64, 64), nthreads=0) -> np.ndarray:
    """Reference result (m x n float64, row-major) for operands given as
    ``workloads.Operand`` objects (``C`` likewise, read only if beta != 0)."""
    L = lib()
    out = np.empty((m, n), dtype=np.float64)
    ta, tb = _cpu(A), _cpu(B)
    tc = _cpu(C) if (C is not None and beta != 0.0) else None
    rc = L.oracle_gemm_f64(m, n, k, float(alpha), float(beta), DT[A.dtype],
                           DT[C.dtype] if C is not None else DT[c_type],
                           ORD[A.order], ORD[B.order],
                           ORD[C.order] if C is not None else 0,
                           A.ld, B.ld, C.ld if C is not None else n,
                           _ptr(ta), _ptr(tb), _ptr(tc), float(A.scale), float(B.scale),
                           out.ctypes.data, blk[0], blk[1], blk[2], int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_gemm_f64 failed with code {rc}")
    return out


def gemm_elems(rows, cols, k, A, B, C=None, alpha=1.0, beta=0.0) -> np.ndarray:
    """Reference values at the listed (row, col) positions only."""
    L = lib()
    ta, tb = _cpu(A), _cpu(B)
    tc = _cpu(C) if (C is not None and beta != 0.0) else None
    out = np.empty(len(rows), dtype=np.float64)
    for idx, (i, j) in enumerate(zip(rows, cols)):
        out[idx] = L.oracle_gemm_elem(int(i), int(j), k, float(alpha), float(beta),
                                      DT[A.dtype], DT[C.dtype] if C is not None else 1,
                                      ORD[A.order], ORD[B.order],
                                      ORD[C.order] if C is not None else 0,
                                      A.ld, B.ld, C.ld if C is not None else 0,
                                      _ptr(ta), _ptr(tb), _ptr(tc),
                                      float(A.scale), float(B.scale))
    return out


def round_to(x: np.ndarray, c_type: str) -> np.ndarray:
    """Round float64 values once (nearest, ties to even) into ``c_type`` and
    return the raw stored bits (uint16 / uint32 / float64 array)."""
    L = lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    dt = {"f64": np.float64, "f32": np.uint32, "f16": np.uint16, "bf16": np.uint16}[c_type]
    out = np.empty(x.shape, dtype=dt)
    rc = L.oracle_round(x.ctypes.data, x.size, DT[c_type], out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_round failed")
    return out


def decode(bits: np.ndarray, dtype: str) -> np.ndarray:
    """Exact double values of stored elements given as raw bits."""
    L = lib()
    bits = np.ascontiguousarray(bits)
    out = np.empty(bits.shape, dtype=np.float64)
    L.oracle_decode_vec(bits.ctypes.data, DT[dtype], bits.size, out.ctypes.data)
    return out


def decode_operand(op) -> np.ndarray:
    """Exact double values (rows x cols, scale applied) of an Operand."""
    L = lib()
    t = _cpu(op)
    out = np.empty((op.rows, op.cols), dtype=np.float64)
    L.oracle_decode(_ptr(t), DT[op.dtype], ORD[op.order], op.ld, op.rows, op.cols,
                    float(op.scale), out.ctypes.data)
    return out
