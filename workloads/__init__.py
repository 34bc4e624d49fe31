"""Seeded synthetic inputs for the Stream-K GEMM workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
draws random numbers and lays them out in memory; it performs none of the
GEMM arithmetic (no products, no sums, no tiling), so neither the CPU oracle
nor the HIP path depends on the other through it.

Random draws follow one convention everywhere: ``numpy.random.default_rng``
(PCG64) with the stated seed, values drawn in float64, A before B, each matrix
filled in row-major order of its logical (rows x cols) shape, then rounded to
the storage dtype by the library conversion (round to nearest even).  Large
benchmark operands, whose host generation would dominate a run, are instead
drawn on the device with a seeded ``torch.Generator``; both recipes give the
value distributions of the paper's workloads (uniform[-1,1] and N(0,1)
entries, section 6 "Dataset"), and neither is used to decide correctness.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# dtype names used throughout the harness; the numeric codes are the C-ABI's
# (see include/streamk.h) and are restated here only as an interface table.
DTYPE_CODES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f8e4m3": 4}
DTYPE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f8e4m3": 1}
ORDER_CODES = {"row": 0, "col": 1}

FP8_E4M3_MAX = 448.0


def _torch():
    import torch  # imported lazily: the oracle tests need only numpy
    return torch


def torch_dtype(name: str):
    t = _torch()
    return {
        "f64": t.float64,
        "f32": t.float32,
        "f16": t.float16,
        "bf16": t.bfloat16,
        "f8e4m3": t.float8_e4m3fn,
    }[name]


# ---------------------------------------------------------------------------
# value draws (float64, host)
# ---------------------------------------------------------------------------

def uniform(shape: Sequence[int], rng: np.random.Generator, lo=-1.0, hi=1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=tuple(shape))


def normal(shape: Sequence[int], rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(size=tuple(shape))


def small_integers(shape: Sequence[int], rng: np.random.Generator, lo=-4, hi=4) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=tuple(shape)).astype(np.float64)


def draw(dist: str, shape: Sequence[int], rng: np.random.Generator) -> np.ndarray:
    if dist == "uniform":
        return uniform(shape, rng)
    if dist == "normal":
        return normal(shape, rng)
    if dist == "int4":
        return small_integers(shape, rng)
    if dist == "zeros":
        return np.zeros(tuple(shape))
    raise ValueError(f"unknown distribution {dist!r}")


# ---------------------------------------------------------------------------
# storage: logical matrix -> bytes in the requested dtype and major order
# ---------------------------------------------------------------------------

@dataclass
class Operand:
    """A matrix as it is handed to the library: a contiguous CPU tensor whose
    bytes hold the logical (rows x cols) matrix in ``order`` with leading
    dimension ``ld`` (elements), plus the FP8 dequantisation scale."""
    tensor: object          # torch.Tensor (CPU or device), contiguous
    rows: int
    cols: int
    dtype: str
    order: str
    ld: int
    scale: float = 1.0

    def to(self, device) -> "Operand":
        return Operand(self.tensor.to(device), self.rows, self.cols, self.dtype,
                       self.order, self.ld, self.scale)


def fp8_absmax_scale(x: np.ndarray) -> float:
    """Per-tensor scale s = absmax / 448, held in FP32 (the precision set's FP8 recipe)."""
    amax = float(np.max(np.abs(x))) if x.size else 0.0
    s = np.float32(amax / FP8_E4M3_MAX) if amax > 0 else np.float32(1.0)
    return float(s)


def store(x: np.ndarray, dtype: str, order: str, scale: Optional[float] = None) -> Operand:
    """Round ``x`` (float64, logical rows x cols) to ``dtype`` with the library
    conversion and lay it out in ``order``.  For FP8 the stored code is
    RNE(x / scale) in OCP e4m3fn; ``scale=None`` picks the absmax scale and
    ``scale=1.0`` stores the values themselves (integer-exact tests)."""
    t = _torch()
    rows, cols = x.shape
    s = 1.0
    src = x
    if dtype == "f8e4m3":
        s = fp8_absmax_scale(x) if scale is None else float(scale)
        src = x / np.float64(s) if s != 1.0 else x
        src = np.clip(src, -FP8_E4M3_MAX, FP8_E4M3_MAX)
    tx = t.from_numpy(np.ascontiguousarray(src))
    if dtype == "f8e4m3":
        # float64 -> float32 is exact for the clipped quotients we need only
        # when followed by one more rounding; go through float32 explicitly
        # and then to e4m3 (both steps round to nearest even).
        tx = tx.to(t.float32).to(t.float8_e4m3fn)
    else:
        tx = tx.to(torch_dtype(dtype))
    if order == "row":
        tx = tx.contiguous()
        ld = cols
    else:
        tx = tx.t().contiguous()
        ld = rows
    return Operand(tx, rows, cols, dtype, order, ld, s)


# ---------------------------------------------------------------------------
# workload recipes (the configurations the paper's evaluation is shaped like)
# ---------------------------------------------------------------------------

def round8_clamped(x: float, lo=128, hi=8192) -> int:
    v = int(round(x / 8.0)) * 8
    return max(lo, min(hi, v))


def sweep_shapes(count: int = 2048, seed: int = 1) -> List[Tuple[int, int, int]]:
    """Geometry sweep standing in for the paper's 32,824-problem corpus
    (section 6 "Dataset": m, n, k log-sampled in [128, 8192]).  Per problem
    draw m, then n, then k as exp(U(ln 128, ln 8192)), rounded to the nearest
    multiple of 8 and clamped to the domain."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(128.0), math.log(8192.0)
    out = []
    for _ in range(count):
        m, n, k = (round8_clamped(math.exp(rng.uniform(lo, hi))) for _ in range(3))
        out.append((m, n, k))
    return out


def grouped_shapes(count: int = 512, seed: int = 3) -> List[Tuple[int, int, int]]:
    """Grouped batch: m, n uniform over multiples of 64 in [64, 2048], k
    uniform over multiples of 128 in [128, 8192]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = 64 * int(rng.integers(1, 33))
        n = 64 * int(rng.integers(1, 33))
        k = 128 * int(rng.integers(1, 65))
        out.append((m, n, k))
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    m: int
    n: int
    k: int
    dtype: str  # "bf16" or "f16"


def serving_trace(rate_per_s: float = 20000.0, duration_s: float = 10.0,
                  seed: int = 4, max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals of mixed-shape GEMM requests: 60% small (m,n in
    [64,512], k in [256,2048]), 30% medium (m,n in [512,2048], k in
    [1024,8192]), 10% large (m,n in [2048,8192], k in [2048,16384]); sizes
    uniform within the class range rounded to multiples of 8; dtype BF16 or
    FP16 with equal probability."""
    rng = np.random.default_rng(seed)
    classes = [((64, 512), (256, 2048)), ((512, 2048), (1024, 8192)),
               ((2048, 8192), (2048, 16384))]
    probs = np.array([0.6, 0.3, 0.1])
    t = 0.0
    reqs: List[Request] = []
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        c = int(rng.choice(3, p=probs))
        (mlo, mhi), (klo, khi) = classes[c]
        m = int(round(rng.uniform(mlo, mhi) / 8)) * 8
        n = int(round(rng.uniform(mlo, mhi) / 8)) * 8
        k = int(round(rng.uniform(klo, khi) / 8)) * 8
        dt = "bf16" if rng.uniform() < 0.5 else "f16"
        reqs.append(Request(len(reqs), t, m, n, k, dt))
        if max_requests is not None and len(reqs) >= max_requests:
            break
    return reqs


PRECISION_SHAPES = {
    "a": (8192, 8192, 8192),
    "b": (256, 256, 65536),
    "c": (4096, 1024, 4096),
}


def gemm_operands(m: int, n: int, k: int, dtype: str, seed: int, dist: str,
                  a_order="row", b_order="row", fp8_scale: Optional[float] = None):
    """Draw A (m x k) then B (k x n) from one generator and store them."""
    rng = np.random.default_rng(seed)
    a = draw(dist, (m, k), rng)
    b = draw(dist, (k, n), rng)
    return store(a, dtype, a_order, fp8_scale), store(b, dtype, b_order, fp8_scale)


# ---------------------------------------------------------------------------
# device-side draws for large benchmark operands
# ---------------------------------------------------------------------------

def device_fill_(tensor, dist: str, gen) -> None:
    """Fill a device tensor in place from a seeded torch.Generator."""
    t = _torch()
    if dist == "uniform":
        tmp = t.empty(tensor.shape, dtype=t.float32, device=tensor.device)
        tmp.uniform_(-1.0, 1.0, generator=gen)
    elif dist == "normal":
        tmp = t.empty(tensor.shape, dtype=t.float32, device=tensor.device)
        tmp.normal_(0.0, 1.0, generator=gen)
    elif dist == "int4":
        tmp = t.randint(-4, 5, tensor.shape, generator=gen, device=tensor.device,
                        dtype=t.int32).to(t.float32)
    else:
        raise ValueError(dist)
    if tensor.dtype == t.float8_e4m3fn:
        tensor.copy_(tmp.clamp_(-FP8_E4M3_MAX, FP8_E4M3_MAX).to(t.float8_e4m3fn))
    else:
        tensor.copy_(tmp)
