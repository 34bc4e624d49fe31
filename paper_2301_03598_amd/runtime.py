"""Device-side conveniences over the C ABI: a zero-initialised workspace
that grows on demand and calls that take torch tensors.  torch supplies
device memory and streams only; the GEMM runs in libstreamk.so."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import streamk as S


class Workspace:
    """Zero-filled device bytes for one call in flight at a time.  The
    library raises its flags with a per-call epoch and never needs them
    cleared, so a completed call leaves the workspace ready for the next."""

    def __init__(self, device="cuda", nbytes: int = 0):
        self.device = torch.device(device)
        self.buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def ensure(self, nbytes: int) -> None:
        if nbytes > self.buf.numel():
            self.buf = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
            # the zero fill runs on the current stream; a launch on another
            # stream must not see the buffer before it is clear
            torch.cuda.current_stream(self.device).synchronize()

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    @property
    def nbytes(self) -> int:
        return self.buf.numel()

    def check(self, stream: Optional[int] = None) -> None:
        s = torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream
        S.check(S.sk_workspace_check(self.ptr, self.nbytes, s), "sk_workspace_check")


def stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def operand_desc_fields(op):
    """(pointer, order, ld, dtype, scale) of a workloads.Operand-like object."""
    return op.tensor, op.order, op.ld, op.dtype, op.scale


def gemm(m: int, n: int, k: int, A, B, C: torch.Tensor, *, c_type: str, c_order: str = "row",
         ldc: int = 0, alpha: float = 1.0, beta: float = 0.0, cfg: Optional[S.sk_config_t] = None,
         ws: Optional[Workspace] = None, stream=None) -> S.sk_plan_t:
    """C = alpha*A*B + beta*C through sk_gemm.  A and B are Operand-like
    (tensor, order, ld, dtype, scale) already on the device."""
    d = S.make_desc(m, n, k, A.tensor, B.tensor, C, ab_type=A.dtype, c_type=c_type,
                    a_order=A.order, b_order=B.order, c_order=c_order,
                    lda=A.ld, ldb=B.ld, ldc=ldc, alpha=alpha, beta=beta,
                    a_scale=A.scale, b_scale=B.scale)
    st, plan = S.sk_plan(d, cfg)
    S.check(st, "sk_plan")
    if ws is None:
        ws = Workspace(C.device)
    ws.ensure(plan.workspace_bytes)
    S.check(S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, stream_ptr(stream)), "sk_gemm")
    return plan


def gemm_grouped(descs: Sequence[S.sk_gemm_desc_t], *, cfg: Optional[S.sk_config_t] = None,
                 ws: Optional[Workspace] = None, stream=None, device="cuda"):
    """All descriptors in one persistent launch through sk_gemm_grouped.
    The descriptor array lives in pinned host memory owned by the returned
    handle, which must outlive the launch."""
    n = len(descs)
    raw = torch.empty(n * __import__("ctypes").sizeof(S.sk_gemm_desc_t), dtype=torch.uint8,
                      pin_memory=True)
    arr = (S.sk_gemm_desc_t * n).from_address(raw.data_ptr())
    for i, d in enumerate(descs):
        arr[i] = d
    st, plan = S.sk_plan(arr, cfg)
    S.check(st, "sk_plan")
    if ws is None:
        ws = Workspace(device)
    ws.ensure(plan.workspace_bytes)
    S.check(S.sk_gemm_grouped((raw.data_ptr(), n), cfg, ws.ptr, ws.nbytes, stream_ptr(stream)),
            "sk_gemm_grouped")
    return plan, raw


def read_trace(buf: torch.Tensor):
    """Decode a segment trace buffer: list of (wg, seq, tile, k0, k1, role, last, x)."""
    host = buf.cpu()
    count = int(host[0])
    cap = (host.numel() - 8) // 8
    recs = host[8:8 + 8 * min(count, cap)].view(-1, 8).tolist()
    return count, [tuple(r) for r in recs]
