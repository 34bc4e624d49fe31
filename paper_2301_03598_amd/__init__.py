"""Stream-K GEMM for AMD MI355X (gfx950).

``streamk`` is the ctypes binding of the C ABI in include/streamk.h;
``runtime`` adds device workspaces and torch-tensor marshalling.  All GEMM
work runs in the HIP library libstreamk.so built from ``csrc/``.
"""
from . import streamk  # noqa: F401

__all__ = ["streamk"]
