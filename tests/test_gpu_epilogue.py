"""GPU checks of the C store paths through the C ABI, against the CPU oracle.

Tiles with no partial sums to add write C in whole rows through the LDS when
C's rows are 16-byte aligned (16-bit inputs, 128x128 and 256x256 tiles); the
other tiles, and every tile of a C whose rows are not 16-byte aligned, store
from the MFMA layout.  A row ending inside the last 16-byte chunk (n not a
multiple of 4 with a padded leading dimension) and rows past m must be left
alone: integer inputs give exact products, so C[:, :n] must match the
oracle bit for bit and the padding columns must keep their sentinel.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import expected_bits, say

pytestmark = pytest.mark.gpu

M, N, K = 300, 333, 192          # edge tiles in both dimensions; n % 4 == 1


@pytest.mark.parametrize("ab", ["f16", "bf16"])
@pytest.mark.parametrize("ct", ["f32", "same"])
@pytest.mark.parametrize("blk", [(128, 128, 64), (256, 256, 64)])
@pytest.mark.parametrize("ldc", [336, 333])     # rows 16-byte aligned / not
@pytest.mark.parametrize("beta", [0.0, 2.0])
def test_store_paths_edges_and_padding(ab, ct, blk, ldc, beta):
    ct = ab if ct == "same" else ct
    say(f"epilogue {ab}->{ct} blk={blk[0]} ldc={ldc} beta={beta}")
    # B column-major: its leading dimension is k, which keeps its rows 16-byte aligned
    A, B = W.gemm_operands(M, N, K, ab, 3, "int4", "row", "col")
    Ad, Bd = A.to("cuda"), B.to("cuda")
    Cop = None
    C = torch.full((M, ldc), float("nan"), dtype=W.torch_dtype(ct), device="cuda")
    if beta != 0.0:
        C0 = W.small_integers((M, N), np.random.default_rng(7))
        Cop = W.store(C0, ct, "row")
        C[:, :N] = torch.from_numpy(oracle.decode_operand(Cop)).to(C.dtype).to("cuda")
    d = S.make_desc(M, N, K, Ad.tensor, Bd.tensor, C, ab_type=ab, c_type=ct, b_order="col", ldc=ldc, beta=beta,
                    a_scale=A.scale, b_scale=B.scale)
    ws = R.Workspace("cuda")
    for sched in ("dp", "sk"):
        if beta == 0.0:
            C[:, :N] = float("nan")
        elif sched == "sk":
            C[:, :N] = torch.from_numpy(oracle.decode_operand(Cop)).to(C.dtype).to("cuda")
        cfg = S.make_config(sched=sched, blk=blk, grid=0 if sched == "dp" else 5)
        st, plan = S.sk_plan(d, cfg)
        S.check(st, "sk_plan")
        ws.ensure(plan.workspace_bytes)
        S.check(S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, torch.cuda.current_stream().cuda_stream), "sk_gemm")
        torch.cuda.synchronize()
        ws.check()
        cref = oracle.gemm(M, N, K, A, B, Cop, alpha=1.0, beta=beta, c_type=ct)
        want = expected_bits(cref, ct)
        h = C.cpu()
        bits = (h.view(torch.int32) if ct == "f32" else h.view(torch.int16)).numpy()   # FP32 / 16-bit C
        got = bits[:, :N].view(want.dtype)
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{sched}: {len(bad)} mismatches, first at {bad[0]}"
        assert torch.isnan(h[:, N:].float()).all(), f"{sched}: padding columns written"
