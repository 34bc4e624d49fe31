"""GPU checks of sk_gemm_noalloc, the entry point that allocates nothing.

It runs the same plan and kernels as sk_gemm, with the library's fixed
per-device scratch array as its workspace, so its results must equal
sk_gemm's bit for bit on the same inputs (and the oracle's exactly on
integer-valued inputs).  Two calls in a row, the second smaller, show that
the shared array carries nothing from one call into the next; a plan whose
workspace exceeds the array is refused before anything is enqueued; a fixup
wait forced to give up is reported through the caller's error word, and the
next call is correct again.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import c_bits, c_tensor, dev, expected_bits, say
from tests.test_gpu_parity import operands

pytestmark = pytest.mark.gpu


def _gemm(entry, m, n, k, A, B, ab, ct, cfg, ws=None, err=None):
    Ct, ldc = c_tensor(m, n, ct, "row")
    d = S.make_desc(m, n, k, A.tensor, B.tensor, Ct, ab_type=ab, c_type=ct,
                    a_order=A.order, b_order=B.order, lda=A.ld, ldb=B.ld, ldc=ldc,
                    a_scale=A.scale, b_scale=B.scale)
    stream = torch.cuda.current_stream().cuda_stream
    if entry == "noalloc":
        st = S.sk_gemm_noalloc(d, cfg, err.data_ptr() if err is not None else 0, stream)
    else:
        ws.ensure(S.sk_workspace_size(d, cfg)[1])
        st = S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, stream)
    S.check(st, entry)
    torch.cuda.synchronize()
    return Ct


@pytest.mark.parametrize("ab,ct,blk,fixup", [("bf16", "f32", (128, 128, 64), "spread"),
                                              ("f64", "f64", (128, 128, 16), "serial"),
                                              ("f8e4m3", "bf16", (128, 128, 128), "spread")])
def test_noalloc_equals_sk_gemm_two_calls(ab, ct, blk, fixup):
    ws = R.Workspace("cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    # the second call is smaller (fewer tiles, fewer workgroups, fewer peers)
    for (m, n, k, grid, dist) in ((5 * blk[0] - 24, 3 * blk[1] + 48, 24 * blk[2] + 16, 37, "int4"),
                                  (2 * blk[0] - 8, blk[1] + 16, 9 * blk[2], 11, "int4"),
                                  (3 * blk[0] + 8, 2 * blk[1] - 48, 17 * blk[2] + 32, 29, "normal")):
        say(f"noalloc {ab}->{ct} {m}x{n}x{k} grid={grid} fixup={fixup} {dist}")
        A, B = operands(m, n, k, ab, 11, dist)
        Ad, Bd = dev(A), dev(B)
        cfg = S.make_config(sched="sk", blk=blk, grid=grid, fixup=fixup)
        st, plan = S.sk_plan(S.make_desc(m, n, k, 16, 16, 16, ab_type=ab, c_type=ct), cfg)
        S.check(st, "plan")
        assert plan.max_peers >= 1 and plan.workspace_bytes <= S.SK_NOALLOC_SCRATCH_BYTES
        got = c_bits(_gemm("noalloc", m, n, k, Ad, Bd, ab, ct, cfg, err=err), m, n, "row")
        ref = c_bits(_gemm("ws", m, n, k, Ad, Bd, ab, ct, cfg, ws=ws), m, n, "row")
        assert np.array_equal(got, ref)
        assert int(err.item()) == 0
        if dist == "int4":
            cref = oracle.gemm(m, n, k, A, B, None, c_type=ct)
            assert np.array_equal(got, expected_bits(cref, ct))


def test_noalloc_default_config_and_k_zero():
    m, n, k = 520, 264, 1536
    A, B = operands(m, n, k, "bf16", 3, "normal")
    Ad, Bd = dev(A), dev(B)
    ws = R.Workspace("cuda")
    got = c_bits(_gemm("noalloc", m, n, k, Ad, Bd, "bf16", "bf16", None), m, n, "row")
    ref = c_bits(_gemm("ws", m, n, k, Ad, Bd, "bf16", "bf16", None, ws=ws), m, n, "row")
    assert np.array_equal(got, ref)
    # k == 0: C = beta * C with beta = 0 -> zeros, no workspace involved
    got0 = _gemm("noalloc", m, n, 0, Ad, Bd, "bf16", "f32", None)
    assert int(torch.count_nonzero(got0)) == 0


def test_noalloc_refuses_plans_beyond_the_scratch():
    # 256x256 FP32 partial tiles, spread fixup (two slots per workgroup) on
    # 200 workgroups: 100 MiB of partials > the array
    m, n, k = 1024, 1024, 8192
    cfg = S.make_config(sched="sk", blk=(256, 256, 64), grid=200, wg_slots=256, fixup="spread")
    d = S.make_desc(m, n, k, 16, 16, 16, ab_type="bf16", c_type="f32")
    st, need = S.sk_workspace_size(d, cfg)
    assert st == S.SK_OK and need > S.SK_NOALLOC_SCRATCH_BYTES
    C = torch.full((m, n), 7.0, dtype=torch.float32, device="cuda")
    d.C = C.data_ptr()
    st = S.sk_gemm_noalloc(d, cfg, 0, torch.cuda.current_stream().cuda_stream)
    assert st == S.SK_ERR_WORKSPACE_TOO_SMALL
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())          # nothing was launched


def test_noalloc_forced_timeout_is_reported_and_next_call_exact():
    m, n, k = 384, 384, 1024
    A, B = operands(m, n, k, "f64", 0, "int4")
    Ad, Bd = dev(A), dev(B)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    bad = S.make_config(sched="sk", blk=(128, 128, 16), grid=48, fixup="serial", wait_limit_us=-1)
    say("noalloc forced timeout")
    _gemm("noalloc", m, n, k, Ad, Bd, "f64", "f64", bad, err=err)
    assert int(err.item()) == 1
    err.zero_()
    cref = oracle.gemm(m, n, k, A, B, None, c_type="f64")
    for fx in ("serial", "spread"):
        good = S.make_config(sched="sk", blk=(128, 128, 16), grid=48, fixup=fx)
        got = c_bits(_gemm("noalloc", m, n, k, Ad, Bd, "f64", "f64", good, err=err), m, n, "row")
        assert np.array_equal(got, expected_bits(cref, "f64"))
        assert int(err.item()) == 0
