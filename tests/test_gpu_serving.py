"""Continuous-batching server on the GPU: every request completes, requests
are batched into grouped launches on several streams, and each result is the
same computed alone as inside the mix (bit for bit on integer-valued
operands, whose products are exact), and equal to the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import serve as SV
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def int_pool(dtype, n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randint(-4, 5, (n,), generator=g, device="cuda", dtype=torch.int32).to(W.torch_dtype(dtype))


def small_trace(count, rate, seed):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        m, n = (int(rng.integers(1, 9)) * 64 for _ in range(2))
        k = int(rng.integers(1, 17)) * 128
        out.append(W.Request(i, t, m, n, k, "bf16" if rng.uniform() < 0.5 else "f16"))
    return out


def test_serving_alone_equals_mix_and_oracle():
    pools = {"bf16": int_pool("bf16", 1 << 24, 1), "f16": int_pool("f16", 1 << 24, 2)}
    reqs = SV.make_requests(small_trace(400, 50000.0, 3), pools, seed=4)
    srv = SV.Server(pools, hbm_budget=1 << 30, out_bytes=1 << 30, streams=2, max_batch=64)
    say("serving 400 requests")
    st = srv.run(reqs, keep_outputs=True)
    torch.cuda.synchronize()
    say(f"stats {st.completed}/{st.requests} launches {st.launches} mean batch {st.mean_batch:.1f} "
        f"p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms")
    assert st.completed == len(reqs)
    assert st.launches < len(reqs)              # requests were batched
    assert st.mean_batch > 1.0
    assert all(r.done >= r.launched >= r.admitted >= r.arrival for r in reqs)
    ws = R.Workspace("cuda")
    for r in reqs[::37]:
        mix = srv.output(r).clone()
        alone = torch.empty((r.m, r.n), dtype=torch.float32, device="cuda")
        pool = pools[r.dtype]
        eb = pool.element_size()
        d = S.make_desc(r.m, r.n, r.k, pool.data_ptr() + r.a_off * eb, pool.data_ptr() + r.b_off * eb,
                        alone, ab_type=r.dtype, c_type="f32")
        st_, pl = S.sk_plan(d, None)
        ws.ensure(pl.workspace_bytes)
        S.check(S.sk_gemm(d, None, ws.ptr, ws.nbytes, torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert torch.equal(mix.view(torch.int32), alone.view(torch.int32)), f"request {r.rid}"
        # and against the oracle on the exact stored operands
        A = W.Operand(pool[r.a_off:r.a_off + r.m * r.k].cpu(), r.m, r.k, r.dtype, "row", r.k)
        B = W.Operand(pool[r.b_off:r.b_off + r.k * r.n].cpu(), r.k, r.n, r.dtype, "row", r.n)
        cref = oracle.gemm(r.m, r.n, r.k, A, B, c_type="f32")
        assert np.array_equal(alone.cpu().double().numpy(), cref)


def test_admission_respects_budget():
    pools = {"bf16": int_pool("bf16", 1 << 22, 5)}
    trace = [W.Request(i, 0.0, 512, 512, 1024, "bf16") for i in range(40)]
    reqs = SV.make_requests(trace, pools, seed=6)
    one = reqs[0].nbytes(2, 4)
    srv = SV.Server(pools, hbm_budget=3 * one, out_bytes=1 << 28, streams=2, max_batch=8)
    st = srv.run(reqs)
    assert st.completed == 40
    # never more than three requests admitted at once
    events = sorted([(r.admitted, 1) for r in reqs] + [(r.done, -1) for r in reqs])
    live = peak = 0
    for _, dlt in events:
        live += dlt
        peak = max(peak, live)
    assert peak <= 3


def test_serving_mixed_tiles_share_slots_per_kernel():
    # batches of small requests (64x64 tiles) and of large ones (128x128 or
    # 256x256 tiles) in flight together on two streams: each launch is planned
    # on its own kernel's share of the resident slots, so no fixup wait runs
    # into its bound (the run raises SkError(SK_ERR_TIMEOUT) if one does) and
    # every result equals the same GEMM computed alone
    pools = {"bf16": int_pool("bf16", 1 << 25, 7)}
    rng = np.random.default_rng(8)
    trace, t = [], 0.0
    for i in range(240):
        t += rng.exponential(1.0 / 40000.0)
        if i % 6 == 5:
            m, n, k = int(rng.integers(8, 17)) * 128, int(rng.integers(8, 17)) * 128, int(rng.integers(8, 33)) * 128
        else:
            m, n, k = int(rng.integers(1, 9)) * 64, int(rng.integers(1, 9)) * 64, int(rng.integers(2, 33)) * 128
        trace.append(W.Request(i, t, m, n, k, "bf16"))
    reqs = SV.make_requests(trace, pools, seed=9)
    srv = SV.Server(pools, hbm_budget=4 << 30, out_bytes=2 << 30, streams=2, max_batch=16,
                    max_batch_flops=2e10)
    say("serving 240 mixed requests")
    st = srv.run(reqs, keep_outputs=True)
    torch.cuda.synchronize()
    assert st.completed == len(reqs)
    assert len(srv.slots) >= 2, srv.slots          # launches on more than one kernel
    ws = R.Workspace("cuda")
    for r in reqs[::11]:
        mix = srv.output(r).clone()
        alone = torch.empty((r.m, r.n), dtype=torch.float32, device="cuda")
        pool = pools[r.dtype]
        eb = pool.element_size()
        d = S.make_desc(r.m, r.n, r.k, pool.data_ptr() + r.a_off * eb, pool.data_ptr() + r.b_off * eb,
                        alone, ab_type=r.dtype, c_type="f32")
        st_, pl = S.sk_plan(d, None)
        ws.ensure(pl.workspace_bytes)
        S.check(S.sk_gemm(d, None, ws.ptr, ws.nbytes, torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert torch.equal(mix.view(torch.int32), alone.view(torch.int32)), f"request {r.rid}"
