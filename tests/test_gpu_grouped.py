"""GPU parity of the grouped Stream-K launch (sk_gemm_grouped) against the
CPU oracle: many uneven GEMMs in one persistent launch whose iteration space
is the concatenation of the problems' spaces.

Integer-valued inputs give exact products, so every problem's result must
match the oracle bit for bit whatever the schedule, grid or batch
composition; the segment trace must equal the schedule oracle's; a problem
must give the same bits alone and inside a mix; and a captured HIP graph of
the call must reproduce the eager result on every replay.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import bound_for, compare_trace, expected_bits, rel_err, say

pytestmark = pytest.mark.gpu


def make_batch(shapes, ab, ct, dist, seed, c_order="row"):
    probs = []
    for i, (m, n, k) in enumerate(shapes):
        A, B = W.gemm_operands(m, n, k, ab, seed + i, dist,
                               fp8_scale=1.0 if (ab == "f8e4m3" and dist == "int4") else None)
        Ad, Bd = A.to("cuda"), B.to("cuda")
        C = torch.full((m, n) if c_order == "row" else (n, m), float("nan"),
                       dtype=W.torch_dtype(ct), device="cuda")
        d = S.make_desc(m, n, k, Ad.tensor, Bd.tensor, C, ab_type=ab, c_type=ct, c_order=c_order,
                        a_scale=A.scale, b_scale=B.scale)
        probs.append(dict(m=m, n=n, k=k, A=A, B=B, Ad=Ad, Bd=Bd, C=C, d=d))
    return probs


def result(p, ct, c_order="row"):
    h = p["C"].cpu()
    return h if c_order == "row" else h.t().contiguous()


def check_results(probs, ab, ct, dist, c_order="row"):
    for i, p in enumerate(probs):
        cref = oracle.gemm(p["m"], p["n"], p["k"], p["A"], p["B"], c_type=ct)
        got = result(p, ct, c_order)
        if dist == "int4":
            h = got
            bits = (h.view(torch.int64) if ct == "f64" else
                    h.view(torch.int32) if ct == "f32" else h.view(torch.int16)).numpy()
            want = expected_bits(cref, ct)
            assert np.array_equal(bits.view(want.dtype), want), f"problem {i} {p['m']}x{p['n']}x{p['k']}"
        else:
            Ad, Bd = oracle.decode_operand(p["A"]), oracle.decode_operand(p["B"])
            err = rel_err(got.double().numpy(), cref, Ad, Bd)
            assert err <= bound_for(ab, ct, cref, Ad, Bd), f"problem {i}: {err}"


SHAPES = [(64 * (1 + (7 * i) % 9), 64 * (1 + (5 * i) % 7), 128 * (1 + (3 * i) % 11)) for i in range(23)] + \
         [(0, 64, 128), (192, 0, 256)]          # empty problems are allowed in a batch


@pytest.mark.parametrize("sched,grid,slots,flags", [("sk", 0, 0, 0), ("sk", 37, 0, 0), ("dp", 0, 0, 0),
                                                    ("2tsk", 0, 16, 0), ("dp1sk", 0, 16, 0), ("auto", 0, 0, 0),
                                                    ("2tsk", 0, 16, S.SK_FLAG_STATIC_DP_TILES),
                                                    ("dp1sk", 0, 16, S.SK_FLAG_STATIC_DP_TILES)])
def test_grouped_integer_exact_and_trace(sched, grid, slots, flags):
    say(f"grouped sched={sched} grid={grid} slots={slots} flags={flags}")
    probs = make_batch(SHAPES, "bf16", "f32", "int4", 10)
    tr = torch.zeros(8 + 8 * 8192, dtype=torch.int32, device="cuda")
    cfg = S.make_config(sched=sched, blk=(128, 128, 64), grid=grid, wg_slots=slots, flags=flags,
                        trace_ptr=tr.data_ptr(), trace_capacity=8192)
    ws = R.Workspace("cuda")
    plan, raw = R.gemm_grouped([p["d"] for p in probs], cfg=cfg, ws=ws)
    torch.cuda.synchronize()
    ws.check()
    check_results(probs, "bf16", "f32", "int4")
    compare_trace(R.read_trace(tr), plan, [(p["m"], p["n"], p["k"]) for p in probs],
                  static_dp=bool(flags & S.SK_FLAG_STATIC_DP_TILES))


@pytest.mark.parametrize("sched", ["sk", "dp"])
def test_grouped_64_tile_integer_exact_and_trace(sched):
    # the 64x64 tile the automatic policy gives small batches
    say(f"grouped 64x64 sched={sched}")
    probs = make_batch(SHAPES, "f16", "f32", "int4", 60)
    tr = torch.zeros(8 + 8 * 16384, dtype=torch.int32, device="cuda")
    cfg = S.make_config(sched=sched, blk=(64, 64, 64), grid=0 if sched == "dp" else 97,
                        trace_ptr=tr.data_ptr(), trace_capacity=16384)
    ws = R.Workspace("cuda")
    plan, raw = R.gemm_grouped([p["d"] for p in probs], cfg=cfg, ws=ws)
    torch.cuda.synchronize()
    ws.check()
    check_results(probs, "f16", "f32", "int4")
    compare_trace(R.read_trace(tr), plan, [(p["m"], p["n"], p["k"]) for p in probs])


@pytest.mark.parametrize("ab,ct", [("f64", "f64"), ("f16", "f16"), ("bf16", "bf16"), ("f8e4m3", "f32")])
def test_grouped_dtypes_real_valued(ab, ct):
    shapes = [(m, n, (k + 127) // 128 * 128) for (m, n, k) in SHAPES[:12]]
    probs = make_batch(shapes, ab, ct, "normal", 20)
    ws = R.Workspace("cuda")
    R.gemm_grouped([p["d"] for p in probs], cfg=S.make_config(sched="auto"), ws=ws)
    torch.cuda.synchronize()
    ws.check()
    check_results(probs, ab, ct, "normal")


def test_grouped_col_major_c_integer_exact():
    probs = make_batch(SHAPES[:10], "f16", "f32", "int4", 30, c_order="col")
    ws = R.Workspace("cuda")
    R.gemm_grouped([p["d"] for p in probs], cfg=S.make_config(sched="sk", blk=(128, 128, 64)), ws=ws)
    torch.cuda.synchronize()
    check_results(probs, "f16", "f32", "int4", c_order="col")


def test_alone_and_in_mix_identical():
    probs = make_batch(SHAPES, "bf16", "bf16", "int4", 40)
    ws = R.Workspace("cuda")
    R.gemm_grouped([p["d"] for p in probs], cfg=S.make_config(sched="sk", blk=(128, 128, 64)), ws=ws)
    torch.cuda.synchronize()
    mix = [p["C"].clone() for p in probs]
    for i in (0, 5, 17):
        probs[i]["C"].fill_(float("nan"))
        R.gemm_grouped([probs[i]["d"]], cfg=S.make_config(sched="sk", blk=(128, 128, 64)), ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(probs[i]["C"].view(torch.int16), mix[i].view(torch.int16))


def test_grouped_hipgraph_replays_match_eager():
    probs = make_batch(SHAPES[:16], "bf16", "f32", "normal", 50)
    ws = R.Workspace("cuda")
    cfg = S.make_config(sched="auto")
    st, plan = S.sk_plan((S.sk_gemm_desc_t * 16)(*[p["d"] for p in probs]), cfg)
    S.check(st)
    ws.ensure(plan.workspace_bytes)
    R.gemm_grouped([p["d"] for p in probs], cfg=cfg, ws=ws)
    torch.cuda.synchronize()
    eager = [p["C"].clone() for p in probs]
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    keep = None
    with torch.cuda.graph(g, stream=stream):
        _, keep = R.gemm_grouped([p["d"] for p in probs], cfg=cfg, ws=ws, stream=stream)
    for rep in range(3):
        for p in probs:
            p["C"].fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            assert torch.equal(p["C"].view(torch.int32), eager[i].view(torch.int32)), f"replay {rep} problem {i}"
    del keep


@pytest.mark.parametrize("slots", [16, 32])
def test_grouped_dp_tile_queues_same_bits_and_replays(slots):
    # a persistent two-tile hybrid takes its data-parallel tiles after the
    # first wave from the per-XCD queues: the same bits as the static order,
    # eagerly and on every graph replay (the last workgroup of each launch
    # returns the queue counters to zero)
    probs = make_batch(SHAPES, "bf16", "f32", "normal", 70)
    descs = [p["d"] for p in probs]
    ws = R.Workspace("cuda")
    static = S.make_config(sched="2tsk", blk=(128, 128, 64), wg_slots=slots, flags=S.SK_FLAG_STATIC_DP_TILES)
    R.gemm_grouped(descs, cfg=static, ws=ws)
    torch.cuda.synchronize()
    ws.check()
    ref = [p["C"].clone() for p in probs]
    dyn = S.make_config(sched="2tsk", blk=(128, 128, 64), wg_slots=slots)
    plan, keep0 = R.gemm_grouped(descs, cfg=dyn, ws=ws)
    torch.cuda.synchronize()
    ws.check()
    assert plan.dp_tiles > plan.grid
    for i, p in enumerate(probs):
        assert torch.equal(p["C"].view(torch.int32), ref[i].view(torch.int32)), f"problem {i}"
    del keep0          # its pinned descriptor block is reused inside the capture
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        _, keep = R.gemm_grouped(descs, cfg=dyn, ws=ws, stream=stream)
    for rep in range(3):
        for p in probs:
            p["C"].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            assert torch.equal(p["C"].view(torch.int32), ref[i].view(torch.int32)), f"replay {rep} problem {i}"
    ws.check()
    words = ws.buf[:44].view(torch.int32).cpu().tolist()
    assert words[0] == 0 and words[2] == 0 and words[3:11] == [0] * 8, words
    del keep
