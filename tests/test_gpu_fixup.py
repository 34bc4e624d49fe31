"""GPU checks of the two fixups of split tiles, through the C ABI.

The spread fixup (every contributor reduces a slice of its tile over all
contributors' partial tiles) adds the same values in the same ascending
order as the paper's serial fixup (Algorithm 5: the owner adds its peers'
partials), so the two must give identical bits on real-valued data; both
must match the oracle bit for bit on integer-valued data.  Also here: the
bounded wait forced to give up from the host (every kernel still exits
normally; the call reports SK_ERR_TIMEOUT and the next call on the same
workspace is correct), and a workspace shared by grouped data-parallel and
grouped Stream-K launches.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import (c_bits, c_values, compare_trace, dev, expected_bits, run_gemm, say,
                            ws_header)
from tests.test_gpu_parity import BIG_TILE, PAIRS, SMALL_TILE, check_case, operands

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return R.Workspace("cuda")


@pytest.mark.parametrize("ab,ct", PAIRS)
@pytest.mark.parametrize("big", [False, True])
def test_spread_integer_exact_with_trace(ab, ct, big, ws):
    # several split tiles with many contributors (grid 23 over 6 tiles),
    # ragged edges, both operand contiguities
    blk = BIG_TILE[ab] if big else SMALL_TILE[ab]
    m, n, k = (2 * blk[0] + 48, 3 * blk[1] - 16, 16 * blk[2] + 64)
    for (ao, bo, co) in (("row", "row", "row"), ("col", "col", "col")):
        cfg = S.make_config(sched="sk", blk=blk, grid=23, fixup="spread")
        _, plan = check_case(m, n, k, ab, ct, dist="int4", a_order=ao, b_order=bo, c_order=co, cfg=cfg,
                             ws=ws)
        assert plan.fixup == S.SK_FIXUP_SPREAD and plan.max_peers >= 2


@pytest.mark.parametrize("ab,ct", PAIRS)
@pytest.mark.parametrize("sched,grid,slots", [("sk", 37, 0), ("sk", 0, 0), ("dp1sk", 0, 24), ("2tsk", 0, 8)])
def test_spread_equals_serial_bitwise(ab, ct, sched, grid, slots, ws):
    blk = SMALL_TILE[ab]
    m, n, k = 5 * blk[0] - 24, 3 * blk[1] + 48, 24 * blk[2] + 16
    dist = "uniform" if ab in ("f64", "f16") else "normal"
    A, B = operands(m, n, k, ab, 7, dist)
    bits, plans = [], []
    # the model's grid depends on the fixup (its constants differ), so the
    # serial run takes the grid the spread plan resolved: same segments,
    # same partial sums, same order of additions
    for fx in ("spread", "serial"):
        g = plans[0].grid if plans else grid
        cfg = S.make_config(sched=sched, blk=blk, grid=g, wg_slots=slots, fixup=fx)
        say(f"spread-vs-serial {ab}->{ct} {sched} grid={g} slots={slots} fixup={fx}")
        Ct, plan, _ = run_gemm(m, n, k, dev(A), dev(B), c_type=ct, cfg=cfg, ws=ws)
        bits.append(c_bits(Ct, m, n, "row"))
        plans.append(plan)
    assert [(p.sched, p.grid, p.sk_tile_begin, p.sk_tile_end) for p in plans[:1]] == \
        [(p.sched, p.grid, p.sk_tile_begin, p.sk_tile_end) for p in plans[1:]]
    assert plans[1].fixup == S.SK_FIXUP_SERIAL
    assert np.array_equal(bits[0], bits[1])
    # and within the bound against the oracle
    check_case(m, n, k, ab, ct, dist=dist, seed=7, cfg=S.make_config(sched=sched, blk=blk, grid=grid,
                                                                     wg_slots=slots, fixup="spread"),
               ws=ws)


@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_forced_timeout_reports_and_next_call_is_correct(fixup, ws):
    # wait_limit_us < 0: every fixup wait gives up at once.  The kernels all
    # exit normally; the call reports SK_ERR_TIMEOUT; the next call on the
    # same workspace (normal bound) is exact.
    m, n, k = 384, 384, 1024
    A, B = operands(m, n, k, "f64", 0, "int4")
    bad = S.make_config(sched="sk", blk=(128, 128, 16), grid=48, fixup=fixup, wait_limit_us=-1)
    Ct, ldc = torch.empty((m, n), dtype=torch.float64, device="cuda"), n
    say(f"forced timeout, fixup={fixup}")
    plan = R.gemm(m, n, k, dev(A), dev(B), Ct, c_type="f64", cfg=bad, ws=ws)
    torch.cuda.synchronize()
    st = S.sk_workspace_check(ws.ptr, ws.nbytes, torch.cuda.current_stream().cuda_stream)
    assert st == S.SK_ERR_TIMEOUT
    assert ws_header(ws) == (0, 0, 0)      # the check restored a fresh header
    for _ in range(2):
        good = S.make_config(sched="sk", blk=(128, 128, 16), grid=48, fixup=fixup)
        check_case(m, n, k, "f64", "f64", dist="int4", cfg=good, ws=ws)


def test_grouped_dp_then_sk_on_one_workspace():
    # a grouped data-parallel launch writes its descriptor tables into the
    # workspace; the next grouped Stream-K launch on the same workspace must
    # find its flag region untouched and be exact
    from tests.test_gpu_grouped import SHAPES, check_results, make_batch
    ws = R.Workspace("cuda")
    for sched in ("dp", "sk", "dp", "sk", "sk"):
        say(f"grouped reuse {sched}")
        probs = make_batch(SHAPES, "bf16", "f32", "int4", 10)
        cfg = S.make_config(sched=sched, blk=(128, 128, 64), grid=0 if sched == "dp" else 41)
        plan, raw = R.gemm_grouped([p["d"] for p in probs], cfg=cfg, ws=ws)
        torch.cuda.synchronize()
        ws.check()
        check_results(probs, "bf16", "f32", "int4")
        err, gen, done = ws_header(ws)
        assert err == 0 and done == 0
