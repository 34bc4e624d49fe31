"""GPU checks of the fixed-split generalisation and of the autotuner.

* Section 4: Stream-K with g = s t, where s divides the iterations per tile,
  is the fixed-split schedule of Algorithm 4 -- the executed segments must be
  exactly the oracle's fixed_split_segments, and the results exact.
* The autotuner measures the paper's configuration (one tile per precision,
  the two-tile hybrid, the model's grid) first and returns the fastest
  candidate; that choice must compute the product bit for bit.
"""
import pytest
import torch

from oracle import schedule as O
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from paper_2301_03598_amd import tune as T
from tests.gpu_util import dev, run_gemm, say
from tests.test_gpu_parity import check_case, operands

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return R.Workspace("cuda")


@pytest.mark.parametrize("ab,ct,m,n,k,blk,s", [("f64", "f64", 384, 384, 1024, (128, 128, 16), 4),
                                               ("bf16", "f32", 256, 256, 4096, (128, 128, 64), 8),
                                               ("f16", "f32", 520, 264, 2048, (128, 128, 64), 2)])
@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_streamk_g_st_is_fixed_split(ab, ct, m, n, k, blk, s, fixup, ws):
    geo = O.geometry(m, n, k, *blk)
    assert geo.I % s == 0
    cfg = S.make_config(sched="sk", blk=blk, grid=s * geo.t, fixup=fixup)
    say(f"fixed split {ab} {m}x{n}x{k} t={geo.t} I={geo.I} s={s} fixup={fixup}")
    A, B = operands(m, n, k, ab, 4, "int4")
    Ct, plan, trace = run_gemm(m, n, k, dev(A), dev(B), c_type=ct, cfg=cfg, ws=ws, trace_cap=4096)
    count, recs = trace
    got = {}
    for (wg, seq, tile, k0, k1, role, last, _x) in recs:
        if role != 4:
            got.setdefault(wg, []).append((tile, k0, k1, role, last))
    want = {}
    for lst in O.fixed_split_segments(geo.t, geo.I, s):
        for sg in lst:
            want.setdefault(sg.wg, []).append((sg.tile, sg.k_begin, sg.k_end, sg.role,
                                               sg.peers[-1] if sg.peers else -1))
    assert got == want
    check_case(m, n, k, ab, ct, dist="int4", seed=4, cfg=cfg, ws=ws)


@pytest.mark.parametrize("ab,ct,m,n,k,blk,s", [("bf16", "f32", 256, 384, 100 * 64, (128, 128, 64), 7),
                                               ("bf16", "f32", 256, 384, 100 * 64, (128, 128, 64), 33),
                                               ("f16", "f16", 208, 336, 9 * 64, (128, 128, 64), 4),
                                               ("f64", "f64", 384, 256, 13 * 16, (128, 128, 16), 5),
                                               ("f8e4m3", "f32", 256, 256, 11 * 128, (128, 128, 128), 3)])
@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_fixed_split_schedule(ab, ct, m, n, k, blk, s, fixup, ws):
    # Algorithm 4 as its own schedule: pieces of ceil(I / s) iterations, the
    # last shorter or empty (I = 100, s = 33: 25 non-empty pieces; I = 9,
    # s = 4: the fourth empty); trace = the oracle's fixed_split_segments
    cfg = S.make_config(sched="fs", blk=blk, split=s, fixup=fixup)
    say(f"fixed split schedule {ab} {m}x{n}x{k} s={s} fixup={fixup}")
    _, plan = check_case(m, n, k, ab, ct, dist="int4", seed=6, cfg=cfg, ws=ws)
    geo = O.geometry(m, n, k, *blk)
    assert (plan.sched, plan.split, plan.grid) == (S.SK_SCHED_FIXED_SPLIT, s, s * geo.t)


def test_tuner_choice_is_exact():
    tuner = T.Tuner()
    m, n, k = 384, 640, 2048
    best = tuner.tune("bf16", m, n, k, reps=2)
    entry = tuner.table[T.bucket("bf16", m, n, k)]
    say(f"tuner: best {best} baseline {entry['baseline']} {entry['baseline_us']} us")
    assert entry["baseline_us"] is not None and entry["baseline"]["sched"] == "2tsk"
    assert tuple(entry["baseline"]["blk"]) == T.PAPER_TILE["bf16"]
    assert best.us <= entry["baseline_us"]
    check_case(m, n, k, "bf16", "f32", dist="int4", seed=6, cfg=best.config(), ws=tuner.ws)
