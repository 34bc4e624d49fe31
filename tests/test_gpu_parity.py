"""GPU parity of the Stream-K library against the CPU oracle, through the C ABI.

Integer-valued inputs (entries in {-4..4}) make every partial sum exact in
FP32 and FP64, so results must match the oracle bit for bit for every
schedule, grid and operand layout (the oracle's exact value rounded once to
the output type).  Real-valued inputs must meet the normwise bound
||C - Cref||_F / (||A||_F ||B||_F) <= 1e-13 (FP64) or 5e-5 (FP32
accumulation), measured against the oracle on the stored (rounded or
dequantised) inputs.  Traces of the executed segments must equal the
schedule oracle's segment lists, and reruns must be bitwise identical.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import (bound_for, c_bits, c_values, compare_trace, dev, expected_bits,
                            rel_err, run_gemm, say)

pytestmark = pytest.mark.gpu

PAIRS = [("f64", "f64"), ("f16", "f32"), ("f16", "f16"), ("bf16", "bf16"), ("bf16", "f32"),
         ("f8e4m3", "bf16"), ("f8e4m3", "f32")]
SMALL_TILE = {"f64": (64, 64, 16), "f16": (128, 128, 64), "bf16": (128, 128, 64),
              "f8e4m3": (128, 128, 128)}
BIG_TILE = {"f64": (128, 128, 16), "f16": (256, 256, 64), "bf16": (256, 256, 64),
            "f8e4m3": (256, 256, 128)}
# the third tile of the 16-bit and FP8 types (FP64's small tile is 64x64)
TINY_TILE = {"f16": (64, 64, 64), "bf16": (64, 64, 64), "f8e4m3": (64, 64, 128)}


@pytest.fixture(scope="module")
def ws():
    return R.Workspace("cuda")


def operands(m, n, k, dtype, seed, dist, a_order="row", b_order="row", scale=None):
    if dtype == "f8e4m3" and dist == "int4":
        scale = 1.0
    A, B = W.gemm_operands(m, n, k, dtype, seed, dist, a_order, b_order, fp8_scale=scale)
    return A, B


def check_case(m, n, k, ab, ct, *, dist, seed=0, a_order="row", b_order="row", c_order="row",
               cfg=None, alpha=1.0, beta=0.0, ws=None, trace=True):
    say(f"case m={m} n={n} k={k} {ab}->{ct} {a_order}/{b_order}/{c_order} {dist} "
        f"alpha={alpha} beta={beta} sched={cfg.sched if cfg else 0} grid={cfg.grid if cfg else 0}")
    A, B = operands(m, n, k, ab, seed, dist, a_order, b_order)
    C0 = None
    Cop = None
    if beta != 0.0:
        rng = np.random.default_rng(seed + 99)
        C0 = W.small_integers((m, n), rng) if dist == "int4" else W.uniform((m, n), rng)
        Cop = W.store(C0, ct, c_order)
        C0 = oracle.decode_operand(Cop)          # the exact stored C values
    Ct, plan, tr = run_gemm(m, n, k, dev(A), dev(B), c_type=ct, c_order=c_order, C0=C0, alpha=alpha,
                            beta=beta, cfg=cfg, ws=ws, trace_cap=16384 if trace else 0)
    cref = oracle.gemm(m, n, k, A, B, Cop, alpha=alpha, beta=beta, c_type=ct)
    if dist == "int4":
        got = c_bits(Ct, m, n, c_order)
        want = expected_bits(cref, ct)
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[0]}: " \
                              f"{c_values(Ct, m, n, c_order)[tuple(bad[0])]} vs {cref[tuple(bad[0])]}"
    else:
        Ad, Bd = oracle.decode_operand(A), oracle.decode_operand(B)
        err = rel_err(c_values(Ct, m, n, c_order), cref, Ad, Bd)
        bound = bound_for(ab, ct, cref, Ad, Bd)
        say(f"  rel err {err:.3e} (bound {bound:.3e})")
        assert err <= bound
    if tr is not None:
        compare_trace(tr, plan, [(m, n, k)], c_order, acc_bytes=8 if ab == "f64" else 4,
                      static_dp=bool(cfg is not None and cfg.flags & S.SK_FLAG_STATIC_DP_TILES))
    return Ct, plan


# ---------------------------------------------------------------- config 1

CFG1 = (384, 384, 1024)


@pytest.mark.parametrize("grid", [9, 16, 64, 256, 0])
@pytest.mark.parametrize("dist", ["int4", "uniform"])
def test_config1_fp64_streamk_grids(grid, dist, ws):
    m, n, k = CFG1
    cfg = S.make_config(sched="sk", blk=(128, 128, 16), grid=grid)
    Ct, plan = check_case(m, n, k, "f64", "f64", dist=dist, cfg=cfg, ws=ws)
    assert plan.tiles == 9 and plan.iters_total == 576
    if grid:
        assert plan.grid == grid
    # reruns are bitwise identical (fixed fixup order)
    cfg2 = S.make_config(sched="sk", blk=(128, 128, 16), grid=grid)
    Ct2, _ = check_case(m, n, k, "f64", "f64", dist=dist, cfg=cfg2, ws=ws, trace=False)
    assert torch.equal(Ct.view(torch.int64), Ct2.view(torch.int64))


def test_streamk_with_g_equal_tiles_is_data_parallel(ws):
    m, n, k = CFG1
    A, B = operands(m, n, k, "f64", 0, "uniform")
    outs = []
    for cfg in (S.make_config(sched="sk", blk=(128, 128, 16), grid=9),
                S.make_config(sched="dp", blk=(128, 128, 16))):
        Ct, plan, _ = run_gemm(m, n, k, dev(A), dev(B), c_type="f64", cfg=cfg, ws=ws)
        outs.append(Ct.view(torch.int64).cpu())
    assert torch.equal(outs[0], outs[1])


# ---------------------------------------------------------------- dtypes x layouts x schedules

RAGGED = (208, 336, 400)     # not multiples of any tile; multiples of 16


@pytest.mark.parametrize("ab,ct", PAIRS)
@pytest.mark.parametrize("layout", ["row/row/row", "col/row/row", "row/col/row", "col/col/col",
                                    "row/row/col"])
@pytest.mark.parametrize("sched", ["dp", "sk"])
def test_dtypes_layouts_integer_exact(ab, ct, layout, sched, ws):
    ao, bo, co = layout.split("/")
    m, n, k = RAGGED
    for blk in (SMALL_TILE[ab], BIG_TILE[ab]) + ((TINY_TILE[ab],) if ab in TINY_TILE else ()):
        cfg = S.make_config(sched=sched, blk=blk, grid=0 if sched == "dp" else 7)
        check_case(m, n, k, ab, ct, dist="int4", a_order=ao, b_order=bo, c_order=co, cfg=cfg, ws=ws)


@pytest.mark.parametrize("ab,ct", PAIRS)
def test_dtypes_real_valued_bound(ab, ct, ws):
    m, n, k = RAGGED
    dist = "uniform" if ab in ("f64", "f16") else "normal"
    for sched in ("dp", "sk", "auto"):
        cfg = S.make_config(sched=sched, blk=SMALL_TILE[ab])
        check_case(m, n, k, ab, ct, dist=dist, cfg=cfg, ws=ws, seed=5)
    if ab in TINY_TILE:
        for sched in ("dp", "sk"):
            cfg = S.make_config(sched=sched, blk=TINY_TILE[ab])
            check_case(m, n, k, ab, ct, dist=dist, cfg=cfg, ws=ws, seed=5)


@pytest.mark.parametrize("ab,ct", [("f64", "f64"), ("bf16", "f32"), ("f16", "f16"), ("f8e4m3", "bf16")])
def test_alpha_beta_integer_exact(ab, ct, ws):
    m, n, k = 144, 272, 256
    for c_order in ("row", "col"):
        cfg = S.make_config(sched="sk", blk=SMALL_TILE[ab], grid=5)
        check_case(m, n, k, ab, ct, dist="int4", alpha=2.0, beta=-1.0, c_order=c_order, cfg=cfg,
                   ws=ws)


@pytest.mark.parametrize("sched", ["2tsk", "dp1sk", "auto"])
@pytest.mark.parametrize("slots", [4, 8, 13])
def test_hybrids_on_few_slots(sched, slots, ws):
    # wg_slots below the machine's capacity exercises full DP waves plus a
    # Stream-K region on a small problem (t = 5 x 7 = 35 tiles of 64 x 64)
    m, n, k = 320, 448, 320
    cfg = S.make_config(sched=sched, blk=(64, 64, 16), wg_slots=slots)
    check_case(m, n, k, "f64", "f64", dist="int4", cfg=cfg, ws=ws)
    cfg = S.make_config(sched=sched, blk=(128, 128, 64), wg_slots=slots)
    check_case(720, 1040, 512, "bf16", "f32", dist="int4", cfg=cfg, ws=ws)


@pytest.mark.parametrize("ab,m,n,k,blk_m,sched", [
    ("bf16", 1024, 1024, 2048, 64, S.SK_SCHED_FIXED_SPLIT),     # 256 64x64 tiles, 32 iterations each
    ("bf16", 192, 192, 8192, 64, S.SK_SCHED_SK),                # 9 64x64 tiles: the model's grid
    ("bf16", 2048, 1664, 2048, 128, S.SK_SCHED_FIXED_SPLIT),    # k-aligned split: 2 workgroups per tile
    ("f8e4m3", 2048, 1664, 4096, 128, S.SK_SCHED_FIXED_SPLIT),  # the same with FP8's 128x128x128 tile
    ("bf16", 1024, 1024, 127 * 64, 128, S.SK_SCHED_FIXED_SPLIT),  # I = 127: 8 pieces of 16, the last 15
    ("bf16", 4096, 4352, 2048, 256, S.SK_SCHED_DP_1TILE_SK),    # 272 256x256 tiles: 256 DP + 16 split
    ("bf16", 4096, 2560, 2048, 256, S.SK_SCHED_DP),             # 160 256x256 tiles, one wave
    ("bf16", 2048, 4096, 3072, 256, S.SK_SCHED_SK)])            # 128 256x256 tiles: Stream-K
def test_default_schedule_refinements(ab, m, n, k, blk_m, sched, ws):
    # the default configuration's measured refinements of the schedule, on
    # the machine's own slot counts
    _, plan = check_case(m, n, k, ab, "f32", dist="int4", ws=ws)
    assert (plan.blk_m, plan.sched) == (blk_m, sched), (plan.blk_m, plan.sched, plan.grid)
    if sched == S.SK_SCHED_FIXED_SPLIT:
        assert plan.grid == plan.split * plan.tiles and plan.max_peers == plan.split - 1
    if sched == S.SK_SCHED_DP_1TILE_SK:
        assert plan.dp_tiles == plan.grid and plan.sk_tile_end - plan.sk_tile_begin == plan.tiles - plan.grid


@pytest.mark.parametrize("ab,ct,m,n,k,blk,slots,split", [
    ("f64", "f64", 320, 448, 320, (64, 64, 16), 8, 2),          # 35 tiles: 32 DP + 3 tail, pieces of 10
    ("bf16", "f32", 720, 1040, 512, (128, 128, 64), 16, 2),     # 54 tiles: 48 DP + 6 tail
    ("f16", "f16", 720, 1040, 13 * 64, (128, 128, 64), 24, 4),  # 54 = 48 + 6 tail, I = 13: pieces 4,4,4,1
    ("f8e4m3", "f32", 720, 1040, 5 * 128, (128, 128, 128), 24, 3)])  # I = 5: pieces 2, 2, 1
@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_dp1sk_fixed_split_tail(ab, ct, m, n, k, blk, slots, split, fixup, ws):
    # DP + one-tile SK with its tail as a fixed split (Algorithm 4 on the tail
    # tiles): exact, trace = DP waves + the oracle's fixed_split_segments
    cfg = S.make_config(sched="dp1sk", blk=blk, wg_slots=slots, split=split, fixup=fixup)
    _, plan = check_case(m, n, k, ab, ct, dist="int4", cfg=cfg, ws=ws)
    assert plan.sched == S.SK_SCHED_DP_1TILE_SK and plan.split == split and plan.dp_tiles > 0


@pytest.mark.parametrize("m,n,k", [(384, 384, 64), (256, 640, 128)])
def test_dp1sk_region_smaller_than_grid(m, n, k, ws):
    # DP + one-tile SK where the Stream-K region has fewer iterations than the
    # grid (9 tiles / 1 iteration, 10 tiles / 2 iterations on 8 slots): the
    # grid stays 8 for the DP wave and some workgroups get no SK work
    cfg = S.make_config(sched="dp1sk", blk=(128, 128, 64), wg_slots=8)
    _, plan = check_case(m, n, k, "bf16", "f32", dist="int4", cfg=cfg, ws=ws)
    assert plan.grid == 8 and plan.sk_iters < plan.grid


def test_xcd_remap_off_same_bits(ws):
    m, n, k = 512, 512, 2048
    A, B = operands(m, n, k, "bf16", 3, "normal")
    outs = []
    for flags in (0, S.SK_FLAG_NO_XCD_REMAP):
        cfg = S.make_config(sched="sk", blk=(128, 128, 64), grid=64, flags=flags)
        Ct, _, _ = run_gemm(m, n, k, dev(A), dev(B), c_type="f32", cfg=cfg, ws=ws)
        outs.append(Ct.view(torch.int32).cpu())
    # same logical schedule and order: identical results
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("sched,grid", [("dp", 0), ("sk", 96), ("auto", 0)])
def test_tile_raster_orders(sched, grid, ws):
    # banded (default) and row-major tile rasters, with and without the XCD
    # remap, over 11 x 13 tiles (ragged in both dimensions, not a multiple of
    # the band): integer-valued data makes every order exact against the oracle
    m, n, k = 11 * 128 - 40, 13 * 128 - 24, 1024
    for flags in (0, S.SK_FLAG_ROW_MAJOR_TILES, S.SK_FLAG_NO_XCD_REMAP,
                  S.SK_FLAG_NO_XCD_REMAP | S.SK_FLAG_ROW_MAJOR_TILES):
        cfg = S.make_config(sched=sched, blk=(128, 128, 64), grid=grid, flags=flags)
        check_case(m, n, k, "bf16", "f32", dist="int4", seed=5, cfg=cfg, ws=ws, trace=False)


def test_k_zero_and_alpha_zero_scale_c(ws):
    m, n = 100, 64
    rng = np.random.default_rng(1)
    C0 = W.small_integers((m, n), rng)
    for k, alpha in ((0, 1.0), (64, 0.0)):
        A, B = operands(m, n, max(k, 1) if k else 16, "bf16", 1, "int4")
        Ct, _, _ = run_gemm(m, n, k, dev(A), dev(B), c_type="f32", C0=C0, alpha=alpha, beta=-2.0, ws=ws)
        assert np.array_equal(c_values(Ct, m, n, "row"), -2.0 * C0)
        Ct, _, _ = run_gemm(m, n, k, dev(A), dev(B), c_type="bf16", C0=C0, alpha=alpha, beta=0.0, ws=ws)
        assert np.array_equal(c_values(Ct, m, n, "row"), np.zeros((m, n)))


def test_single_tile_deep_k_strong_scaling(ws):
    # one output tile, k split over many workgroups (section 4; Fig. 8 shape family)
    m, n, k = 128, 128, 16384
    for ab, ct in (("bf16", "f32"), ("f64", "f64")):
        cfg = S.make_config(sched="sk", blk=SMALL_TILE[ab] if ab == "f64" else (128, 128, 64), grid=8)
        check_case(m, n, k, ab, ct, dist="int4", cfg=cfg, ws=ws)
        cfg = S.make_config(sched="sk", blk=(64, 64, 16) if ab == "f64" else (128, 128, 64), grid=0)
        check_case(m, n, k, ab, ct, dist="normal", cfg=cfg, ws=ws, seed=2)


@pytest.mark.skip(reason="its first run (FP64 128x128x16384, one tile, grid 256: the owner waits for "
                         "255 peers) left the GPU faulted; no cause has been shown, so the case stays off "
                         "the GPU, and the planner now refuses owners with more than SK_MAX_PEERS peers")
@pytest.mark.parametrize("ab,ct,blk,k,grid", [("f64", "f64", (128, 128, 16), 16384, 256),
                                               ("f16", "f32", (128, 128, 64), 8192, 128)])
def test_owner_with_more_than_64_peers(ab, ct, blk, k, grid, ws):
    # one output tile split over the whole grid: its owner waits for grid-1
    # peers, more than one 64-lane polling round, and adds them all in order
    cfg = S.make_config(sched="sk", blk=blk, grid=grid)
    Ct, plan = check_case(128, 128, k, ab, ct, dist="int4", cfg=cfg, ws=ws)
    assert plan.tiles == 1 and plan.grid == grid
    Ct2, _ = check_case(128, 128, k, ab, ct, dist="uniform", cfg=cfg, ws=ws, trace=False)


@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_single_tile_at_the_peer_bound(fixup, ws):
    # one FP64 tile whose model grid is limited by SK_MAX_PEERS: the owner (or
    # every contributor) waits on up to 64 others, one full polling round
    cfg = S.make_config(sched="sk", blk=(128, 128, 16), grid=65, fixup=fixup)
    Ct, plan = check_case(128, 128, 16384, "f64", "f64", dist="int4", cfg=cfg, ws=ws)
    assert plan.tiles == 1 and plan.grid == 65 and plan.max_peers == 64


def test_workspace_state_after_calls(ws):
    # flags are raised with the call's epoch and never cleared; every
    # Stream-K launch advances the generation once and leaves the done
    # counter at zero, so the workspace is ready for the next call
    from tests.gpu_util import ws_header
    m, n, k = CFG1
    cfg = S.make_config(sched="sk", blk=(128, 128, 16), grid=60)
    check_case(m, n, k, "f64", "f64", dist="int4", cfg=cfg, ws=ws, trace=False)
    torch.cuda.synchronize()
    err, gen0, done = ws_header(ws)
    assert err == 0 and done == 0
    for i in range(3):
        check_case(m, n, k, "f64", "f64", dist="int4", cfg=cfg, ws=ws, trace=False)
        torch.cuda.synchronize()
        err, gen, done = ws_header(ws)
        assert (err, gen, done) == (0, gen0 + i + 1, 0)
    # only flags hold non-zero words in the flag region, and only epochs
    flags = ws.buf[256:256 + 2 * S.SK_MAX_GRID * 64].view(torch.int32).cpu().view(-1, 16)
    assert int(flags[:, 1:].abs().sum()) == 0
    assert int(flags[:, 0].max()) <= gen0 + 3
