"""Host-side checks of the C ABI (no GPU, no compute calls).

The library must load and export every function include/streamk.h declares;
argument validation must return the documented status before anything is
enqueued; and the C++ planner (sk_plan) must agree with the independent
schedule oracle on the Stream-K region, the grid size and the resolved
schedule.
"""
import ctypes
import os
import re

import pytest
from hypothesis import given, settings, strategies as st

from oracle import schedule as O
from paper_2301_03598_amd import streamk as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "streamk.h")
MODEL = (2.0, 10.0, 1.0, 8.5)


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sk_status_t|const char \*)\s*(sk_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(S.EXPORTS)
    L = S.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_layouts_match_header():
    # compile the C header with the host compiler and compare every struct's
    # size and field offsets with the ctypes binding
    import subprocess
    import tempfile
    structs = {"sk_gemm_desc_t": S.sk_gemm_desc_t, "sk_config_t": S.sk_config_t, "sk_plan_t": S.sk_plan_t}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "streamk.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append('printf("SK_MAX_GRID %d\\nSK_MAX_PEERS %d\\n", SK_MAX_GRID, SK_MAX_PEERS); return 0; }')
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    got = dict(zip(out[0::2], (int(v) for v in out[1::2])))
    for name, cls in structs.items():
        assert got[name] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[f"{name}.{f}"] == getattr(cls, f).offset, f"{name}.{f}"
    assert (got["SK_MAX_GRID"], got["SK_MAX_PEERS"]) == (S.SK_MAX_GRID, S.SK_MAX_PEERS)


def test_status_strings():
    for code in range(7):
        assert S.sk_status_string(code).startswith("SK_")
    assert S.sk_status_string(99) == "SK_ERR_UNKNOWN"


FAKE = 0x10000   # never dereferenced: validation fails or the call is a no-op


def desc(**kw):
    base = dict(m=64, n=64, k=64, A=FAKE, B=FAKE, C=FAKE, ab_type="bf16", c_type="f32")
    base.update(kw)
    return S.make_desc(**base)


@pytest.mark.parametrize("kw,code", [
    (dict(m=-1), S.SK_ERR_INVALID_VALUE),
    (dict(k=-5), S.SK_ERR_INVALID_VALUE),
    (dict(a_order=2), S.SK_ERR_INVALID_VALUE),
    (dict(ab_type="f64", c_type="f32"), S.SK_ERR_UNSUPPORTED),
    (dict(ab_type="bf16", c_type="f16"), S.SK_ERR_UNSUPPORTED),
    (dict(ab_type="f32", c_type="f32"), S.SK_ERR_UNSUPPORTED),
    (dict(ab_type="f8e4m3", c_type="bf16", a_scale=0.0), S.SK_ERR_INVALID_VALUE),
    (dict(ab_type="f8e4m3", c_type="bf16", b_scale=float("inf")), S.SK_ERR_INVALID_VALUE),
    (dict(a_scale=2.0), S.SK_ERR_INVALID_VALUE),
    (dict(lda=32), S.SK_ERR_INVALID_VALUE),            # row-major A needs lda >= k
    (dict(ldc=10), S.SK_ERR_INVALID_VALUE),
    (dict(A=0), S.SK_ERR_INVALID_VALUE),
    (dict(C=0), S.SK_ERR_INVALID_VALUE),
    (dict(A=FAKE + 8), S.SK_ERR_MISALIGNED),           # A not 16-byte aligned
    (dict(k=60), S.SK_ERR_MISALIGNED),                 # k not a multiple of 8 (bf16 rows)
    (dict(ldb=68), S.SK_ERR_MISALIGNED),
    (dict(ab_type="f8e4m3", c_type="f32", a_scale=0.5, b_scale=0.5, k=72), S.SK_ERR_MISALIGNED),
    (dict(C=FAKE + 1, c_type="f32"), S.SK_ERR_MISALIGNED),
])
def test_validation_errors(kw, code):
    d = desc(**kw)
    assert S.sk_gemm(d, None, FAKE, 1 << 20, 0) == code
    st, _ = S.sk_workspace_size(d)
    assert st == code


def test_plan_of_k_zero():
    # k == 0 (C = beta*C): planned without MAC-loop work, for every schedule
    for sched in ("auto", "dp", "sk", "2tsk", "dp1sk"):
        st, pl = S.sk_plan(desc(m=100, n=64, k=0), S.make_config(sched=sched, wg_slots=256))
        assert st == S.SK_OK and pl.iters_total == 0 and pl.grid == 0, sched
        assert S.sk_workspace_size(desc(m=100, n=64, k=0), S.make_config(sched=sched, wg_slots=256))[0] == S.SK_OK


def test_noops_need_no_device():
    # m == 0 or n == 0: nothing to do, no pointers needed
    assert S.sk_gemm(desc(m=0, A=0, B=0, C=0), None, 0, 0, 0) == S.SK_OK
    assert S.sk_gemm(desc(n=0, A=0, B=0, C=0), None, 0, 0, 0) == S.SK_OK


def test_config_errors():
    d = desc()
    assert S.sk_plan(d, S.make_config(sched=9, wg_slots=8))[0] == S.SK_ERR_INVALID_VALUE
    assert S.sk_plan(d, S.make_config(grid=300, wg_slots=256))[0] == S.SK_ERR_INVALID_VALUE
    assert S.sk_plan(d, S.make_config(blk=(96, 96, 64), wg_slots=8))[0] == S.SK_ERR_UNSUPPORTED
    assert S.sk_plan(d, S.make_config(wg_slots=-1))[0] == S.SK_ERR_INVALID_VALUE


def test_workspace_too_small_before_launch():
    d = desc(m=384, n=384, k=1024, ab_type="f64", c_type="f64")
    cfg = S.make_config(sched="sk", grid=64, wg_slots=256)
    st, need = S.sk_workspace_size(d, cfg)
    assert st == S.SK_OK and need > 64 * 128 * 128 * 8
    assert S.sk_gemm(d, cfg, FAKE, need - 1, 0) == S.SK_ERR_WORKSPACE_TOO_SMALL
    assert S.sk_gemm(d, cfg, 0, need, 0) == S.SK_ERR_WORKSPACE_TOO_SMALL


def test_grouped_rejects_mixed_types():
    ds = [desc(), desc(ab_type="f16", c_type="f32")]
    arr = (S.sk_gemm_desc_t * 2)(*ds)
    assert S.sk_gemm_grouped(arr, None, FAKE, 1 << 20, 0) == S.SK_ERR_UNSUPPORTED
    ds = [desc(), desc(k=0)]
    arr = (S.sk_gemm_desc_t * 2)(*ds)
    assert S.sk_gemm_grouped(arr, None, FAKE, 1 << 20, 0) == S.SK_ERR_UNSUPPORTED


def oracle_problems(shapes, blk):
    geos = [O.geometry(m, n, k, *blk) for (m, n, k) in shapes]
    return O.Problems([(g.t if (m > 0 and n > 0) else 0, g.I) for g, (m, n, k) in zip(geos, shapes)])


def oracle_max_peers(probs, op):
    """Largest peer count of any owner in the oracle's schedule."""
    if op.sk_tile_end <= op.sk_tile_begin:
        return 0
    return max((len(sg.peers) for lst in O.segments(probs, op) for sg in lst if sg.role == O.ROLE_OWNER),
               default=0)


def check_plan_agrees(shapes, dtype, blk, p, sched, grid, threshold=0, c_order="row"):
    """The library's plan against the schedule oracle's plan of the same
    schedule.  An automatic schedule is first resolved by the library (its
    policy is the library's, not the paper's) and the resolved schedule is
    planned again by the oracle with the same model constants."""
    ds = [desc(m=m, n=n, k=k, ab_type=dtype, c_type={"f64": "f64", "bf16": "f32", "f16": "f32",
                                                       "f8e4m3": "f32"}[dtype],
               a_scale=0.5 if dtype == "f8e4m3" else 1.0, b_scale=0.5 if dtype == "f8e4m3" else 1.0,
               c_order=c_order)
          for (m, n, k) in shapes]
    sched = S.SCHED[sched] if isinstance(sched, str) else sched
    cfg = S.make_config(sched=sched, blk=blk, grid=grid, wg_slots=p, threshold=threshold, model=MODEL)
    st, pl = S.sk_plan(ds if len(ds) > 1 else ds[0], cfg)
    # a column-major C is computed as C^T = B^T A^T: the tile grid is n x m
    oshapes = [(n, m, k) if c_order == "col" else (m, n, k) for (m, n, k) in shapes]
    probs = oracle_problems(oshapes, blk)
    if sched == S.SK_SCHED_FIXED_SPLIT or (st == S.SK_OK and pl.sched == S.SK_SCHED_FIXED_SPLIT):
        return check_fixed_split_plan(st, pl, probs, p, grid, len(shapes), sched)
    if sched == S.SK_SCHED_AUTO:
        assert st == S.SK_OK, S.sk_status_string(st)
        osched = pl.sched if probs.tiles else S.SK_SCHED_DP
        ogrid = grid
    else:
        osched, ogrid = sched, grid
    op = O.plan_problems(probs, p=p, sched=osched, grid=ogrid, consts=MODEL, threshold=threshold or 2)
    if st == S.SK_OK and pl.sched == S.SK_SCHED_DP_1TILE_SK and pl.split > 0:
        # the automatic hybrid's fixed-split tail: the oracle's region and
        # grid, Algorithm 4 on the tail tiles
        assert sched == S.SK_SCHED_AUTO and len(shapes) == 1
        assert (pl.sk_tile_begin, pl.sk_tile_end, pl.grid, pl.dp_tiles) == \
            (op.sk_tile_begin, op.sk_tile_end, op.g, len(op.dp_tiles))
        r = pl.sk_tile_end - pl.sk_tile_begin
        segs = O.fixed_split_segments(r, probs.Ip[0], pl.split)
        assert 2 <= pl.split <= 16 and pl.split * r <= pl.grid
        assert pl.max_peers == max(len(sg.peers) for lst in segs for sg in lst)
        return pl
    if sched == S.SK_SCHED_AUTO and grid == 0 and pl.sched == S.SK_SCHED_SK and pl.grid != op.g:
        # the library's k-aligned split instead of the model's grid: s
        # workgroups per tile, s dividing the tile's iteration count, filling
        # at least half of the slots; the oracle plans that grid
        s_, t_ = pl.grid // pl.tiles, pl.tiles
        it = probs.total // t_
        assert len(shapes) == 1 and pl.grid == s_ * t_ and s_ >= 2 and it % s_ == 0
        assert s_ * t_ <= p <= 2 * s_ * t_ and s_ <= S.SK_MAX_PEERS + 1
        op = O.plan_problems(probs, p=p, sched=osched, grid=pl.grid, consts=MODEL, threshold=threshold or 2)
    omp = oracle_max_peers(probs, op)
    if omp > S.SK_MAX_PEERS:
        # the paper's plan needs an owner with more peers than the library
        # serves: a caller-fixed grid or hybrid is refused; a model grid is
        # replaced by the best grid within the bound
        if sched != S.SK_SCHED_AUTO and (grid > 0 or op.sched != O.SCHED_SK):
            assert st == S.SK_ERR_UNSUPPORTED, (st, omp)
            return None
        assert st == S.SK_OK, S.sk_status_string(st)
        assert pl.max_peers <= S.SK_MAX_PEERS and pl.grid < op.g
        return pl
    assert st == S.SK_OK, S.sk_status_string(st)
    assert pl.tiles == probs.tiles
    assert pl.iters_total == probs.total
    assert pl.grid == op.g
    assert (pl.sk_tile_begin, pl.sk_tile_end) == (op.sk_tile_begin, op.sk_tile_end) or \
        (pl.sk_tile_end == pl.sk_tile_begin and op.sk_tile_end == op.sk_tile_begin)
    assert pl.dp_tiles == len(op.dp_tiles)
    assert bool(pl.dp_first) == (op.dp_first and op.sk_tile_end > op.sk_tile_begin) or \
        op.sk_tile_end == op.sk_tile_begin or pl.sched == S.SK_SCHED_DP
    if op.sk_tile_end > op.sk_tile_begin:
        assert pl.sk_iters == probs.region_iters(op.sk_tile_begin, op.sk_tile_end)
        assert pl.sk_iter_begin == probs.tile_iter_begin(op.sk_tile_begin)
    assert pl.sched == op.sched
    assert pl.max_peers == omp
    return pl


def check_fixed_split_plan(st, pl, probs, p, grid, count, sched):
    """A fixed-split plan (Algorithm 4) against the oracle's segments: the
    library's automatic factor is the largest s <= SK_MAX_PEERS + 1 with
    s t <= p and no empty piece (s = 1: the data-parallel schedule)."""
    if count != 1:
        assert st == S.SK_ERR_UNSUPPORTED
        return None
    t, I = probs.tiles, probs.Ip[0] if probs.tiles else 0
    if t == 0:
        assert st == S.SK_OK
        return pl
    cands = [s for s in range(2, min(I, S.SK_MAX_PEERS + 1) + 1)
             if s * t <= min(p, S.SK_MAX_GRID) and (s - 1) * O.cdiv(I, s) < I]
    s = max(cands) if cands else 1          # none: s = 1, the data-parallel schedule
    if grid > 0 and grid != s * t:
        assert st == S.SK_ERR_INVALID_VALUE, (st, t, I, p, grid)
        return None
    assert st == S.SK_OK, S.sk_status_string(st)
    if sched == S.SK_SCHED_AUTO:
        s = pl.split                 # the automatic schedule's own choice of s
        assert 2 * s * t >= p and s in cands
    if s == 1:
        assert pl.sched == S.SK_SCHED_DP and pl.grid == t
        return pl
    segs = O.fixed_split_segments(t, I, s)
    O.check_invariants(probs, O.Plan(s * t, 0, t, False, O.SCHED_SK, t, []), segs)
    assert (pl.sched, pl.split, pl.grid, pl.sk_tile_begin, pl.sk_tile_end, pl.dp_tiles) == \
        (S.SK_SCHED_FIXED_SPLIT, s, s * t, 0, t, 0)
    assert pl.sk_iters == probs.total and pl.sk_iter_begin == 0
    assert pl.max_peers == max(len(sg.peers) for lst in segs for sg in lst)
    return pl


def test_plan_config1_model_grid():
    pl = check_plan_agrees([(384, 384, 1024)], "f64", (128, 128, 16), 256, "sk", 0)
    assert pl.tiles == 9 and pl.iters_total == 576


@settings(max_examples=200, deadline=None)
@given(m=st.integers(1, 9000), n=st.integers(1, 9000), k=st.integers(1, 9000),
       dtype=st.sampled_from(["f64", "bf16", "f16", "f8e4m3"]), ti=st.integers(0, 2),
       p=st.sampled_from([8, 64, 256, 512]),
       sched=st.sampled_from(["dp", "sk", "dp1sk", "2tsk", "auto", "fs"]),
       grid=st.integers(0, 64), thr=st.sampled_from([0, 1, 3]),
       c_order=st.sampled_from(["row", "col"]))
def test_plan_matches_schedule_oracle(m, n, k, dtype, ti, p, sched, grid, thr, c_order):
    tiles = {"f64": [(128, 128, 16), (64, 64, 16)],
             "bf16": [(256, 256, 64), (128, 128, 64), (64, 64, 64)],
             "f16": [(256, 256, 64), (128, 128, 64), (64, 64, 64)],
             "f8e4m3": [(256, 256, 128), (128, 128, 128), (64, 64, 128)]}[dtype]
    blk = tiles[ti % len(tiles)]
    grid = min(grid, p)
    m, n, k = (-(-v // 16) * 16 for v in (m, n, k))    # satisfy the 16-byte rule for every dtype
    check_plan_agrees([(m, n, k)], dtype, blk, p, S.SCHED[sched], grid, thr, c_order)


@settings(max_examples=60, deadline=None)
@given(shapes=st.lists(st.tuples(st.integers(0, 700), st.integers(0, 700), st.integers(1, 3000)),
                       min_size=2, max_size=20),
       p=st.sampled_from([16, 256]), sched=st.sampled_from(["sk", "dp", "2tsk", "dp1sk"]),
       grid=st.integers(0, 16))
def test_grouped_plan_matches_schedule_oracle(shapes, p, sched, grid):
    shapes = [(-(-m // 8) * 8, -(-n // 8) * 8, -(-k // 8) * 8) for (m, n, k) in shapes]
    if sum(1 for (m, n, k) in shapes if m > 0 and n > 0) == 0:
        return
    check_plan_agrees(shapes, "bf16", (128, 128, 64), p, S.SCHED[sched], min(grid, p))


def test_auto_tile_and_schedule_policy():
    # FP16/BF16 without a tile: 128x128 unless 2 full waves of it (t >= 2 p);
    # small problems take 64x64 (fewer than 64 such tiles and k <= 8192:
    # Stream-K; at most 3/4 CUs 128x128 tiles and k <= 4096: data-parallel)
    cfg = S.make_config(wg_slots=512)
    # (the schedules of the 256x256 cases are not checked: wg_slots = 512 is
    # the 128x128 kernel's slot count, not the 256x256 one's)
    for (m, n, k, blk_m, sched) in ((8192, 8192, 512, 256, None), (8192, 4096, 512, 256, None),
                                    (4096, 4096, 512, 256, None), (4096, 2048, 512, 128, S.SK_SCHED_DP),
                                    (4096, 4096 - 128, 512, 128, S.SK_SCHED_DP),
                                    (4096 + 128, 4096, 512, 256, None),
                                    (256, 256, 512, 64, None), (512, 448, 2048, 64, S.SK_SCHED_FIXED_SPLIT),
                                    (256, 256, 65536, 128, S.SK_SCHED_FIXED_SPLIT),
                                    (2048, 1536, 4096, 64, S.SK_SCHED_DP),
                                    (2048, 1536, 4104, 128, S.SK_SCHED_FIXED_SPLIT),
                                    (2048, 1536 + 128, 2048, 128, S.SK_SCHED_FIXED_SPLIT),
                                    (4096, 1024, 4096, 128, S.SK_SCHED_FIXED_SPLIT),
                                    (2048, 2048 + 128, 2048, 128, S.SK_SCHED_DP)):
        st, pl = S.sk_plan(desc(m=m, n=n, k=k, ab_type="bf16", c_type="f32"), cfg)
        assert st == S.SK_OK and pl.blk_m == blk_m, (m, n, k, pl.blk_m)
        assert sched is None or pl.sched == sched, (m, n, k, pl.sched)
    # FP8 follows the same rule (t >= 8 p of its 128x128x128 tile -> 256x256x128)
    for (m, n, blk_m) in ((8192, 8192, 256), (8192, 4096, 128), (256, 256, 128)):
        st, pl = S.sk_plan(desc(m=m, n=n, k=512, ab_type="f8e4m3", c_type="bf16", a_scale=0.5, b_scale=0.5), cfg)
        assert st == S.SK_OK and (pl.blk_m, pl.blk_k) == (blk_m, 128), (m, n, pl.blk_m)
    # FP64 keeps its default tile (128x128x16)
    st, pl = S.sk_plan(desc(m=256, n=256, k=512, ab_type="f64", c_type="f64"), cfg)
    assert st == S.SK_OK and (pl.blk_m, pl.blk_k) == (128, 16)
    # AUTO: Stream-K while t <= CUs (= wg_slots / LDS-bound workgroups per CU), else DP; here
    # as the k-aligned fixed split, which fills at least half of the slots in these cases
    blk = (128, 128, 64)
    # (with wg_slots = 512 the 128x128x64 kernel's LDS allows 2 workgroups per CU: 256 CUs)
    for (m, n, k, want) in ((1024, 1024, 8192, S.SK_SCHED_FIXED_SPLIT),
                            (2048, 2048 - 128, 8192, S.SK_SCHED_FIXED_SPLIT),
                            (2048, 2048, 8192, S.SK_SCHED_FIXED_SPLIT), (2048, 2048 + 128, 8192, S.SK_SCHED_DP),
                            (256, 128, 8192, S.SK_SCHED_SK),    # 2 tiles: no split fills half the slots
                            (4096, 4096, 8192, S.SK_SCHED_DP),
                            # shallow k: the model grid is one workgroup per tile, i.e. DP
                            (1024, 1024, 512, S.SK_SCHED_DP), (2048, 2048, 512, S.SK_SCHED_DP)):
        st, pl = S.sk_plan(desc(m=m, n=n, k=k, ab_type="f16", c_type="f32"),
                           S.make_config(blk=blk, wg_slots=512))
        assert st == S.SK_OK and pl.sched == want, (m, n, k, pl.sched)
    # the one-workgroup-per-tile shortcut is for single GEMMs: a grouped call
    # of the same shallow problems keeps basic Stream-K over their union
    d1 = desc(m=1024, n=1024, k=512, ab_type="f16", c_type="f32")
    st, pl = S.sk_plan([d1, d1], S.make_config(blk=blk, wg_slots=512))
    assert st == S.SK_OK and pl.sched == S.SK_SCHED_SK and pl.tiles == 128
    # an explicit grid is honoured as Stream-K even when it equals t
    st, pl = S.sk_plan(d1, S.make_config(blk=blk, wg_slots=512, grid=64))
    assert st == S.SK_OK and pl.sched == S.SK_SCHED_SK and pl.grid == 64


def test_auto_refinements():
    # FP16/BF16 only; measured rules, not the paper's
    cfg = S.make_config(wg_slots=512)

    def plan(m, n, k, dt="bf16", c=cfg):
        st, pl = S.sk_plan(desc(m=m, n=n, k=k, ab_type=dt, c_type="f32" if dt != "f8e4m3" else "bf16",
                                a_scale=0.5 if dt == "f8e4m3" else 1.0, b_scale=0.5 if dt == "f8e4m3" else 1.0), c)
        assert st == S.SK_OK, S.sk_status_string(st)
        return pl
    # 64x64 tile, fewer than 1.5 CUs' worth of tiles: Stream-K from 32
    # k-iterations per tile on, one workgroup per tile below (1280 slots:
    # five 64x64 workgroups per CU by LDS, 256 CUs)
    c64 = S.make_config(wg_slots=1280)
    pl = plan(1024, 1024, 2048, c=c64)                 # as a fixed split filling 5/8 of the slots
    assert (pl.blk_m, pl.tiles, pl.sched, pl.split) == (64, 256, S.SK_SCHED_FIXED_SPLIT, 4) and pl.grid > 256
    pl = plan(1024, 640, 2048, c=c64)                  # 160 tiles: s = 6 (grids stop at SK_MAX_GRID = 1024)
    assert (pl.blk_m, pl.sched, pl.split) == (64, S.SK_SCHED_FIXED_SPLIT, 6)
    pl = plan(192, 192, 8192, c=c64)                   # 9 tiles: 65 x 9 < 5/8 x 1024: the model's grid
    assert (pl.blk_m, pl.sched) == (64, S.SK_SCHED_SK)
    pl = plan(1024, 1024, 1024, c=c64)
    assert (pl.blk_m, pl.sched) == (64, S.SK_SCHED_DP)
    pl = plan(2048, 1536, 4096, c=c64)                 # 768 such tiles: data-parallel
    assert (pl.blk_m, pl.sched) == (64, S.SK_SCHED_DP)
    pl = plan(1280, 1280, 2048, c=c64)                 # 400 >= 384 such tiles: data-parallel
    assert (pl.blk_m, pl.tiles, pl.sched) == (64, 400, S.SK_SCHED_DP)
    # 128x128 Stream-K: k-aligned fixed split, s t <= p <= 2 s t
    for (m, n, k, g) in ((2048, 1664, 2048, 416), (4096, 1024, 4096, 512), (1024, 1024, 8192, 512),
                         (128 * 9, 128 * 20, 8192, 360)):
        pl = plan(m, n, k)
        assert (pl.blk_m, pl.sched, pl.grid) == (128, S.SK_SCHED_FIXED_SPLIT, g), (m, n, k, pl.grid)
        assert pl.split == g // pl.tiles and pl.max_peers == pl.split - 1
    # I = 127 has no divisor that fills half the slots: pieces of 16 (the last 15)
    pl = plan(1024, 1024, 127 * 64)
    assert (pl.sched, pl.split, pl.grid, pl.max_peers) == (S.SK_SCHED_FIXED_SPLIT, 8, 512, 7)
    # few tiles: the model's grid (no s fills enough of the slots); 256x256
    # (16 tiles of 64x64) fills 5/8 of them with s = 32
    pl = plan(128, 128, 8192)
    assert (pl.blk_m, pl.sched) == (64, S.SK_SCHED_SK)
    pl = plan(256, 256, 8192)
    assert (pl.blk_m, pl.sched, pl.split) == (64, S.SK_SCHED_FIXED_SPLIT, 32)
    # FP8's 128x128x128 tile too
    pl = plan(2048, 1664, 4096, dt="f8e4m3")
    assert (pl.blk_m, pl.blk_k, pl.sched, pl.grid) == (128, 128, S.SK_SCHED_FIXED_SPLIT, 416)
    # grouped calls keep the model's grid
    d = desc(m=1024, n=1024, k=8192, ab_type="bf16", c_type="f32")
    st, pl = S.sk_plan([d, d], S.make_config(blk=(128, 128, 64), wg_slots=512))
    assert st == S.SK_OK and pl.sched == S.SK_SCHED_SK
    # deep single GEMMs with between half and all of the CUs' worth of
    # 256x256 tiles keep that tile (here 256 CUs: two 128x128 workgroups per
    # CU in 512 slots); shallow ones and grouped calls keep 128x128
    for (m, n, k, blk_m) in ((4096, 2560, 4096, 256), (2048, 4096, 3072, 256), (4096, 4096, 2048, 256),
                             (4096, 2560, 2048, 256), (2048, 4096, 2048, 128),
                             (2048, 3840, 4096, 128), (4096, 2560, 1024, 128), (2048, 2048, 4096, 128)):
        assert plan(m, n, k).blk_m == blk_m, (m, n, k)
    d = desc(m=4096, n=2560, k=4096, ab_type="bf16", c_type="f32")
    st, pl = S.sk_plan([d, d], cfg)
    assert st == S.SK_OK and pl.blk_m == 256      # 320 tiles of 128x128 per problem: 2 p in all
    st, pl = S.sk_plan([d], cfg)                  # one problem given as a list
    assert st == S.SK_OK and pl.blk_m == 256
    d = desc(m=2048, n=2560, k=4096, ab_type="bf16", c_type="f32")
    st, pl = S.sk_plan([d, d], cfg)               # 2 x 80 256x256 tiles: not a single GEMM
    assert st == S.SK_OK and pl.blk_m == 128
    # 256x256 past a full wave: DP waves + one-tile Stream-K with a
    # fixed-split tail (s <= 16 pieces per tail tile) when the last wave holds
    # at most half of the slots and k has >= 32 iterations per tile
    c256 = S.make_config(wg_slots=256)                 # one 256x256 workgroup per CU
    for (m, n, k, split, peers) in ((4096, 4096 + 256, 4096, 16, 15),   # 272 tiles: 256 + 16
                                    (4096, 256 * 22, 4096, 2, 1),       # 352 tiles: a 96-tile tail
                                    (256 * 257, 256, 4096, 16, 15),     # one leftover tile
                                    (256 * 257, 256, 8192, 16, 15)):
        pl = plan(m, n, k, c=c256)
        assert (pl.blk_m, pl.sched, pl.grid, pl.dp_tiles, pl.split, pl.max_peers) == \
            (256, S.SK_SCHED_DP_1TILE_SK, 256, 256, split, peers), (m, n, k)
    for (m, n, k) in ((4096, 4096 + 256, 1024),          # 16 iterations per tile
                      (4096, 256 * 25, 4096),            # a 144-tile tail: more than half the slots
                      (4096, 4096, 4096)):               # no partial wave
        pl = plan(m, n, k, c=c256)
        assert (pl.blk_m, pl.sched) == (256, S.SK_SCHED_DP), (m, n, k, pl.sched)


def test_owner_peer_gate():
    # deep-k single tiles whose paper model grid would give the owner more
    # than SK_MAX_PEERS peers: the library's model grid stays within it
    for (m, n, k, dt) in ((128, 128, 524288, "f64"), (128, 128, 2097152, "bf16"), (128, 128, 16384, "f64")):
        d = desc(m=m, n=n, k=k, ab_type=dt, c_type="f64" if dt == "f64" else "f32")
        for fx in ("auto", "serial", "spread"):
            for sched in ("auto", "sk"):
                blk = (128, 128, 64) if dt == "bf16" else None     # one tile (the default would be 64x64)
                st, pl = S.sk_plan(d, S.make_config(sched=sched, wg_slots=256, fixup=fx, blk=blk))
                assert st == S.SK_OK, (m, n, k, dt, fx, sched)
                assert pl.tiles == 1 and pl.max_peers <= S.SK_MAX_PEERS and pl.grid == pl.max_peers + 1, \
                    (pl.grid, pl.max_peers)
    # a caller-fixed grid that needs more peers is refused before any launch
    d = desc(m=128, n=128, k=16384, ab_type="f64", c_type="f64")
    cfg = S.make_config(sched="sk", blk=(128, 128, 16), grid=256, wg_slots=256)
    assert S.sk_plan(d, cfg)[0] == S.SK_ERR_UNSUPPORTED
    assert S.sk_gemm(d, cfg, FAKE, 1 << 30, 0) == S.SK_ERR_UNSUPPORTED
    assert S.sk_plan(d, S.make_config(sched="sk", blk=(128, 128, 16), grid=65, wg_slots=256))[0] == S.SK_OK
    assert S.sk_plan(d, S.make_config(sched="sk", blk=(128, 128, 16), grid=66, wg_slots=256))[0] == \
        S.SK_ERR_UNSUPPORTED
    # DP + one-tile SK with one leftover tile on 256 slots: 255 peers, refused;
    # the automatic schedule of the same FP64 problem avoids it
    d = desc(m=257 * 128, n=128, k=16384, ab_type="f64", c_type="f64")
    st, pl = S.sk_plan(d, S.make_config(sched="dp1sk", blk=(128, 128, 16), wg_slots=256))
    assert st == S.SK_ERR_UNSUPPORTED
    st, pl = S.sk_plan(d, S.make_config(blk=(128, 128, 16), wg_slots=256))
    assert st == S.SK_OK and pl.max_peers <= S.SK_MAX_PEERS


def test_fixup_mode_resolution():
    # explicit modes are honoured; AUTO takes the spread fixup only where an
    # owner has at least two peers
    d = desc(m=256, n=256, k=65536, ab_type="bf16", c_type="bf16")
    for fx, want in (("serial", S.SK_FIXUP_SERIAL), ("spread", S.SK_FIXUP_SPREAD)):
        st, pl = S.sk_plan(d, S.make_config(sched="sk", blk=(128, 128, 64), grid=64, wg_slots=512, fixup=fx))
        assert st == S.SK_OK and pl.fixup == want
    st, pl = S.sk_plan(d, S.make_config(sched="sk", blk=(128, 128, 64), grid=64, wg_slots=512))
    assert st == S.SK_OK and pl.max_peers >= 2 and pl.fixup == S.SK_FIXUP_SPREAD
    # the two-tile hybrid: every owner has at most one peer -> serial
    d = desc(m=4096, n=4096, k=1024, ab_type="f64", c_type="f64")
    st, pl = S.sk_plan(d, S.make_config(sched="2tsk", blk=(128, 128, 16), wg_slots=256, threshold=1))
    assert st == S.SK_OK and pl.max_peers <= 1 and pl.fixup == S.SK_FIXUP_SERIAL
    assert S.sk_plan(d, S.make_config(fixup=7, wg_slots=256))[0] == S.SK_ERR_INVALID_VALUE


def test_workspace_reserves_flag_region_for_every_schedule():
    # header (256 B) + flag region (2 x SK_MAX_GRID flags, 64 B apart) come
    # first in every workspace, whatever the schedule; a spread plan holds two
    # partial slots per workgroup
    base = 256 + 2 * S.SK_MAX_GRID * 64
    d = desc(m=1024, n=1024, k=1024, ab_type="bf16", c_type="f32")
    st, pl = S.sk_plan(d, S.make_config(sched="dp", wg_slots=512))
    assert st == S.SK_OK and pl.workspace_bytes >= base
    slot = 128 * 128 * 4
    for fx, per in (("serial", 1), ("spread", 2)):
        st, pl = S.sk_plan(d, S.make_config(sched="sk", blk=(128, 128, 64), grid=100, wg_slots=512, fixup=fx))
        assert st == S.SK_OK and pl.workspace_bytes >= base + per * 100 * slot
    assert S.sk_plan(d, S.make_config(sched="sk", grid=S.SK_MAX_GRID + 1, wg_slots=4096))[0] == \
        S.SK_ERR_INVALID_VALUE


def test_model_memory_term():
    # the optional memory term charges every workgroup of a tile-splitting
    # plan for writing and reading back a partial tile: a scarce bandwidth
    # pushes the model's grid down, an ample one leaves it unchanged
    d = desc(m=256, n=256, k=65536, ab_type="bf16", c_type="f32")
    grids = {}
    for bw in (0.0, 1e12, 4e6, 1e4):
        cfg = S.make_config(sched="sk", blk=(128, 128, 64), wg_slots=512, fixup="spread")
        cfg.model_bw = bw
        st, pl = S.sk_plan(d, cfg)
        assert st == S.SK_OK
        grids[bw] = pl.grid
    assert grids[1e12] == grids[0.0]
    assert grids[1e4] < grids[4e6] <= grids[0.0]


def test_fixed_split_plans():
    # Algorithm 4 with s not dividing I: pieces of ceil(I / s), the last shorter
    d = desc(m=512, n=512, k=100 * 64, ab_type="bf16", c_type="f32")          # t = 16, I = 100
    pl = check_plan_agrees([(512, 512, 100 * 64)], "bf16", (128, 128, 64), 512, "fs", 0)
    # automatic s: 25 (s = 26..32 would give pieces of 4 and leave empty ones)
    assert (pl.split, pl.grid, pl.max_peers) == (25, 400, 24)
    # an explicit s may leave empty pieces (Algorithm 4): s = 33, pieces of 4, 25 of them non-empty
    for s_, peers in ((3, 2), (7, 6), (9, 8), (33, 24)):
        st, pl = S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=1024, split=s_))
        assert st == S.SK_OK and (pl.sched, pl.split, pl.grid, pl.max_peers) == \
            (S.SK_SCHED_FIXED_SPLIT, s_, 16 * s_, peers), (s_, pl.max_peers)
    # s = 50: pieces of 2
    st, pl = S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=1024, split=50))
    assert st == S.SK_OK and pl.max_peers == 49
    # I = 9, s = 4: pieces of 3, the last empty (Algorithm 4 allows it)
    d9 = desc(m=128, n=128, k=9 * 64, ab_type="bf16", c_type="f32")
    st, pl = S.sk_plan(d9, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=64, split=4))
    assert st == S.SK_OK and (pl.grid, pl.max_peers) == (4, 2)
    # s = 1 is the data-parallel schedule, also with more tiles than slots
    st, pl = S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=512, split=1))
    assert st == S.SK_OK and (pl.sched, pl.grid) == (S.SK_SCHED_DP, 16)
    dbig = desc(m=4096, n=4096, k=4096, ab_type="bf16", c_type="f32")          # t = 1024 > 512 slots
    st, pl = S.sk_plan(dbig, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=512))
    assert st == S.SK_OK and (pl.sched, pl.grid) == (S.SK_SCHED_DP, 1024)
    # errors: more peers than served, more workgroups than slots, a grid
    # other than s t, grouped calls
    assert S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=2048, split=66))[0] == \
        S.SK_ERR_UNSUPPORTED
    assert S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=256, split=17))[0] == \
        S.SK_ERR_INVALID_VALUE
    assert S.sk_plan(d, S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=512, split=4, grid=60))[0] == \
        S.SK_ERR_INVALID_VALUE
    assert S.sk_plan([d, d], S.make_config(sched="fs", blk=(128, 128, 64), wg_slots=512))[0] == \
        S.SK_ERR_UNSUPPORTED
    assert S.sk_plan(d, S.make_config(sched="fs", split=-1))[0] == S.SK_ERR_INVALID_VALUE
