"""Helpers for the GPU parity tests: run the library through the C ABI on
seeded inputs and compare with the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import workloads as W
from oracle import schedule as O
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S

F64_BOUND = 1e-13           # normwise, FP64
LOWP_BOUND = 5e-5           # normwise, FP16/BF16/FP8 with FP32 accumulation (k <= 65536)


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(op: W.Operand) -> W.Operand:
    return op.to("cuda")


def c_tensor(m, n, c_type, c_order, init: np.ndarray | None = None):
    """Device C in its storage order (logical m x n) and its ld."""
    if init is None:
        logical = torch.full((m, n), float("nan"), dtype=torch.float64)
    else:
        logical = torch.from_numpy(np.ascontiguousarray(init))
    t = logical.to(W.torch_dtype(c_type))
    if c_order == "row":
        return t.contiguous().cuda(), n
    return t.t().contiguous().cuda(), m


def c_logical(Ct: torch.Tensor, m, n, c_order) -> torch.Tensor:
    h = Ct.cpu()
    return h if c_order == "row" else h.t()


def c_values(Ct, m, n, c_order) -> np.ndarray:
    return c_logical(Ct, m, n, c_order).double().numpy()


def c_bits(Ct, m, n, c_order) -> np.ndarray:
    h = c_logical(Ct, m, n, c_order).contiguous()
    if h.dtype == torch.float64:
        return h.view(torch.int64).numpy()
    if h.dtype == torch.float32:
        return h.view(torch.int32).numpy().view(np.uint32)
    return h.view(torch.int16).numpy().view(np.uint16)


def expected_bits(cref: np.ndarray, c_type: str) -> np.ndarray:
    if c_type == "f64":
        return np.ascontiguousarray(cref).view(np.int64)
    return oracle.round_to(cref, c_type)


def rel_err(C: np.ndarray, Cref: np.ndarray, Ad: np.ndarray, Bd: np.ndarray) -> float:
    den = np.linalg.norm(Ad) * np.linalg.norm(Bd)
    return float(np.linalg.norm(C - Cref) / den) if den > 0 else float(np.linalg.norm(C - Cref))


def bound_for(ab_type: str, c_type: str, cref, Ad, Bd) -> float:
    if ab_type == "f64":
        return F64_BOUND
    b = LOWP_BOUND
    if c_type in ("bf16", "f16"):
        # the output's own rounding is allowed on top (one rounding of Cref)
        rounded = oracle.decode(oracle.round_to(cref, c_type), c_type)
        b += rel_err(rounded, cref, Ad, Bd)
    return b


def run_gemm(m, n, k, A, B, *, c_type, c_order="row", C0=None, alpha=1.0, beta=0.0, cfg=None,
             ws=None, trace_cap=0):
    """Launch sk_gemm on device operands; returns (C tensor, plan, trace)."""
    Ct, ldc = c_tensor(m, n, c_type, c_order, C0)
    tr = None
    if trace_cap:
        tr = torch.zeros(8 + 8 * trace_cap, dtype=torch.int32, device="cuda")
        cfg = cfg or S.make_config()
        cfg.trace = tr.data_ptr()
        cfg.trace_capacity = trace_cap
    ws = ws or R.Workspace("cuda")
    plan = R.gemm(m, n, k, A, B, Ct, c_type=c_type, c_order=c_order, ldc=ldc, alpha=alpha,
                  beta=beta, cfg=cfg, ws=ws)
    torch.cuda.synchronize()
    ws.check()
    trace = R.read_trace(tr) if tr is not None else None
    return Ct, plan, trace


def oracle_segments(plan, shapes, c_order="row"):
    """Per-WG segment lists the schedule oracle predicts for a library plan
    (a fixed-split plan: Algorithm 4's)."""
    blk = (plan.blk_m, plan.blk_n, plan.blk_k)
    oshapes = [(n, m, k) if c_order == "col" else (m, n, k) for (m, n, k) in shapes]
    geos = [O.geometry(m, n, k, *blk) for (m, n, k) in oshapes]
    if plan.sched == S.SK_SCHED_FIXED_SPLIT:
        assert len(geos) == 1
        return O.fixed_split_segments(geos[0].t, geos[0].I, plan.split)
    if plan.sched == S.SK_SCHED_DP_1TILE_SK and plan.split > 0:
        # data-parallel waves (tile j on workgroup j mod g), then Algorithm 4
        # on the tail tiles
        assert len(geos) == 1 and plan.dp_first
        g, I = plan.grid, geos[0].I
        out = [[] for _ in range(g)]
        for j in range(plan.dp_tiles):
            out[j % g].append(O.Segment(j % g, j, 0, I, O.ROLE_DP))
        r = plan.sk_tile_end - plan.sk_tile_begin
        for lst in O.fixed_split_segments(r, I, plan.split):
            for sg in lst:
                out[sg.wg].append(O.Segment(sg.wg, plan.sk_tile_begin + sg.tile, sg.k_begin, sg.k_end,
                                            sg.role, sg.peers))
        return out
    probs = O.Problems([(g.t if (m > 0 and n > 0) else 0, g.I) for g, (m, n, k) in zip(geos, oshapes)])
    op = O.Plan(plan.grid, plan.sk_tile_begin, plan.sk_tile_end, bool(plan.dp_first), plan.sched,
                probs.tiles,
                [t for t in range(probs.tiles) if not (plan.sk_tile_begin <= t < plan.sk_tile_end)])
    segs = O.segments(probs, op)
    O.check_invariants(probs, op, segs)
    return segs


ROLE_REDUCE = 4


def compare_trace(trace, plan, shapes, c_order="row", acc_bytes=4, static_dp=False):
    """The executed segments must be the schedule oracle's, record by record.
    A persistent launch of several problems with more data-parallel tiles
    than workgroups takes them, after each workgroup's first, from per-XCD
    queues (unless SK_FLAG_STATIC_DP_TILES, `static_dp`): then each
    workgroup's Stream-K
    segments and first data-parallel tile are the oracle's, and the
    data-parallel tiles, whichever workgroup ran them, are the oracle's, each
    exactly once.  Slice reductions of the spread fixup (role 4) are checked
    separately: every split tile's partial chunks are reduced exactly once, by
    each of its contributors in turn, in ascending slices."""
    count, recs = trace
    segs = oracle_segments(plan, shapes, c_order)
    seg_recs = [r for r in recs if r[5] != ROLE_REDUCE]
    red_recs = [r for r in recs if r[5] == ROLE_REDUCE]
    expect = sum(len(l) for l in segs)
    assert len(seg_recs) == expect, f"trace has {len(seg_recs)} segment records, oracle {expect}"
    got = {}
    for (wg, seq, tile, k0, k1, role, last, _x) in seg_recs:
        got.setdefault(wg, []).append((seq, tile, k0, k1, role, last))
    dyn = not static_dp and len(shapes) > 1 and plan.sched != S.SK_SCHED_DP and plan.dp_tiles > plan.grid

    def rec(sg):
        return (sg.tile, sg.k_begin, sg.k_end, sg.role, sg.peers[-1] if sg.peers else -1)
    if dyn:
        dp_got = sorted(r[1] for lst in got.values() for r in lst if r[4] == O.ROLE_DP)
        dp_want = sorted(sg.tile for lst in segs for sg in lst if sg.role == O.ROLE_DP)
        assert dp_got == dp_want, "data-parallel tiles differ from the oracle's or repeat"
        for x, lst in enumerate(segs):
            mine = [r[1:] for r in sorted(got.get(x, []))]
            mine_sk = [r for r in mine if r[3] != O.ROLE_DP]
            want_sk = [rec(sg) for sg in lst if sg.role != O.ROLE_DP]
            assert mine_sk == want_sk, f"workgroup {x}: {mine_sk[:4]} != {want_sk[:4]}"
            mine_dp = [r for r in mine if r[3] == O.ROLE_DP]
            want_dp = [rec(sg) for sg in lst if sg.role == O.ROLE_DP]
            assert mine_dp[:1] == want_dp[:1], f"workgroup {x}: first data-parallel tile"
    else:
        for x, lst in enumerate(segs):
            mine = [r[1:] for r in sorted(got.get(x, []))]
            want = [rec(sg) for sg in lst]
            assert mine == want, f"workgroup {x}: {mine[:4]} != {want[:4]}"
    split = {}
    for lst in segs:
        for sg in lst:
            if sg.role == O.ROLE_OWNER:
                split[sg.tile] = (sg.wg, sg.peers[-1])
    if plan.fixup != S.SK_FIXUP_SPREAD:
        assert not red_recs, "slice reductions in a serial-fixup launch"
        return
    nchunks = plan.blk_m * plan.blk_n * acc_bytes // 16
    by_tile = {}
    for (wg, seq, tile, c0, c1, role, last, first) in red_recs:
        by_tile.setdefault(tile, []).append((wg, c0, c1, first, last))
    assert set(by_tile) == set(split), "reduced tiles differ from the split tiles"
    for tile, lst in by_tile.items():
        f, l = split[tile]
        lst.sort()
        assert [r[0] for r in lst] == list(range(f, l + 1)), f"tile {tile}: reducers {[r[0] for r in lst]}"
        assert all(r[3] == f and r[4] == l for r in lst)
        pos = 0
        for (wg, c0, c1, _f, _l) in lst:
            assert c0 == pos and c1 > c0, f"tile {tile}: slice [{c0},{c1}) after {pos}"
            pos = c1
        assert pos == nchunks, f"tile {tile}: slices end at {pos}, not {nchunks}"


def ws_header(ws):
    """(error word, generation, done counter) of a workspace."""
    h = ws.buf[:12].view(torch.int32).cpu().tolist()
    return tuple(h)
