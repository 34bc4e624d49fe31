#!/usr/bin/env python3
"""Stream-K GEMM benchmark on one MI355X.

Workload (one "step"): the geometry sweep -- 2048 GEMMs with m, n, k drawn
log-uniformly from [128, 8192] (seed 1, rounded to multiples of 8), FP16
inputs uniform in [-1, 1], FP32 accumulation and output, alpha = 1,
beta = 0, row-major -- each run once through sk_gemm with the library's
default configuration (per problem: a 64x64, 128x128 or 256x256 tile by size
and depth; data-parallel, k-aligned fixed split, basic Stream-K, or
data-parallel waves with a fixed-split tail).  Inputs are resident in HBM
before timing starts.

Reported on one JSON line: aggregate TFLOP/s of the step (value), % of the
FP16 dense MFMA peak, per-GEMM latency p50/p99, the same sweep under the
data-parallel, basic Stream-K and the paper's two-tile Stream-K + DP hybrid
schedules (the paper's comparison), the fixed split and the best of the
library's data-parallel tiles per problem, the roofline of the dominant
kernel (and of every other kernel symbol) measured with HIP events on the
launch stream, and the CPU oracle timed on a bounded sample of the same
workload.

`--extended` adds the FP64 sweep and the precision set (BF16 and FP8 on
8192^3, 256x256x65536, 4096x1024x4096).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f16": 2516.6, "bf16": 2516.6, "f8e4m3": 5033.2}
HBM_GBS = 8000.0
METRIC = "TFLOP/s and % dtype MFMA peak, Stream-K vs data-parallel tiling; p50/p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


class Sweep:
    """All problems of a sweep with operands resident in rotating device
    arenas (consecutive problems never share operand memory)."""

    def __init__(self, shapes, ab, ct, seed, arena_bytes=4 << 30):
        import torch
        import workloads as W
        from paper_2301_03598_amd import streamk as S
        self.shapes = shapes
        self.ab, self.ct = ab, ct
        eb = W.DTYPE_BYTES[ab]
        cb = W.DTYPE_BYTES[ct]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        tdt, cdt = W.torch_dtype(ab), W.torch_dtype(ct)

        def arena(nbytes, dt, esize, fill):
            t = torch.empty(nbytes // esize, dtype=dt, device="cuda")
            if fill:
                t.uniform_(-1.0, 1.0, generator=gen)
            return t
        self.A = arena(arena_bytes, tdt, eb, True)
        self.B = arena(arena_bytes, tdt, eb, True)
        self.C = arena(arena_bytes, cdt, cb, False)
        offs = {"A": 0, "B": 0, "C": 0}

        def place(name, nelem, esize, total):
            nbytes = (nelem * esize + 255) // 256 * 256
            if offs[name] + nbytes > total:
                offs[name] = 0
            o = offs[name]
            offs[name] += nbytes
            return o
        self.descs = (S.sk_gemm_desc_t * len(shapes))()
        self.flops = []
        for i, (m, n, k) in enumerate(shapes):
            oa = place("A", m * k, eb, arena_bytes)
            ob = place("B", k * n, eb, arena_bytes)
            oc = place("C", m * n, cb, arena_bytes)
            self.descs[i] = S.make_desc(m, n, k, self.A.data_ptr() + oa, self.B.data_ptr() + ob,
                                        self.C.data_ptr() + oc, ab_type=ab, c_type=ct)
            self.flops.append(2.0 * m * n * k)
        self.total_flops = sum(self.flops)


class Runner:
    """Launches sk_gemm for every problem of a sweep on the current stream.

    `cfg` is one configuration for every problem or a list with one per
    problem; a problem whose plan the library refuses under it (an owner
    would wait on more peers than the library serves) runs with the default
    configuration instead and is counted in `fallbacks`.

    `step_timed` is the timed form: the launches grouped by kernel symbol
    (the problems of one symbol back to back -- the order of a sweep's
    independent GEMMs is free), one HIP event at each group boundary and no
    other GPU work.  `step_events` brackets every launch with an event pair
    (per-GEMM latency); each pair costs several microseconds of GPU time, so
    it is kept out of the timed region."""

    def __init__(self, sweep, cfg):
        import torch
        from paper_2301_03598_amd import runtime as R
        from paper_2301_03598_amd import streamk as S
        self.S = S
        self.sweep = sweep
        n = len(sweep.shapes)
        cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg] * n
        self.L = S.lib()
        need = 256
        self.plans = []
        self.cfgs = []
        self.fallbacks = 0
        for i in range(n):
            st, pl = S.sk_plan(sweep.descs[i], cfgs[i])
            c = cfgs[i]
            if st == S.SK_ERR_UNSUPPORTED:
                c = S.make_config()
                st, pl = S.sk_plan(sweep.descs[i], c)
                self.fallbacks += 1
            S.check(st, "sk_plan")
            self.plans.append(pl)
            self.cfgs.append(c)
            need = max(need, pl.workspace_bytes)
        self.ws = R.Workspace("cuda", need)
        self.stream = torch.cuda.current_stream()
        self.sptr = ctypes.c_void_p(self.stream.cuda_stream)
        self.wsp = ctypes.c_void_p(self.ws.ptr)
        self.cfgps = [ctypes.byref(c) if c is not None else None for c in self.cfgs]
        self.dptrs = [ctypes.byref(sweep.descs[i]) for i in range(n)]
        self.ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        self.ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        # problems grouped by kernel symbol, in sweep order within a group
        self.groups = {}
        for i, pl in enumerate(self.plans):
            self.groups.setdefault(kernel_of(pl, sweep.ab), []).append(i)
        self.gev = []                   # per timed step: {symbol: (start, end)}
        self.group_ms = {k: 0.0 for k in self.groups}
        self.group_steps = 0

    def _launch(self, i):
        st = self.L.sk_gemm(self.dptrs[i], self.cfgps[i], self.wsp, self.ws.nbytes, self.sptr)
        if st != 0:
            raise RuntimeError(f"sk_gemm failed on problem {i}: {self.S.sk_status_string(st)}")

    def step_plain(self):
        for i in range(len(self.dptrs)):
            self._launch(i)

    def step_timed(self):
        import torch
        ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in self.groups}
        self.gev.append(ev)
        for k, idx in self.groups.items():
            e0, e1 = ev[k]
            e0.record(self.stream)
            for i in idx:
                self._launch(i)
            e1.record(self.stream)

    def collect_timed(self):
        """Per-symbol GPU time of every timed step so far (after a sync)."""
        for ev in self.gev:
            for k, (e0, e1) in ev.items():
                self.group_ms[k] += e0.elapsed_time(e1)
            self.group_steps += 1
        self.gev = []

    def step_events(self, durations):
        for i in range(len(self.dptrs)):
            self.ev0[i].record(self.stream)
            self._launch(i)
            self.ev1[i].record(self.stream)
        self.stream.synchronize()
        durations.append([self.ev0[i].elapsed_time(self.ev1[i]) for i in range(len(self.dptrs))])


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*_traffic.md with a machine-readable line for that kernel), or
    None when there is none or the kernel source changed since it was taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2301_03598_amd", "csrc", "sk_kernel.hpp")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        try:
            for line in open(path):
                if line.startswith("machine-readable: "):
                    rec = json.loads(line[len("machine-readable: "):])
                    if rec.get("kernel") == kernel and rec.get("kernel_source_sha256_16") == h:
                        return rec["traffic_bytes_per_launch"]
        except OSError:
            pass
    return None


def geomean(xs):
    xs = [x for x in xs if x > 0]
    return math.exp(sum(math.log(x) for x in xs) / len(xs)) if xs else 0.0


def pct(xs, q):
    ys = sorted(xs)
    if not ys:
        return 0.0
    idx = min(len(ys) - 1, max(0, int(math.ceil(q / 100.0 * len(ys))) - 1))
    return ys[idx]


def kernel_of(pl, ab: str = "f16") -> str:
    """The kernel symbol a planned launch runs (data-parallel or Stream-K
    entry, input type, tile; the sweeps are row-major)."""
    from paper_2301_03598_amd import streamk as S
    kern = "dp_kernel" if pl.sched == S.SK_SCHED_DP else "sk_kernel"
    return f"{kern}<{ab.upper()}, {pl.blk_m}x{pl.blk_n}x{pl.blk_k}, A k-contiguous, B n-contiguous>"


def schedule_leg(sweep, cfg, passes=2):
    """Aggregate TFLOP/s of a sweep under one configuration (or one per
    problem; plain launches, wall clock) and per-problem TFLOP/s from a
    separate event pass."""
    import torch
    from paper_2301_03598_amd import streamk as S
    if isinstance(cfg, str):
        cfg = S.make_config(sched=cfg)
    run = Runner(sweep, cfg)
    run.step_plain()                # warm-up pass
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        run.step_plain()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / passes
    durs = []
    run.step_events(durs)
    per = durs[0]
    tf = [sweep.flops[i] / (per[i] * 1e-3) / 1e12 for i in range(len(per))]
    res = {"tflops": round(sweep.total_flops / wall / 1e12, 2),
           "geomean_tflops": round(geomean(tf), 2),
           "pct_peak": round(100 * sweep.total_flops / wall / 1e12 / PEAK_TFLOPS[sweep.ab], 2)}
    if run.fallbacks:
        res["fallbacks_to_default"] = run.fallbacks
    return res, tf, run


def fixed_split_configs(sweep, blk):
    """Algorithm 4 (fixed split, SK_SCHED_FIXED_SPLIT) per problem with the
    library's splitting factor: the largest s <= SK_MAX_PEERS + 1 with s t <= p
    (one wave on the resident slots) whose pieces of ceil(I / s) iterations
    leave none empty; s = 1 (the tiles alone fill the slots) is the
    data-parallel schedule of the same tile."""
    from paper_2301_03598_amd import streamk as S
    out, splits = [], []
    for d in sweep.descs:
        cfg = S.make_config(sched="fs", blk=blk)
        st, pl = S.sk_plan(d, cfg)
        S.check(st, "sk_plan")
        splits.append(pl.split if pl.sched == S.SK_SCHED_FIXED_SPLIT else 1)
        out.append(cfg)
    return out, splits


def ensemble_leg(sweep, tiles, passes=1):
    """The idealized data-parallel ensemble (the paper's oracle column): per
    problem the fastest of the library's data-parallel kernels over the given
    tiles, by per-launch events; aggregate TFLOP/s from the summed best times."""
    from paper_2301_03598_amd import streamk as S
    best = None
    for blk in tiles:
        run = Runner(sweep, S.make_config(sched="dp", blk=blk))
        run.step_plain()
        durs = []
        for _ in range(passes):
            run.step_events(durs)
        per = [min(d[i] for d in durs) for i in range(len(sweep.shapes))]
        best = per if best is None else [min(a, b) for a, b in zip(best, per)]
        del run
    tf = [sweep.flops[i] / (best[i] * 1e-3) / 1e12 for i in range(len(best))]
    tot_ms = sum(best)
    return {"tflops": round(sweep.total_flops / (tot_ms * 1e-3) / 1e12, 2),
            "geomean_tflops": round(geomean(tf), 2),
            "tiles": [f"{b[0]}x{b[1]}x{b[2]}" for b in tiles],
            "timing": "sum of per-launch event times of the best tile per problem"}, tf


def attainable_tflops(m, n, k, in_b, out_b, peak_tflops):
    """min(MFMA peak, arithmetic intensity x HBM bandwidth) of one GEMM, with
    its compulsory bytes (A and B read once, C written once)."""
    flops = 2.0 * m * n * k
    bytes_ = (m * k + k * n) * in_b + m * n * out_b
    return min(peak_tflops, flops / bytes_ * HBM_GBS / 1e3)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_error_vs(cref, m, n, k, A, B, ct):
    """||C - Cref||_F / (||A||_F ||B||_F) of the library's result on the
    stored inputs A, B against an oracle result Cref (and, for a 16-bit
    output, the same statistic of Cref's own rounding to that type, which
    the error cannot go below)."""
    import numpy as np
    import torch
    import oracle
    import workloads as W
    from paper_2301_03598_amd import runtime as R
    Ad, Bd = A.to("cuda"), B.to("cuda")
    C = torch.empty((m, n), dtype=W.torch_dtype(ct), device="cuda")
    R.gemm(m, n, k, Ad, Bd, C, c_type=ct)
    torch.cuda.synchronize()
    got = C.cpu().double().numpy()
    den = float(np.linalg.norm(oracle.decode_operand(A)) * np.linalg.norm(oracle.decode_operand(B)))
    out = {"err": float(np.linalg.norm(got - cref) / den)}
    if ct in ("bf16", "f16"):
        out["output_rounding"] = float(np.linalg.norm(oracle.decode(oracle.round_to(cref, ct), ct) - cref) / den)
    return {k2: float(f"{v:.4g}") for k2, v in out.items()}


def cpu_baseline(budget_flops=7.0e11):
    """The CPU oracle, as it stands, on a bounded sample of the sweep (the
    problems in draw order whose flops fit the budget, FP16 inputs), plus
    configuration 1 (FP64 384x384x1024) and the precision set's
    4096x1024x4096 on BF16 and FP8 inputs, each timed once; for these three
    the library's error against the oracle result is reported beside the
    timing."""
    import oracle
    import workloads as W
    shapes = W.sweep_shapes()
    pick, tot = [], 0.0
    for (m, n, k) in shapes:
        f = 2.0 * m * n * k
        if tot + f <= budget_flops:
            pick.append((m, n, k))
            tot += f
    oracle.build(force=False)
    t = 0.0
    for i, (m, n, k) in enumerate(pick):
        A, B = W.gemm_operands(m, n, k, "f16", 1000 + i, "uniform")
        t0 = time.perf_counter()
        oracle.gemm(m, n, k, A, B, c_type="f32")
        t += time.perf_counter() - t0
    extra = {}
    for name, (m, n, k), ab, ct, dist, seed in (("config1_f64_384x384x1024", (384, 384, 1024), "f64", "f64",
                                                  "uniform", 0),
                                                 ("precision_c_bf16_4096x1024x4096", (4096, 1024, 4096), "bf16",
                                                  "bf16", "normal", 2),
                                                 ("precision_c_f8e4m3_4096x1024x4096", (4096, 1024, 4096), "f8e4m3",
                                                  "bf16", "normal", 2)):
        A, B = W.gemm_operands(m, n, k, ab, seed, dist)
        t0 = time.perf_counter()
        cref = oracle.gemm(m, n, k, A, B, c_type=ct)
        dt = time.perf_counter() - t0
        extra[name] = {"gflops": round(2.0 * m * n * k / dt / 1e9, 2), "s": round(dt, 3)}
        # the same inputs through the library (default configuration): its
        # normwise error against this oracle result
        extra[name]["gpu_rel_err"] = gpu_error_vs(cref, m, n, k, A, B, ct)
    cores = int(os.environ.get("OMP_NUM_THREADS", 0) or len(os.sched_getaffinity(0)))
    return {"value": round(tot / t / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(pick)} sweep problems (draw order, FP16->FP32) fitting a "
                      f"{budget_flops:.1e}-flop budget; {tot:.3e} flop in {t:.1f} s",
            "configs": extra}


def extended():
    """FP64 sweep under the three schedules and the precision set."""
    import torch
    import workloads as W
    from paper_2301_03598_amd import runtime as R
    from paper_2301_03598_amd import streamk as S
    out = {}
    sw = Sweep(W.sweep_shapes(), "f64", "f64", seed=11)
    for sched in ("dp", "sk", "2tsk", "auto"):
        out[f"f64_sweep_{sched}"], _, _ = schedule_leg(sw, sched, passes=1)
        log("f64", sched, out[f"f64_sweep_{sched}"])
    del sw
    torch.cuda.empty_cache()
    ws = R.Workspace("cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    for name, (m, n, k) in W.PRECISION_SHAPES.items():
        for ab, ct in (("bf16", "bf16"), ("f8e4m3", "bf16")):
            A = torch.empty(m * k, dtype=W.torch_dtype(ab), device="cuda")
            B = torch.empty(k * n, dtype=W.torch_dtype(ab), device="cuda")
            W.device_fill_(A, "normal", gen)
            W.device_fill_(B, "normal", gen)
            C = torch.empty(m * n, dtype=W.torch_dtype(ct), device="cuda")
            for sched in ("dp", "auto"):
                cfg = S.make_config(sched=sched)
                d = S.make_desc(m, n, k, A, B, C, ab_type=ab, c_type=ct,
                                a_scale=1.0, b_scale=1.0)
                st, pl = S.sk_plan(d, cfg)
                S.check(st, "sk_plan")
                ws.ensure(pl.workspace_bytes)
                s = torch.cuda.current_stream().cuda_stream
                for _ in range(3):
                    S.check(S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, s), "sk_gemm")
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 10
                e0.record()
                for _ in range(reps):
                    S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, s)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
                key = f"{name}_{m}x{n}x{k}_{ab}_{sched}"
                out[key] = {"ms": round(ms, 4), "tflops": round(tf, 1),
                            "pct_peak": round(100 * tf / PEAK_TFLOPS[ab], 2),
                            "sched": S.SCHED_NAME.get(pl.sched, pl.sched), "grid": pl.grid}
                log(key, out[key])
            del A, B, C
    return out


def one_gemm(m: int, n: int, k: int, ab: str, reps: int = 20, flags: int = 0, ldc: int = 0) -> dict:
    """One precision-set style GEMM (N(0,1) operands from seed 2, BF16 output
    for 16-bit and FP8 inputs, FP64 for FP64), default configuration (plus
    the given SK_FLAG_* bits; C's leading dimension `ldc`, 0 for n): 3
    warm-up launches, then `reps` timed back to back."""
    import torch
    import workloads as W
    from paper_2301_03598_amd import runtime as R
    from paper_2301_03598_amd import streamk as S
    ct = "f64" if ab == "f64" else "bf16"
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    A = torch.empty(m * k, dtype=W.torch_dtype(ab), device="cuda")
    B = torch.empty(k * n, dtype=W.torch_dtype(ab), device="cuda")
    W.device_fill_(A, "normal", gen)
    W.device_fill_(B, "normal", gen)
    C = torch.empty(m * (ldc or n), dtype=W.torch_dtype(ct), device="cuda")
    cfg = S.make_config(flags=flags)
    d = S.make_desc(m, n, k, A, B, C, ab_type=ab, c_type=ct, ldc=ldc, a_scale=1.0, b_scale=1.0)
    st, pl = S.sk_plan(d, cfg)
    S.check(st, "sk_plan")
    ws = R.Workspace("cuda", pl.workspace_bytes)
    s = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        S.check(S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, s), "sk_gemm")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        S.sk_gemm(d, cfg, ws.ptr, ws.nbytes, s)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
    return {"gemm": f"{m}x{n}x{k}", "ab": ab, "c": ct, "reps": reps, "ms": round(ms, 4),
            "tflops": round(tf, 1), "pct_peak": round(100 * tf / PEAK_TFLOPS[ab], 2),
            "sched": S.SCHED_NAME.get(pl.sched, pl.sched), "grid": pl.grid,
            "split": pl.split, "tile": f"{pl.blk_m}x{pl.blk_n}x{pl.blk_k}", "flags": flags,
            "xcd_remap": pl.xcd_remap, "ldc": ldc or n}


def grouped_leg(tune: bool = True):
    """512 BF16 GEMMs (seed 3): one grouped persistent launch captured in a
    HIP graph and replayed, against 512 separate sk_gemm launches; the
    grouped configuration comes from the autotuner (library default shown
    beside it)."""
    import torch
    import workloads as W
    from paper_2301_03598_amd import runtime as R
    from paper_2301_03598_amd import streamk as S
    from paper_2301_03598_amd import tune as T
    shapes = W.grouped_shapes()
    sw = Sweep(shapes, "bf16", "f32", seed=3, arena_bytes=6 << 30)
    descs = list(sw.descs)
    flops = sw.total_flops
    out = {"problems": len(shapes), "flops": flops}
    # separate launches, library default per problem
    run = Runner(sw, S.make_config(sched="auto"))
    run.step_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        run.step_plain()
    torch.cuda.synchronize()
    sep_ms = (time.perf_counter() - t0) / 3 * 1e3
    out["separate_launches"] = {"ms": round(sep_ms, 3), "tflops": round(flops / sep_ms / 1e9, 1)}

    def grouped_time(cfg, label):
        ws = R.Workspace("cuda")
        arr = (S.sk_gemm_desc_t * len(descs))(*descs)
        st, plan = S.sk_plan(arr, cfg)
        S.check(st, "sk_plan")
        ws.ensure(plan.workspace_bytes)
        R.gemm_grouped(descs, cfg=cfg, ws=ws)
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            _, keep = R.gemm_grouped(descs, cfg=cfg, ws=ws, stream=stream)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        del keep
        return {"ms": round(ms, 3), "tflops": round(flops / ms / 1e9, 1),
                "sched": S.SCHED_NAME.get(plan.sched, plan.sched), "grid": plan.grid,
                "tile": f"{plan.blk_m}x{plan.blk_n}x{plan.blk_k}", "fixup": S.FIXUP_NAME.get(plan.fixup),
                "persistent": plan.sched != S.SK_SCHED_DP, "label": label}
    # one persistent launch of the whole batch under each schedule
    out["grouped_default"] = grouped_time(S.make_config(sched="auto"), "library default")
    out["grouped_sk_basic"] = grouped_time(S.make_config(sched="sk"), "basic Stream-K, model grid")
    out["grouped_hybrid_2tile"] = grouped_time(S.make_config(sched="2tsk"), "two-tile SK + DP")
    out["grouped_dp"] = grouped_time(S.make_config(sched="dp"), "data-parallel, one workgroup per tile")
    base = T.paper_baseline("bf16")
    out["grouped_paper_rule"] = grouped_time(base.config(), "paper rule: one tile, two-tile hybrid, model grid")
    if tune:
        tuner = T.Tuner()
        best = tuner.tune_grouped(descs, "bf16", "grouped512", reps=2)
        out["grouped_tuned"] = grouped_time(best.config(), "autotuned")
        out["grouped_tuned"]["choice"] = {"sched": best.sched, "blk": list(best.blk), "grid": best.grid,
                                          "threshold": best.threshold, "fixup": best.fixup, "split": best.split}
        out["speedup_tuned_vs_paper_rule"] = round(out["grouped_tuned"]["tflops"] /
                                                   out["grouped_paper_rule"]["tflops"], 3)
    best_g = max(v["tflops"] for k, v in out.items() if k.startswith("grouped_"))
    out["speedup_grouped_vs_separate"] = round(best_g / out["separate_launches"]["tflops"], 3)
    del sw
    torch.cuda.empty_cache()
    return out


def serving_leg(duration_s: float = 10.0, rate: float = 20000.0):
    """Poisson arrivals of mixed BF16/FP16 GEMMs (seed 4) through the
    continuous-batching server: p50/p99 latency and sustained TFLOP/s."""
    import torch
    import workloads as W
    from paper_2301_03598_amd import serve as SV
    trace = W.serving_trace(rate_per_s=rate, duration_s=duration_s, seed=4)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    pools = {}
    for dt in ("bf16", "f16"):
        t = torch.empty(1 << 28, dtype=W.torch_dtype(dt), device="cuda")
        t.normal_(0.0, 1.0, generator=gen)
        pools[dt] = t
    reqs = SV.make_requests(trace, pools, seed=4)
    srv = SV.Server(pools, hbm_budget=64 << 30, out_bytes=24 << 30, streams=2, max_batch=512)
    st = srv.run(reqs)
    offered = sum(r.flops for r in reqs) / duration_s / 1e12
    res = {"requests": st.requests, "completed": st.completed, "duration_s": duration_s,
           "offered_tflops": round(offered, 1), "sustained_tflops": round(st.sustained_tflops, 1),
           "makespan_s": round(st.makespan_s, 3), "p50_ms": round(st.p50_ms, 3),
           "p99_ms": round(st.p99_ms, 3), "launches": st.launches,
           "mean_batch": round(st.mean_batch, 1), "max_queue": st.max_queue,
           # requests queued or admitted but not launched, sampled every 10 ms:
           # here once per 0.5 s of the run
           "queue_depth_every_0.5s": st.queue_samples[::50],
           "keeps_up_with_offered_load": bool(st.sustained_tflops >= 0.95 * offered)}
    del pools, srv
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--extended", action="store_true")
    ap.add_argument("--gemm", nargs=4, metavar=("M", "N", "K", "AB"),
                    help="time one GEMM of the given shape and input dtype (default configuration) "
                         "and print its JSON; for profiling a single kernel")
    ap.add_argument("--gemm-flags", type=int, default=0,
                    help="SK_FLAG_* bits for --gemm (1: no XCD remap, 2: row-major tile order)")
    ap.add_argument("--gemm-ldc", type=int, default=0,
                    help="leading dimension of C for --gemm (0: n); rows that are not 16-byte aligned "
                         "take the epilogue that stores from the MFMA layout")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gemm:
        import torch
        from paper_2301_03598_amd import streamk as S
        S.lib()
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        m, n, k = (int(v) for v in args.gemm[:3])
        print(json.dumps(one_gemm(m, n, k, args.gemm[3], flags=args.gemm_flags, ldc=args.gemm_ldc)), flush=True)
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the Stream-K path shards by problem or by C slab, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2301_03598_amd import streamk as S
    S.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    shapes = W.sweep_shapes()
    log(f"sweep: {len(shapes)} problems; allocating operands")
    sweep = Sweep(shapes, "f16", "f32", seed=1)
    torch.cuda.synchronize()
    run = Runner(sweep, S.make_config(sched="auto"))
    kinds = {}
    for pl in run.plans:
        kinds[S.SCHED_NAME.get(pl.sched, str(pl.sched))] = kinds.get(S.SCHED_NAME.get(pl.sched, str(pl.sched)), 0) + 1
    tiles = {}
    for pl in run.plans:
        key = f"{pl.blk_m}x{pl.blk_n}x{pl.blk_k}"
        tiles[key] = tiles.get(key, 0) + 1
    log("schedules resolved:", kinds, "tiles:", tiles)

    for _ in range(args.warmup):
        run.step_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run.step_timed()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run.collect_timed()             # per-symbol GPU time of the timed steps
    ms_step = wall / args.steps * 1e3
    value = sweep.total_flops / (ms_step * 1e-3) / 1e12
    log(f"default sweep: {ms_step:.2f} ms/step, {value:.1f} TFLOP/s")
    lat = []
    run.step_events(lat)
    per = lat[0]
    lat_us = [x * 1e3 for x in per]
    tf = [sweep.flops[i] / (per[i] * 1e-3) / 1e12 for i in range(len(per))]

    compare = {}
    if not args.no_compare:
        legs = {}
        blk = (128, 128, 64)
        for name, sched in (("dp", "dp"), ("sk_basic", "sk"), ("hybrid_2tile", "2tsk"), ("dp_1tile_sk", "dp1sk")):
            res, tf_leg, run_leg = schedule_leg(sweep, S.make_config(sched=sched, blk=blk))
            legs[name] = (res, tf_leg)
            del run_leg
        # Algorithm 4 (fixed split) with the library's splitting factor per problem
        fs_cfgs, splits = fixed_split_configs(sweep, blk)
        res, tf_leg, run_leg = schedule_leg(sweep, fs_cfgs)
        res["split_histogram"] = {str(v): splits.count(v) for v in sorted(set(splits))}
        legs["fixed_split"] = (res, tf_leg)
        del run_leg
        # the idealized data-parallel ensemble over the library's tiles
        ens, tf_ens = ensemble_leg(sweep, [(256, 256, 64), (128, 128, 64), (64, 64, 64)])
        legs["dp_ensemble"] = (ens, tf_ens)
        compare = {k: v[0] for k, v in legs.items()}
        compare["default"] = {"tflops": round(value, 2), "geomean_tflops": round(geomean(tf), 2),
                              "pct_peak": round(100 * value / PEAK_TFLOPS["f16"], 2)}
        compare["tile_of_schedule_legs"] = "128x128x64"
        tf_dp = legs["dp"][1]
        for name, tfl in [("default", tf)] + [(k, v[1]) for k, v in legs.items() if k != "dp"]:
            compare[f"geomean_speedup_{name}_vs_dp"] = round(geomean([a / b for a, b in zip(tfl, tf_dp)]), 3)
        for name, tfl in (("default", tf), ("sk_basic", legs["sk_basic"][1])):
            compare[f"geomean_speedup_{name}_vs_dp_ensemble"] = \
                round(geomean([a / b for a, b in zip(tfl, tf_ens)]), 3)
        compare["min_speedup_default_vs_dp"] = round(min(a / b for a, b in zip(tf, tf_dp)), 3)
        compare["max_speedup_default_vs_dp"] = round(max(a / b for a, b in zip(tf, tf_dp)), 3)
        log("compare:", compare)
    # the dominant kernel: the symbol with the most GPU time in the timed
    # steps; its launches ran back to back between two events in each step
    kname = max(run.group_ms, key=lambda k: run.group_ms[k])
    idx = run.groups[kname]
    klaunch = len(idx) * run.group_steps
    avg_ms = run.group_ms[kname] / klaunch
    avg_flops = sum(sweep.flops[i] for i in idx) / len(idx)
    achieved = avg_flops / (avg_ms * 1e-3) / 1e12
    total_ms = sum(run.group_ms.values())
    # the attainable rate of each of those launches, min(MFMA peak, AI x HBM
    # bandwidth): most sweep problems sit below the ridge point, where the
    # MFMA fraction alone understates how close a launch is to its bound
    att_ms = sum(sweep.flops[i] / (attainable_tflops(*sweep.shapes[i], 2, 4, PEAK_TFLOPS["f16"]) * 1e12) * 1e3
                 for i in idx)
    below_ridge = sum(1 for i in idx if attainable_tflops(*sweep.shapes[i], 2, 4, PEAK_TFLOPS["f16"])
                      < PEAK_TFLOPS["f16"])
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS["f16"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f16"], 4),
                "frac_of_attainable": round(att_ms / (avg_ms * len(idx)), 4),
                "launches_below_ridge": f"{below_ridge} of {len(idx)} problems",
                "traffic": measured_traffic(kname),
                "kernel": kname, "launches": klaunch, "avg_launch_us": round(avg_ms * 1e3, 3),
                "avg_flops_per_launch": avg_flops, "time_share": round(run.group_ms[kname] / total_ms, 3),
                "per_kernel_avg_us": {k: round(run.group_ms[k] * 1e3 / (len(run.groups[k]) * run.group_steps), 3)
                                      for k in run.groups}}
    # the same figures for every kernel symbol: when several carry nearly
    # equal shares of the sweep's time, which one is dominant can change
    # from run to run
    per_kernel = {}
    for k, ids in run.groups.items():
        k_ms = run.group_ms[k] / (len(ids) * run.group_steps)
        k_flops = sum(sweep.flops[i] for i in ids) / len(ids)
        k_att = sum(sweep.flops[i] / (attainable_tflops(*sweep.shapes[i], 2, 4, PEAK_TFLOPS["f16"]) * 1e12) * 1e3
                    for i in ids)
        per_kernel[k] = {"time_share": round(run.group_ms[k] / total_ms, 3),
                         "frac": round(k_flops / (k_ms * 1e-3) / 1e12 / PEAK_TFLOPS["f16"], 4),
                         "frac_of_attainable": round(k_att / (k_ms * len(ids)), 4)}
    roofline["per_kernel"] = per_kernel

    ext = None
    total_flops = sweep.total_flops
    if args.extended:
        del sweep, run
        torch.cuda.empty_cache()
        ext = extended()
        ext["grouped"] = grouped_leg()
        log("grouped:", ext["grouped"])
        ext["serving"] = serving_leg()
        # the same stream at half the rate: below what the GPU sustains on
        # this mix, so the latencies are those of an unsaturated server
        ext["serving_half_rate"] = serving_leg(rate=10000.0)
        log("serving:", ext["serving"], "half rate:", ext["serving_half_rate"])
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    if cpu:
        log("cpu baseline:", cpu)

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "geometry sweep: 2048 GEMMs, m,n,k log-uniform in [128,8192] rounded "
                               "to multiples of 8 (seed 1); FP16 inputs U[-1,1], FP32 accumulate "
                               "and output; alpha=1, beta=0; row-major; library default configuration "
                               "per problem (tile 64x64, 128x128 or 256x256 by size and depth; "
                               "data-parallel, k-aligned fixed split, basic Stream-K, or data-parallel "
                               "waves with a fixed-split tail; counts in 'tiles' and 'schedules')",
                   "problems": len(shapes), "flops_per_step": total_flops,
                   "tiles": tiles, "schedules": kinds},
        "pct_peak": round(100 * value / PEAK_TFLOPS["f16"], 2),
        "latency_us": {"p50": round(pct(lat_us, 50), 2), "p99": round(pct(lat_us, 99), 2)},
        "geomean_tflops": round(geomean(tf), 2),
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if ext is not None:
        line["extended"] = ext
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
