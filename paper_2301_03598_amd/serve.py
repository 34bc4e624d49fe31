"""Continuous-batching GEMM serving over grouped Stream-K launches.

Requests (m, n, k, dtype) arrive over time.  The host loop
  1. moves arrived requests into the queue,
  2. admits queued requests while their operand and output bytes fit the
     HBM budget (memory is released when a request completes),
  3. packs admitted requests of one dtype into the next grouped launch
     (sk_gemm_grouped) on any idle stream, so work that arrives while other
     launches run is admitted and overlaps with them on the device,
  4. polls completion events and records each request's latency.

Concurrent persistent launches share the machine: each launch takes the tile
the library picks for its batch on the whole machine and is planned on
1 / streams of the resident slots of that tile's kernel, so every workgroup
of every launch in flight is co-resident and the Stream-K fixup waits always
make progress.  A wait that gives up anyway (its bound is real time) is
reported when the loop ends: the run raises SkError(SK_ERR_TIMEOUT) instead
of returning results that a fixup did not complete.

Operands come from per-dtype device pools filled once (no host-to-device
copies in the serving path); each request reads its own window of the pool
and writes its own output buffer.
"""
from __future__ import annotations

import bisect
import collections
import ctypes
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import torch

from . import runtime as R
from . import streamk as S

C_TYPE = {"bf16": "f32", "f16": "f32"}


class Arena:
    """First-fit allocator over one device buffer (256-byte granules)."""

    def __init__(self, nbytes: int, dtype=torch.uint8, device="cuda"):
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.free = [(0, nbytes)]            # sorted (offset, size)

    def alloc(self, nbytes: int) -> Optional[int]:
        nbytes = (nbytes + 255) // 256 * 256
        for i, (o, s) in enumerate(self.free):
            if s >= nbytes:
                if s == nbytes:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + nbytes, s - nbytes)
                return o
        return None

    def release(self, off: int, nbytes: int) -> None:
        nbytes = (nbytes + 255) // 256 * 256
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, nbytes))
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


@dataclass
class Served:
    rid: int
    m: int
    n: int
    k: int
    dtype: str
    arrival: float
    a_off: int = 0
    b_off: int = 0
    c_off: int = -1
    admitted: float = -1.0
    launched: float = -1.0
    done: float = -1.0
    batch: int = -1

    @property
    def flops(self) -> float:
        return 2.0 * self.m * self.n * self.k

    def nbytes(self, eb: int, cb: int) -> int:
        return (self.m * self.k + self.k * self.n) * eb + self.m * self.n * cb


@dataclass
class ServeStats:
    requests: int
    completed: int
    makespan_s: float
    sustained_tflops: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    launches: int
    max_queue: int
    queue_samples: List[int] = field(default_factory=list)


class Server:
    def __init__(self, pools: Dict[str, torch.Tensor], hbm_budget: int = 64 << 30,
                 out_bytes: int = 8 << 30, streams: int = 2, max_batch: int = 512,
                 max_batch_flops: float = 5e11, cfg_for: Optional[callable] = None):
        self.pools = pools                    # dtype -> flat device tensor of operand values
        self.budget = hbm_budget
        self.arena = Arena(out_bytes)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.ws = [R.Workspace("cuda") for _ in range(streams)]
        self.max_batch = max_batch
        self.max_batch_flops = max_batch_flops
        self.cfg_for = cfg_for
        self.slots: Dict[tuple, int] = {}

    # -- helpers -----------------------------------------------------------
    def _share(self, dtype: str, descs, cfg: S.sk_config_t) -> S.sk_config_t:
        """cfg with the batch's tile fixed (the library's choice on the whole
        machine unless cfg names one) and wg_slots set to this launch's share
        of that tile's kernel's resident slots."""
        if not (cfg.blk_m or cfg.blk_n or cfg.blk_k):
            st, pl = S.sk_plan(descs, cfg)
            S.check(st, "sk_plan")
            cfg.blk_m, cfg.blk_n, cfg.blk_k = pl.blk_m, pl.blk_n, pl.blk_k
        key = (dtype, cfg.blk_m, cfg.blk_n, cfg.blk_k)
        if key not in self.slots:
            # (a one-workgroup Stream-K plan reports the kernel's slots)
            st, pl = S.sk_plan(descs, S.make_config(sched="sk", blk=(cfg.blk_m, cfg.blk_n, cfg.blk_k), grid=1))
            S.check(st, "sk_plan")
            self.slots[key] = pl.wg_slots
        cfg.wg_slots = max(1, self.slots[key] // len(self.streams))
        cfg.grid = min(cfg.grid, cfg.wg_slots)
        return cfg

    def _desc(self, r: Served) -> S.sk_gemm_desc_t:
        pool = self.pools[r.dtype]
        eb = pool.element_size()
        return S.make_desc(r.m, r.n, r.k, pool.data_ptr() + r.a_off * eb, pool.data_ptr() + r.b_off * eb,
                           self.arena.base + r.c_off, ab_type=r.dtype, c_type=C_TYPE[r.dtype])

    def output(self, r: Served) -> torch.Tensor:
        """The request's result (m x n FP32 view of the output arena)."""
        n = r.m * r.n
        t = self.arena.buf[r.c_off:r.c_off + 4 * n].view(torch.float32)
        return t.view(r.m, r.n)

    # -- the loop ------------------------------------------------------------
    def run(self, reqs: Sequence[Served], time_scale: float = 1.0, keep_outputs: bool = False) -> ServeStats:
        pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        admitted: Dict[str, collections.deque] = {d: collections.deque() for d in self.pools}
        inflight: List[Optional[tuple]] = [None] * len(self.streams)
        used = 0
        launches = 0
        max_q = 0
        qsamples = []
        done: List[Served] = []
        used_streams = set()
        t0 = time.perf_counter()
        next_sample = 0.0
        while pending or queue or any(admitted.values()) or any(x is not None for x in inflight):
            now = (time.perf_counter() - t0) / time_scale
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission against the HBM budget
            while queue:
                r = queue[0]
                eb = self.pools[r.dtype].element_size()
                need = r.nbytes(eb, 4)
                if used + need > self.budget:
                    break
                off = self.arena.alloc(4 * r.m * r.n)
                if off is None:
                    break
                queue.popleft()
                r.c_off = off
                r.admitted = now
                used += need
                admitted[r.dtype].append(r)
            depth = len(queue) + sum(len(v) for v in admitted.values())
            max_q = max(max_q, depth)
            if now >= next_sample:
                qsamples.append(depth)
                next_sample += 0.01
            # completions
            for si, entry in enumerate(inflight):
                if entry is not None and entry[0].query():
                    tdone = (time.perf_counter() - t0) / time_scale
                    for r in entry[1]:
                        r.done = tdone
                        eb = self.pools[r.dtype].element_size()
                        used -= r.nbytes(eb, 4)
                        if not keep_outputs:
                            self.arena.release(r.c_off, 4 * r.m * r.n)
                        done.append(r)
                    inflight[si] = None
            # launches on idle streams
            for si in range(len(self.streams)):
                if inflight[si] is not None:
                    continue
                cands = [d for d in admitted if admitted[d]]
                if not cands:
                    break
                dt = min(cands, key=lambda d: admitted[d][0].arrival)
                batch, fl = [], 0.0
                while admitted[dt] and len(batch) < self.max_batch and (not batch or fl < self.max_batch_flops):
                    r = admitted[dt].popleft()
                    batch.append(r)
                    fl += r.flops
                descs = [self._desc(r) for r in batch]
                cfg = self.cfg_for(dt, batch) if self.cfg_for else S.make_config()
                cfg = self._share(dt, descs, cfg)
                stream = self.streams[si]
                plan, keep = R.gemm_grouped(descs, cfg=cfg, ws=self.ws[si], stream=stream)
                used_streams.add(si)
                ev = torch.cuda.Event()
                ev.record(stream)
                tl = (time.perf_counter() - t0) / time_scale
                for r in batch:
                    r.launched = tl
                    r.batch = launches
                inflight[si] = (ev, batch, keep)
                launches += 1
        end = (time.perf_counter() - t0) / time_scale
        # a fixup wait that gave up in any launch of a stream: raise
        for si in sorted(used_streams):
            self.ws[si].check(self.streams[si].cuda_stream)
        lat = sorted((r.done - r.arrival) * 1e3 for r in done)

        def pct(q):
            return lat[min(len(lat) - 1, max(0, int(math.ceil(q / 100 * len(lat))) - 1))] if lat else 0.0
        first = min((r.arrival for r in done), default=0.0)
        span = max(end - first, 1e-9)
        total = sum(r.flops for r in done)
        sizes = collections.Counter(r.batch for r in done)
        return ServeStats(len(reqs), len(done), span, total / span / 1e12, pct(50), pct(99),
                          sum(sizes.values()) / max(1, len(sizes)), launches, max_q, qsamples)


def make_requests(trace, pools: Dict[str, torch.Tensor], seed: int = 0) -> List[Served]:
    """Attach pool windows to workload requests (workloads.Request)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for r in trace:
        pool = pools[r.dtype]
        total = pool.numel()
        na, nb = r.m * r.k, r.k * r.n
        # 16-byte aligned element offsets inside the pool
        a_off = int(rng.integers(0, max(1, (total - na) // 8))) * 8
        b_off = int(rng.integers(0, max(1, (total - nb) // 8))) * 8
        out.append(Served(r.rid, r.m, r.n, r.k, r.dtype, r.arrival_s, a_off, b_off))
    return out
