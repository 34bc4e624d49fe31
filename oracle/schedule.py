"""Schedule oracle (pure integer) -- TEST INFRASTRUCTURE ONLY.

States, for a GEMM (or a group of GEMMs) and a launch configuration, which
workgroup performs which MAC-loop iterations of which output tile and how
partial sums are reconciled.  It follows the paper directly:

* geometry: tiles ceil(m/BLK_M) x ceil(n/BLK_N), ceil(k/BLK_K) MAC-loop
  iterations per tile (Algorithm 2 and Algorithm 5 preamble);
* basic Stream-K (section 4, Algorithm 5): the m->n->k linearised iteration
  space is split evenly over g workgroups, each range walked tile by tile;
  the workgroup that ran a tile's k=0 iteration writes it after adding the
  partial sums of the later contributors;
* hybrids (section 5.2): "DP + one-tile SK" and "two-tile SK + DP";
* grid-size model (appendix A.1): time(g) = a + b[peers>1] + c*ItersPerCta(g)
  + d*(peers-1);
* fixed split (section 3.3, Algorithm 4) for the generalisation check.

Readings where the paper is silent or garbled (each is listed in the design
notes with its reason):
* tiles are linearised row-major, n fastest (Algorithm 3 divides by the
  m-tile count for both coordinates, which cannot be right when the tile grid
  is not square);
* the even share "within one": q = T // g, r = T % g, and the first r
  workgroups take q+1 iterations (Algorithm 5's ceil form would leave the last
  workgroup short, contradicting "132/133 iterations per CTA" in Fig. 7);
* the peers of an owner are the workgroups x+1 .. owner_of(last iteration of
  the tile) (Algorithm 5's loop bound yields a tile index, not a workgroup);
* hybrids: with w = t // p full waves and r = t % p: r == 0 -> all tiles
  data-parallel on g = p (or the caller's grid); w == 0 -> basic Stream-K with the model's g;
  otherwise two-tile SK+DP when w >= threshold (default 2): SK over the first
  r + p tiles, then DP over the rest; else DP + one-tile SK: DP over the
  first w*p tiles, then SK over the last r tiles, g = p;
* ties in the grid model go to the smallest g.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

ROLE_DP, ROLE_FULL, ROLE_OWNER, ROLE_PRODUCER = 0, 1, 2, 3
ROLE_NAMES = {ROLE_DP: "dp", ROLE_FULL: "full", ROLE_OWNER: "owner", ROLE_PRODUCER: "producer"}

SCHED_DP, SCHED_SK, SCHED_DP1, SCHED_2T = 1, 2, 3, 4


def cdiv(a: int, b: int) -> int:
    return -(-a // b)


@dataclass(frozen=True)
class Geometry:
    tiles_m: int
    tiles_n: int
    t: int          # output tiles
    I: int          # MAC-loop iterations per tile
    T: int          # total iterations


def geometry(m: int, n: int, k: int, blk_m: int, blk_n: int, blk_k: int) -> Geometry:
    tm, tn = cdiv(m, blk_m), cdiv(n, blk_n)
    t = tm * tn
    I = cdiv(k, blk_k)
    return Geometry(tm, tn, t, I, t * I)


def tile_coords(tile: int, tiles_n: int) -> Tuple[int, int]:
    """Row-major tile linearisation, n fastest."""
    return tile // tiles_n, tile % tiles_n


# ---------------------------------------------------------------------------
# even partition of an iteration range over g workgroups
# ---------------------------------------------------------------------------

def wg_range(x: int, total: int, g: int) -> Tuple[int, int]:
    q, r = divmod(total, g)
    b = x * q + min(x, r)
    return b, b + q + (1 if x < r else 0)


def owner_of(i: int, total: int, g: int) -> int:
    """The workgroup whose range holds iteration i (relative to the range start)."""
    q, r = divmod(total, g)
    if i < r * (q + 1):
        return i // (q + 1)
    return r + (i - r * (q + 1)) // q


# ---------------------------------------------------------------------------
# the plan: how tiles split into a Stream-K region and data-parallel tiles
# ---------------------------------------------------------------------------

@dataclass
class Plan:
    g: int                      # workgroups launched
    sk_tile_begin: int          # SK region [begin, end) in tile order
    sk_tile_end: int
    dp_first: bool              # DP tiles before the SK segments in each WG
    sched: int                  # resolved schedule
    tiles: int
    dp_tiles: List[int] = field(default_factory=list)


def model_time(g: int, T: int, I: int, a: float, b: float, c: float, d: float) -> float:
    ipc = cdiv(T, g)
    peers = cdiv(I, ipc)
    return a + b * (1 if peers > 1 else 0) + c * ipc + d * (peers - 1)


def choose_grid(T: int, I: int, p: int, consts: Tuple[float, float, float, float]) -> int:
    """g* = argmin over g in [1, min(p, T)] of the appendix A.1 model; ties
    resolve to the smallest g."""
    a, b, c, d = consts
    best_g, best = 1, None
    for g in range(1, max(1, min(p, T)) + 1):
        v = model_time(g, T, I, a, b, c, d)
        if best is None or v < best:
            best, best_g = v, g
    return best_g


def make_plan(tiles: int, T_of_region, I_max: int, p: int, sched: int,
              grid: int = 0, consts=(0.0, 10.0, 1.0, 8.5), threshold: int = 2) -> Plan:
    """The plan of one of the paper's four schedules: data-parallel
    (Algorithm 2), basic Stream-K (Algorithm 5, appendix A.1 grid) and the
    two hybrids of section 5.2.  ``T_of_region(tb, te)`` returns the
    iteration count of tiles [tb, te).  A library's own automatic choice among
    them is not a passage of the paper, so it has no oracle: asking for it
    raises."""
    if sched not in (SCHED_DP, SCHED_SK, SCHED_DP1, SCHED_2T):
        raise ValueError(f"schedule {sched} is not one of the paper's (DP, SK, DP+1-tile SK, 2-tile SK+DP)")
    t = tiles
    if t == 0:
        return Plan(0, 0, 0, False, sched, 0, [])
    if sched == SCHED_DP:
        return Plan(t, 0, 0, True, SCHED_DP, t, list(range(t)))
    if sched == SCHED_SK:
        T = T_of_region(0, t)
        g = grid if grid > 0 else choose_grid(T, I_max, p, consts)
        g = max(1, min(g, T))
        return Plan(g, 0, t, False, SCHED_SK, t, [])
    w, r = divmod(t, p)
    if r == 0:
        # perfect quantisation: full data-parallel waves on the whole machine
        # (a hybrid whose Stream-K region is empty); a caller-given grid
        # replaces p here as in every persistent schedule
        return Plan(grid if grid > 0 else p, 0, 0, True, SCHED_DP1, t, list(range(t)))
    if w == 0:
        # no full wave: basic Stream-K with the model's grid size
        T = T_of_region(0, t)
        g = grid if grid > 0 else choose_grid(T, I_max, p, consts)
        g = max(1, min(g, T))
        return Plan(g, 0, t, False, SCHED_SK, t, [])
    # a hybrid's grid carries its data-parallel waves too: it stays p (or the
    # caller's grid) even when the Stream-K region has fewer iterations, in
    # which case some workgroups get an empty Stream-K range
    g = grid if grid > 0 else p
    if sched == SCHED_2T and w >= threshold:
        te = r + p
        return Plan(g, 0, te, False, SCHED_2T, t, list(range(te, t)))
    # DP + one-tile SK
    tb = w * p
    return Plan(g, tb, t, True, SCHED_DP1, t, list(range(0, tb)))


# ---------------------------------------------------------------------------
# per-workgroup segment lists
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Segment:
    wg: int
    tile: int
    k_begin: int   # MAC-loop iteration within the tile (inclusive)
    k_end: int     # exclusive
    role: int
    peers: Tuple[int, ...] = ()


class Problems:
    """Concatenated iteration space of one or more GEMMs (problem index
    outermost, then tile, then k)."""

    def __init__(self, tiles_and_iters: Sequence[Tuple[int, int]]):
        self.tp = [t for t, _ in tiles_and_iters]
        self.Ip = [I for _, I in tiles_and_iters]
        self.tile_prefix = [0]
        self.iter_prefix = [0]
        for t, I in tiles_and_iters:
            self.tile_prefix.append(self.tile_prefix[-1] + t)
            self.iter_prefix.append(self.iter_prefix[-1] + t * I)
        self.tiles = self.tile_prefix[-1]
        self.total = self.iter_prefix[-1]

    def problem_of_tile(self, tile: int) -> int:
        lo, hi = 0, len(self.tp)
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if self.tile_prefix[mid] <= tile:
                lo = mid
            else:
                hi = mid
        return lo

    def tile_iter_begin(self, tile: int) -> int:
        p = self.problem_of_tile(tile)
        return self.iter_prefix[p] + (tile - self.tile_prefix[p]) * self.Ip[p]

    def iters_of_tile(self, tile: int) -> int:
        return self.Ip[self.problem_of_tile(tile)]

    def tile_of_iter(self, it: int) -> int:
        lo, hi = 0, len(self.tp)
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if self.iter_prefix[mid] <= it:
                lo = mid
            else:
                hi = mid
        # skip problems with zero iterations (k == 0 cannot occur here)
        return self.tile_prefix[lo] + (it - self.iter_prefix[lo]) // self.Ip[lo]

    def region_iters(self, tb: int, te: int) -> int:
        if te <= tb:
            return 0
        return self.tile_iter_begin(te - 1) + self.iters_of_tile(te - 1) - self.tile_iter_begin(tb)


def plan_problems(probs: Problems, p: int, sched: int, grid: int = 0,
                  consts=(0.0, 10.0, 1.0, 8.5), threshold: int = 2) -> Plan:
    # the model's per-tile iteration count is that of the deepest tile that
    # exists: a problem with no output tiles has no MAC-loop iterations
    depth = max((I for t, I in zip(probs.tp, probs.Ip) if t > 0), default=0)
    return make_plan(probs.tiles, probs.region_iters, depth, p, sched, grid, consts, threshold)


def segments(probs: Problems, plan: Plan) -> List[List[Segment]]:
    """Ordered segment list of every workgroup."""
    g = plan.g
    out: List[List[Segment]] = [[] for _ in range(g)]
    if g == 0:
        return out
    sk: List[List[Segment]] = [[] for _ in range(g)]
    if plan.sk_tile_end > plan.sk_tile_begin:
        base = probs.tile_iter_begin(plan.sk_tile_begin)
        total = probs.region_iters(plan.sk_tile_begin, plan.sk_tile_end)
        for x in range(g):
            b, e = wg_range(x, total, g)
            it = b
            while it < e:
                tile = probs.tile_of_iter(base + it)
                t0 = probs.tile_iter_begin(tile) - base
                t1 = t0 + probs.iters_of_tile(tile)
                k0, k1 = it - t0, min(e, t1) - t0
                started, ended = it == t0, e >= t1
                if not started:
                    seg = Segment(x, tile, k0, k1, ROLE_PRODUCER)
                elif ended:
                    seg = Segment(x, tile, k0, k1, ROLE_FULL)
                else:
                    last = owner_of(t1 - 1, total, g)
                    seg = Segment(x, tile, k0, k1, ROLE_OWNER, tuple(range(x + 1, last + 1)))
                sk[x].append(seg)
                it = t1
    dp: List[List[Segment]] = [[] for _ in range(g)]
    for j, tile in enumerate(plan.dp_tiles):
        x = j % g
        dp[x].append(Segment(x, tile, 0, probs.iters_of_tile(tile), ROLE_DP))
    for x in range(g):
        out[x] = (dp[x] + sk[x]) if plan.dp_first else (sk[x] + dp[x])
    return out


def single(m, n, k, blk) -> Problems:
    geo = geometry(m, n, k, *blk)
    return Problems([(geo.t, geo.I)])


def fixed_split_segments(t: int, I: int, s: int) -> List[List[Segment]]:
    """Algorithm 4: s workgroups per tile, workgroup (x, y) -> index x*s + y."""
    ips = cdiv(I, s)
    out = []
    for x in range(t):
        for y in range(s):
            b = y * ips
            e = min(I, b + ips)
            wg = x * s + y
            if y != 0:
                out.append([Segment(wg, x, b, e, ROLE_PRODUCER)] if e > b else [])
            else:
                peers = tuple(x * s + yy for yy in range(1, s) if yy * ips < I)
                role = ROLE_OWNER if peers else ROLE_FULL
                out.append([Segment(wg, x, b, e, role, peers)])
    return out


def dp_ceiling(t: int, p: int) -> float:
    """Utilisation ceiling of a data-parallel schedule: t / (p * waves)."""
    return t / (p * cdiv(t, p))


def check_invariants(probs: Problems, plan: Plan, segs: List[List[Segment]]) -> None:
    """Raise AssertionError unless the schedule covers every (tile, k-iteration)
    exactly once, every workgroup stores at most one partial, every producer
    is consumed by exactly one owner, and owners precede their peers."""
    cover: Dict[int, List[Tuple[int, int]]] = {}
    producers = {}
    consumed = {}
    for x, lst in enumerate(segs):
        nprod = 0
        for s in lst:
            cover.setdefault(s.tile, []).append((s.k_begin, s.k_end))
            if s.role == ROLE_PRODUCER:
                nprod += 1
                producers[x] = s
            if s.role == ROLE_OWNER:
                for pr in s.peers:
                    assert pr > x
                    assert pr not in consumed, "partial consumed twice"
                    consumed[pr] = s.tile
        assert nprod <= 1, f"workgroup {x} stores {nprod} partials"
    for tile in range(probs.tiles):
        rngs = sorted(cover.get(tile, []))
        assert rngs, f"tile {tile} uncovered"
        pos = 0
        for b, e in rngs:
            assert b == pos, f"tile {tile}: gap/overlap at {pos} vs {b}"
            assert e > b
            pos = e
        assert pos == probs.iters_of_tile(tile), f"tile {tile} ends at {pos}"
    assert set(producers) == set(consumed), "producer without an owner"
    for x, s in producers.items():
        assert consumed[x] == s.tile
