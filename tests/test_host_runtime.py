"""Host-side pieces of the runtime that need no GPU: the serving loop's
output-arena allocator and the autotuner's shape buckets."""
import random

import pytest

torch = pytest.importorskip("torch")

from paper_2301_03598_amd import serve as SV
from paper_2301_03598_amd import tune as T


def test_arena_first_fit_and_coalescing():
    a = SV.Arena(1 << 16, device="cpu")
    o1 = a.alloc(1000)          # rounds to 1024
    o2 = a.alloc(256)
    o3 = a.alloc(4096)
    assert (o1, o2, o3) == (0, 1024, 1280)
    a.release(o2, 256)
    assert a.alloc(200) == 1024             # first fit reuses the hole
    a.release(1024, 200)
    a.release(o1, 1000)
    a.release(o3, 4096)
    assert a.free == [(0, 1 << 16)]         # everything coalesced back


def test_arena_random_never_overlaps():
    rng = random.Random(0)
    a = SV.Arena(1 << 20, device="cpu")
    live = {}
    for step in range(2000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            a.release(off, live.pop(off))
        else:
            n = rng.randint(1, 20000)
            off = a.alloc(n)
            if off is None:
                continue
            size = (n + 255) // 256 * 256
            for o, s in live.items():
                s = (s + 255) // 256 * 256
                assert off + size <= o or o + s <= off
            live[off] = n
    for off, n in list(live.items()):
        a.release(off, n)
    assert a.free == [(0, 1 << 20)]


def test_served_bytes_and_flops():
    r = SV.Served(0, 128, 256, 512, "bf16", 0.0)
    assert r.flops == 2.0 * 128 * 256 * 512
    assert r.nbytes(2, 4) == (128 * 512 + 512 * 256) * 2 + 128 * 256 * 4


def test_tuner_buckets():
    assert T.bucket("bf16", 1024, 1024, 1024) == "bf16:10:10:10"
    assert T.bucket("bf16", 1400, 1024, 1024) == T.bucket("bf16", 1024, 1024, 1024)
    assert T.bucket("f64", 128, 8192, 3000) == "f64:7:13:12"
    cands = T.Tuner.candidates("bf16", {(256, 256, 64): 256, (128, 128, 64): 512})
    assert any(c.sched == "dp" for c in cands) and any(c.sched == "sk" and c.grid == 512 for c in cands)
    assert {c.blk for c in cands} == {(256, 256, 64), (128, 128, 64), (64, 64, 64)}
    # the paper's configuration comes first: one tile per precision, the
    # two-tile hybrid, the model's grid
    assert (cands[0].sched, cands[0].blk, cands[0].grid) == ("2tsk", (256, 256, 64), 0)
    assert {c.fixup for c in cands if c.sched == "sk"} == {"serial", "spread"}
