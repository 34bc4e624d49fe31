"""Build libstreamk.so (gfx950) in-tree with hipcc.

Each kernel-instance unit compiles in its own hipcc process, in parallel;
the objects are linked into ``paper_2301_03598_amd/libstreamk.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libstreamk.so")
ARCH = "gfx950"

CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    f"-I{INCLUDE}", f"-I{CSRC}",
    # no packed-FP32 VALU forms anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h*")) + [os.path.join(INCLUDE, "streamk.h")]


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *_headers()])


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = ["hipcc", *CXXFLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def sync_generated() -> int:
    """Rewrite every generated kernel-instance unit (and the lookup table)
    whose content differs from what gen_instances.py produces now, and
    remove stale units; returns the number of files changed."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_instances", os.path.join(CSRC, "gen_instances.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    want = gen.expected()
    changed = 0
    for f in os.listdir(CSRC):
        if f.startswith("inst_") and f.endswith(".hip") and f not in want:
            os.remove(os.path.join(CSRC, f))
            changed += 1
    for name, text in want.items():
        path = os.path.join(CSRC, name)
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as fh:
                fh.write(text)
            changed += 1
    return changed


def build(jobs: int = 0, verbose: bool = True, force: bool = True) -> str:
    """Regenerate the instance units if they drifted from their generator,
    compile every unit (``force=False``: only those older than their
    sources or headers) and link the library."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    n = sync_generated()
    if verbose and n:
        print(f"[build] {n} generated unit(s) rewritten from gen_instances.py", flush=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB} from {len(srcs)} units in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("-")]
    build(int(args[0]) if args else 0, force="--incremental" not in sys.argv)
