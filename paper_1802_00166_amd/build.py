"""Builds libpcot.so (all HIP kernels and the C ABI) for gfx950 with hipcc.

Objects go to _build/ at the repository root; the library is written next to
this file, where the Python binding loads it.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpcot.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("PCOT_ARCH", "gfx950")

# -ffp-contract=off: the update rules fix the operation order, no fused
# multiply-add.  Packed FP32 instructions are disabled for every HIP source.
CXXFLAGS = ["-std=c++17", "-O3", "-fPIC", "-ffp-contract=off", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas", "-I" + os.path.join(ROOT, "include")]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc()] + CXXFLAGS + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, r.stdout))
    warn = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and verbose:
        print(warn)
    return obj


def _includes(path: str, seen=None) -> set:
    """Local headers a source includes, followed transitively."""
    import re
    seen = set() if seen is None else seen
    with open(path) as f:
        for name in re.findall(r'^#include "([^"]+)"', f.read(), re.M):
            for d in (os.path.dirname(path), CSRC, os.path.join(ROOT, "include")):
                p = os.path.join(d, name)
                if os.path.exists(p) and p not in seen:
                    seen.add(p)
                    _includes(p, seen)
                    break
    return seen


def _stale(src: str) -> bool:
    """Object missing or older than its source or any header it includes."""
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    deps = [src] + sorted(_includes(src))
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compiles every source (incremental=True: only stale objects) and links."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
