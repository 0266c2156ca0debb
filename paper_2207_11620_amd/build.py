"""Build libngvol.so (all HIP sources under csrc/) for gfx950 with hipcc.

Run as ``python -m paper_2207_11620_amd.build``; object files go to
``_build/`` and the library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libngvol.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # binary32 geometry, exact level floors and RNG are written op by op
    "-ffp-contract=off",
    # hardware FP32 atomic add for the scatter into the table gradient
    "-munsafe-fp-atomics",
    # no packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", INCLUDE, "-I", CSRC,
]


# Sources carrying this line are compiled once per MLP precision and width,
# with -DNGV_PSEL=0, 1, 2 and -DNGV_WSEL=32, 64: their kernel instantiations
# are split over six objects that build in parallel.
PSEL_MARK = "// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)"


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def units():
    """(source, precision selector or None) for every object of the library."""
    out = []
    for src in sources():
        with open(src) as fh:
            split = PSEL_MARK in fh.read()
        if split:
            out.extend((src, (p, w)) for p in (0, 1, 2) for w in (64, 32))
        else:
            out.append((src, None))
    # the slowest objects (FP32, width 64) first, so that they do not start last
    return sorted(out, key=lambda u: (u[1] is None, u[1] or (0, 0), u[0]))


def _deps_mtime() -> float:
    """Latest modification time of the headers and build settings every object depends on."""
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    deps.append(os.path.abspath(__file__))
    return max(os.path.getmtime(d) for d in deps)


def _compile(unit, force: bool = True, deps: float = 0.0) -> str:
    src, psel = unit
    name = os.path.basename(src) + ("" if psel is None else f".p{psel[0]}w{psel[1]}")
    obj = os.path.join(BUILD, name + ".o")
    if not force and os.path.exists(obj) and os.path.getmtime(obj) > max(deps, os.path.getmtime(src)):
        return obj
    sel = [] if psel is None else [f"-DNGV_PSEL={psel[0]}", f"-DNGV_WSEL={psel[1]}"]
    cmd = ["hipcc", *FLAGS, *sel, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    if os.environ.get("NGVOL_BUILD_TIMES"):
        print(f"  {name}: {time.time() - t0:.0f} s", flush=True)
    return obj


def build(jobs: int | None = None, verbose: bool = True, force: bool = True) -> str:
    """Compile every object (force) or only those older than their sources and headers, then link."""
    os.makedirs(BUILD, exist_ok=True)
    us = units()
    deps = _deps_mtime()
    jobs = jobs or min(len(us), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, force, deps), us))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    # `python -m paper_2207_11620_amd.build` rebuilds only what changed; `--force` everything
    build(force="--force" in sys.argv)
    sys.exit(0)
