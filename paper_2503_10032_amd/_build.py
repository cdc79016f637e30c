"""Compile the HIP library (libddelm.so) for gfx950 with hipcc, in place.

Every source is compiled to an object of its own, in parallel (the panel and
CG kernel instantiations sit in separate units for this), then the objects
are linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libddelm.so")
CSRC = os.path.join(HERE, "csrc")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [os.path.join(CSRC, "geometry.cpp")]


COMPILE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source into libddelm.so; returns the library path."""
    cc = hipcc()
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), len(os.sched_getaffinity(0)), 16))
    with tempfile.TemporaryDirectory(prefix="ddelm_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in srcs]
        with cf.ThreadPoolExecutor(jobs) as ex:
            futs = [ex.submit(_run, [cc] + COMPILE_FLAGS + ["-c", s, "-o", o], verbose) for s, o in zip(srcs, objs)]
            for f in futs:
                f.result()
        out = LIB + ".tmp"
        _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", out], verbose)
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
