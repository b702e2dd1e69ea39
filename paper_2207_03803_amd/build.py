"""Build libgap.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2207_03803_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgap.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["knm.hip", "knm_lp.hip", "knm_oz.hip", "cur.hip", "potrf.hip", "geqrf.hip", "cqr.hip", "trsv.hip", "refine.hip", "diag.hip", "capi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "'-packed-fp32-ops' is not a recognized feature"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, OUT)
    # the roofline microbenchmarks (a standalone program)
    peaks = os.path.join(HERE, "gap_peaks")
    r = subprocess.run([HIPCC, *FLAGS, os.path.join(CSRC, "peaks.hip"), "-o", peaks + ".tmp"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on peaks.hip:\n{r.stderr}")
    os.replace(peaks + ".tmp", peaks)
    if verbose:
        print(f"built {OUT} and {peaks}")
    return OUT


if __name__ == "__main__":
    build()
