"""Build libardeblur.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1211_0393_amd.build [--jobs N]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libardeblur.so")
SOURCES = ["ar_plan.hip", "ar_blur.hip", "ar_fft.hip", "ar_xform.hip", "ar_x1023.hip", "ar_tune.hip", "ar_iterate.hip",
           "ar_batch.hip", "ar_learned.hip", "ar_dense.hip", "ar_bc.hip", "ar_blur_mfma.hip"]
ARCH = "gfx950"


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return [
        "-O3",
        "-std=c++20",
        f"--offload-arch={ARCH}",
        "-fPIC",
        "-I", INCLUDE,
        "-I", CSRC,
        # keep the compiler from forming packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
    ]


def _stale(obj, src):
    """True when obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC)
                                        if h.endswith(".h")] + [os.path.join(INCLUDE, "ardeblur.h")]
    return any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def compile_one(src, incremental=False):
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and not _stale(obj, src):
        return obj
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=4, verbose=True, incremental=False):
    """Compile every source and link libardeblur.so; rebuilds everything
    unless `incremental` (then only objects older than their sources)."""
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only sources changed since their object was built")
    a = ap.parse_args(argv)
    build(a.jobs, incremental=a.incremental)


if __name__ == "__main__":
    sys.exit(main())
