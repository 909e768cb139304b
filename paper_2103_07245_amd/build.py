"""Build libpbpqlp.so for gfx950 in-tree with hipcc.

    python -m paper_2103_07245_amd.build        # or __graft_entry__.build()
    python -m paper_2103_07245_amd.build --incremental   # only sources newer than their objects

Every HIP source under csrc/ is compiled to an object in _build/ (in
parallel) and linked into paper_2103_07245_amd/libpbpqlp.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpbpqlp.so")

SOURCES = ["stream_gemm.hip", "tallskinny.hip", "small.hip", "apply.hip", "pbpqlp_api.hip",
           "learned.hip", "tune.hip", "reconstruct.hip", "large.hip", "sparse.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the triangular apply relies on full unrolling to keep its tiles in registers
    "-mllvm", "-pragma-unroll-threshold=1000000",
    "-Wno-pass-failed",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(x for x in r.stderr.splitlines() if "packed-fp32-ops" not in x)
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj


def _stale(src: str) -> bool:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "pbpqlp.h"))
    return any(os.path.getmtime(f) > t for f in [os.path.join(CSRC, src), *headers])


def build(verbose: bool = True, incremental: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    todo = [s for s in SOURCES if not incremental or _stale(s)]
    jobs = min(max(1, len(todo)), max(1, int(os.environ.get("MAX_JOBS", "8"))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
