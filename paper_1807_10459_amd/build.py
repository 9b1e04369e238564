"""Build the HIP library ``libksgcmi.so`` for gfx950 in-tree (hipcc, parallel per source)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libksgcmi.so")

SOURCES = [  # longest compiles first, so that the parallel build ends early
    "ksg_window.hip",
    "ksg_alg2.hip",
    "ksg_search_kp5.hip",
    "ksg_search_kp9.hip",
    "ksg_search_kp17.hip",
    "ksg_window_alg2.hip",
    "ksg_search_wide.hip",
    "ksg_group_wide_kp5.hip",
    "ksg_group_wide_kp9.hip",
    "ksg_group_kp5_g8.hip",
    "ksg_group_kp5_g16.hip",
    "ksg_group_kp9_g8.hip",
    "ksg_group_kp9_g16.hip",
    "ksg_yzcount.hip",
    "ksg_misc.hip",
    "ksg_api.hip",
    "batch.hip",
    "ksg_noalloc.hip",
    "greedy.hip",
    "mlp_kernels.hip",
    "mlp_api.hip",
    "autotune.hip",
    "host_stats.cpp",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off; FP32 denormals are kept; no FMA contraction
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=off",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
