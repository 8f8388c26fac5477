"""Builds libaenet_gpu.so (the HIP library behind include/aenet_gpu.h) for gfx950.

Every .hip file under csrc/ is compiled with hipcc into _build/ and linked
into paper_2107_11311_amd/libaenet_gpu.so; probe/peaks.hip (the arithmetic
peak microbenchmarks of bench.py) into libaenet_probe.so.  Packed-FP32 instructions are
disabled for the device code (plain FP32 VALU and MFMA are used instead).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libaenet_gpu.so")
PROBE = os.path.join(HERE, "probe")
PROBE_LIB = os.path.join(HERE, "libaenet_probe.so")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)


def build(jobs: int | None = None) -> str:
    """Compiles every HIP source and links the shared library, and the
    benchmark's peak-rate probes into libaenet_probe.so; returns the
    library's path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    probe_src = os.path.join(PROBE, "peaks.hip")
    jobs = jobs or min(len(srcs) + 1, max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs + [probe_src]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build())
