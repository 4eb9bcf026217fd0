"""Build libnpweno.so (HIP, gfx950) in-tree with hipcc.

The double-precision kernels are compiled without FP contraction so that they evaluate the
scheme in the order it is written; the float kernels may fuse multiply-adds.  Packed-FP32
instructions are disabled for every HIP translation unit.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libnpweno.so")
# stand-alone program that measures the VALU issue ceiling of an instruction mix (bench.py runs it)
PROBE = os.path.join(HERE, "valu_mix_probe")
BUILD = os.path.join(HERE, "_build")

ARCH = os.environ.get("NPW_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]

UNITS = [
    ("npw_kernels_f64.hip", ["-ffp-contract=off"]),
    ("npw_kernels_f32.hip", []),
    ("npw_runtime.cpp", ["-x", "hip"]),
    ("npw_server.cpp", ["-x", "hip"]),
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    return "hipcc"


def _compile(unit, extra):
    src = os.path.join(CSRC, unit)
    obj = os.path.join(BUILD, unit + ".o")
    cmd = [_hipcc(), *COMMON, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stderr}")
    return obj


def _build_probe():
    tmp = PROBE + ".tmp"
    cmd = [_hipcc(), *COMMON, os.path.join(CSRC, "valu_mix_probe.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for valu_mix_probe.hip:\n{r.stderr}")
    os.replace(tmp, PROBE)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(UNITS) + 1) as ex:
        probe = ex.submit(_build_probe)
        objs = list(ex.map(lambda u: _compile(*u), UNITS))
        probe.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, "and", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
