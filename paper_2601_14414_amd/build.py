"""Build libpimpc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2601_14414_amd.build [-v] [-j N]

Each translation unit is compiled to an object file under _build/ (the
lane-per-stage kernels are split into PIMPC_LANE_NPARTS parts so they compile
in parallel), then linked into paper_2601_14414_amd/libpimpc.so.
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
LIB = os.path.join(PKG, "libpimpc.so")
NPARTS = 6

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         # no packed FP32 instructions anywhere in this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC, f"-DPIMPC_LANE_NPARTS={NPARTS}",
         "-Wno-unused-command-line-argument"]


def _units():
    units = [("factor.hip", "factor.o", []), ("admm_row.hip", "admm_row.o", []),
             ("adjoint.hip", "adjoint.o", []),
             ("runtime.cpp", "runtime.o", ["-x", "hip"])]
    for p in range(NPARTS):
        units.append(("admm_lane.hip", f"admm_lane_{p}.o", [f"-DPIMPC_LANE_PART={p}"]))
    return units


def _compile(src, obj, extra, verbose):
    cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} ({obj}):\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(_units()), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, e, verbose) for s, o, e in _units()]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + \
          [os.path.join(BUILD, o) for o in objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-v", action="store_true")
    ap.add_argument("-j", type=int, default=0)
    a = ap.parse_args()
    print(build(verbose=a.v, jobs=a.j))
    sys.exit(0)
