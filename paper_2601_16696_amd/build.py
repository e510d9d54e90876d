"""Builds the gfx950 HIP library liblaps_hip.so in-tree with hipcc.

Each translation unit is compiled separately (in parallel) and linked into one
shared library exporting the C ABI of include/laps.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "liblaps_hip.so")
CAPI = os.path.join(PKG, "laps_capi_run")
OBJ = os.path.join(PKG, "_build")
SOURCES = ["laps_api.hip", "laps_local.hip", "laps_local_gauss.hip", "laps_local_sv.hip", "laps_local_phi4.hip",
           "laps_control.hip", "laps_logreg.hip", "laps_dense.hip", "laps_rng.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-pass-failed", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", OUT + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    # a plain C consumer of the ABI (HIP runtime C API only), used by the tests
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
           "-I/opt/rocm/include", os.path.join(CSRC, "laps_capi_run.c"), "-o", CAPI + ".tmp",
           "-L" + PKG, "-llaps_hip", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN"]
    subprocess.run(cmd, check=True)
    os.replace(CAPI + ".tmp", CAPI)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build()
