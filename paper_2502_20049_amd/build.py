"""Build libpsm.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32
instructions disabled; the mapping kernel and the host kinematics are compiled
without floating-point contraction (their FP64 operation order is part of the
lookup's definition).  Objects go to ``_build/``; the shared library is written
next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpsm.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include")]

SOURCES = [
    ("psm_capi.cpp", ["-x", "hip", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos"]),
    ("geometry.cpp", ["-x", "hip", "-ffp-contract=off"]),
    ("k_mapping.hip", ["-ffp-contract=off"]),
    ("k_misc.hip", []),
    ("k_adjoint.hip", []),
    ("k_sc_f64.hip", []),
    ("k_sc_f32.hip", []),
    ("k_sc_f16.hip", []),
]


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(lambda a: _compile(*a), SOURCES))
    objs = [o for o, _ in res]
    if verbose:
        for _, err in res:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    if "--clean" in sys.argv:
        shutil.rmtree(BUILD, ignore_errors=True)
