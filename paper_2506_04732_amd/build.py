"""Build libt2s2.so (HIP, gfx950) in-tree with hipcc.

Usage:  python -m paper_2506_04732_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libt2s2.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["spectral_host.cpp", "timing.cpp", "readback.hip", "gemm.hip", "tt_kernels.hip", "dense_small.hip", "schur.hip", "linalg.hip", "ddnorm.hip", "kron_hess.hip", "solver.hip", "mlp.hip", "sources.hip", "cross.hip", "api.hip"]

ARCH = os.environ.get("T2S2_ARCH", "gfx950")
# -packed-fp32-ops: hipcc must not emit packed FP32 instructions
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
            "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-I", CSRC, "-I", INCLUDE]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + HIPFLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src == "spectral_host.cpp":
        cmd = [_hipcc()] + ["-O3", "-std=c++17", "-fPIC", "-I", CSRC, "-I", INCLUDE, "-c",
                            os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    workers = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libt2s2.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
