"""Builds libabgmres.so (HIP, gfx950) in-tree from csrc/ with hipcc.

``python -m paper_2110_01481_amd.build`` or ``build()`` compiles every translation unit
(in parallel) into ``_build/`` and links the shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libabgmres.so")
SOURCES = ["capi.cpp", "projectors.hip", "krylov.hip", "ncp.hip", "solver.hip", "batch.hip",
           "lsq.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-result",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
]


# Host-code sanitizer build (device code as usual): every -fsanitize= is preceded by
# -Xarch_host, so only the host side of each translation unit is instrumented.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
# in-tree (not under _build/) so that GPU runs of the sanitizer checks find it
SANITIZED_LIB = os.path.join(HERE, "_san", "libabgmres_hostsan.so")


def _compile(src: str, extra=(), outdir: str = BUILD) -> str:
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


def build_host_sanitized(verbose: bool = False) -> str:
    """The library with its host code built under AddressSanitizer and UBSan
    (paper_2110_01481_amd/_san/libabgmres_hostsan.so), for sanitizer runs of the host logic: a
    program that loads it must carry the sanitizer runtime itself (an instrumented
    executable; tests/native/capi_sanitize_check.cpp)."""
    out = os.path.join(BUILD, "hostsan")
    os.makedirs(out, exist_ok=True)
    os.makedirs(os.path.dirname(SANITIZED_LIB), exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, HOST_SANITIZE, out), SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SANITIZE, *objs, "-o",
           SANITIZED_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(SANITIZED_LIB)
    return SANITIZED_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
