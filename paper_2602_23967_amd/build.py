"""Build step of the gfx950 library: compiles each source in csrc/ with hipcc
(in parallel, objects under _build/ at the repository root) and links
libpdhcg_hip.so inside this package directory."""

from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpdhcg_hip.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "batch.hip", "calib.hip", "host.cpp", "serve.cpp",
                                                  "noalloc.cpp", "prep.cpp")]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed FP32 instructions anywhere (hipcc's host pass warns about
         # the unknown feature; that is harmless)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, "-c", "-x", "hip", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
