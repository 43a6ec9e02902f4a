"""Build step of the gfx950 library: compiles csrc/*.hip, csrc/host.cpp and csrc/serve.cpp
with hipcc into libpdhcg_hip.so inside this package directory."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpdhcg_hip.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "batch.hip", "calib.hip", "host.cpp", "serve.cpp")]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # no packed FP32 instructions anywhere (hipcc's host pass warns about
         # the unknown feature; that is harmless)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *FLAGS, "-o", LIB + ".tmp", "-x", "hip", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
