"""Build libxeng.so (the HIP X-engine) in-tree for gfx950.

    python -m paper_1411_3751_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libxeng.so")
SOURCES = [os.path.join(HERE, "csrc", "xeng.hip")]
HEADERS = [os.path.join(HERE, "csrc", "xcorr_i8.h"), os.path.join(HERE, "csrc", "xcorr_wg.h"),
           os.path.join(HERE, "csrc", "xeng_stream.h"), os.path.join(HERE, "csrc", "xeng_tune.h"),
           os.path.join(HERE, "csrc", "xeng_ingest.h"), os.path.join(HERE, "csrc", "xeng_fengine.h"),
           os.path.join(HERE, "csrc", "xcorr_w1.h"), os.path.join(HERE, "csrc", "xeng_static.h"),
           os.path.join(ROOT, "include", "xeng.h")]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code (they are not
# needed here, and some of their forms are unreliable on this hardware).
HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include")] + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
