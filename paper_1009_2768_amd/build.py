"""Build libtrmc.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrmc.so")
SOURCES = ["runtime.hip", "k_collide.hip", "k_tiled.hip", "k_slab.hip", "noalloc.hip"]
HEADERS = ["trmc_internal.h", "trmc_device.h", "collide_core.h"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off (compiler-generated v_pk_* FP32 ops excluded)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_1009_2768_amd/libtrmc.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    srcs = SOURCES + HEADERS + [os.path.join("..", "..", "include", "trmc.h")]
    return any(os.path.getmtime(os.path.join(CSRC, s)) > t for s in srcs)


if __name__ == "__main__":
    print(build(verbose=True))
