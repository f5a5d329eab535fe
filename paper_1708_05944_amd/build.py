"""Build step of the HIP library: ``python -m paper_1708_05944_amd.build``.

Compiles csrc/*.cpp and csrc/*.hip with hipcc for gfx950 into ``libvlb.so`` next to
this file (in-tree, so it travels with the source tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvlb.so")
SOURCES = ["velocity_set.cpp", "couette_kernels.hip", "couette_wide.hip", "api.cpp", "mlp_kernels.hip", "mlp_api.cpp",
           "channel_kernels.hip", "channel_api.cpp", "noalloc.hip"]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # keep hipcc from emitting packed FP32 instructions (v_pk_*_f32)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, *FLAGS, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
