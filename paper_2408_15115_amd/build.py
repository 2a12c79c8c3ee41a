"""Build libturret.so (the gfx950 HIP library) in-tree with hipcc.

Every call recompiles.  Flags: -O3 for gfx950 only; packed FP32 ops are
switched off (the host pass of hipcc warns that it does not know that
target feature, which is harmless)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libturret.so")
SOURCES = ["stream_collide.hip", "stream_collide19.hip", "moments.hip", "fine.hip", "kernels.hip", "mlp.hip",
           "api.hip"]
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source additions.  The network's inference keeps its matrix-core results
# in ordinary VGPRs, where the SiLU that follows reads them without a copy out
# of the accumulation registers.
SOURCE_FLAGS = {"mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    flags = HIP_FLAGS + list(extra_flags or [])
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = ["hipcc", *flags, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
