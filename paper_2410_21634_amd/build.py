"""Build the native parts in-tree: the gfx950 HIP library and the workload sampler.

``python -m paper_2410_21634_amd.build`` compiles ``libgde.so`` with hipcc for
gfx950 and the native Chung-Lu sampler with gcc.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgde.so")
SOURCES = ["gde_kernels.hip", "gde_hk_small.hip", "gde_api.hip", "gde_det.hip", "gde_batch_kernels.hip",
           "gde_batch.hip", "gde_server.hip", "gde_noalloc.hip", "gde_global.hip", "gde_dyn.hip", "gde_fifo.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_hip(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *HIP_FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


def build_all(verbose: bool = False) -> None:
    from . import workloads

    workloads.build(force=True)
    build_hip(verbose)


if __name__ == "__main__":
    build_all(verbose=True)
    print(LIB)
