"""Build libss.so (HIP, gfx950) in-tree with hipcc.

Flags: -ffp-contract=off keeps the error-free transformations exact; packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["ss_kernels.hip", "ss_fp64.hip", "ss_api.hip", "ss_lbfgs.hip", "ss_batch.hip", "ss_server.hip"]
LIB = os.path.join(HERE, "libss.so")
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str, sources: list[str], extra: list[str] | None = None) -> list[str]:
    return ["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, *(extra or []), "-o", out, *sources]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp, srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libss.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
