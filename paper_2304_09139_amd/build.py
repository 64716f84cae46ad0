"""Build libss.so (HIP, gfx950) in-tree with hipcc.

Flags: -ffp-contract=off keeps the error-free transformations exact; packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["ss_kernels.hip", "ss_fp64.hip", "ss_api.hip", "ss_lbfgs.hip", "ss_batch.hip", "ss_server.hip"]
LIB = os.path.join(HERE, "libss.so")
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of every source the library is built from:
    the HIP sources and headers under csrc/ and the C interface include/ss.h.
    Compiled into libss.so as its build id (ss_build_id)."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "ss.h"), "rb") as fh:
        h.update(b"ss.h")
        h.update(fh.read())
    return h.hexdigest()[:16]


def hipcc_cmd(out: str, sources: list[str], extra: list[str] | None = None) -> list[str]:
    return ["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, *(extra or []), "-o", out, *sources]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp, srcs, [f'-DSS_BUILD_ID="{source_hash()}"'])
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
