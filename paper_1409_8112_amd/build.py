"""Build step of the HIP library: one hipcc call producing librtg.so for gfx950.

Flags:
  -ffp-contract=off   no fused multiply-add unless written out, so the FP64
                      cell coordinates and the FP64 band re-test round every
                      operation on its own, in the order written;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep the compiler from emitting packed FP32 arithmetic.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "librtg.so")
SOURCES = [os.path.join(CSRC, f)
           for f in ("rtg_kernels.hip", "rtg_host.cpp", "rtg_server.cpp", "rtg_tune.cpp",
                     "rtg_plan.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in ("rtg_internal.h", "rtg_runtime.h")] + [
    os.path.join(os.path.dirname(HERE), "include", "rtg.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core results straight into VGPRs (no accumulator-register reads)
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-Wall", "-Wno-unused-result", "-Wno-pass-failed", "-pthread"]


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{err}")
    if verbose and err.strip():
        print(err)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def is_stale() -> bool:
    if not os.path.exists(LIB_PATH):
        return True
    t = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
