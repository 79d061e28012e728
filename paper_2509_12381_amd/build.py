"""Build libai.so in place from csrc/ai.hip with hipcc for gfx950.

    python -m paper_2509_12381_amd.build [--remarks]

--remarks prints the compiler's per-kernel resource usage (VGPRs, AGPRs,
scratch spills, occupancy).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "ai.hip")
HEADER = os.path.join(ROOT, "include", "ai.h")
LIB = os.path.join(PKG, "libai.so")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(remarks: bool = False, out: str = LIB) -> str:
    tmp = out + f".tmp{os.getpid()}"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if remarks:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode})")
    if remarks:
        for line in (res.stdout + res.stderr).splitlines():
            if "remark:" in line and ("Function Name" in line or "GPRs" in line
                                      or "Scratch" in line or "Occupancy" in line):
                print(line.split("remark:")[-1].strip())
    os.replace(tmp, out)
    return out


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    built = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > built for p in (SRC, HEADER))


if __name__ == "__main__":
    print(build(remarks="--remarks" in sys.argv))
