"""Build libai.so in place from csrc/*.hip with hipcc for gfx950.

    python -m paper_2509_12381_amd.build [--remarks] [--cached]

Each source is compiled to an object under _build/ and the objects are linked
into libai.so.  --cached recompiles only objects older than their sources
(the kernel unit takes about a minute); --remarks prints the compiler's per-kernel resource usage (VGPRs,
AGPRs, scratch spills, occupancy).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SOURCES = [os.path.join(CSRC, "ai.hip"), os.path.join(CSRC, "schedule.hip"),
           os.path.join(CSRC, "server.hip")]
HEADERS = [os.path.join(ROOT, "include", "ai.h"), os.path.join(CSRC, "schedule.h"),
           os.path.join(CSRC, "internal.h")]
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libai.so")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # roundings are fixed by the source: fused multiply-adds are written out
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _run(cmd, remarks):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}")
    if remarks:
        for line in (res.stdout + res.stderr).splitlines():
            if "remark:" in line and ("Function Name" in line or "GPRs" in line
                                      or "Scratch" in line or "Occupancy" in line):
                print(line.split("remark:")[-1].strip())


def _object(src: str) -> str:
    return os.path.join(OBJDIR, os.path.basename(src) + ".o")


def _stale_object(src: str) -> bool:
    obj = _object(src)
    if not os.path.exists(obj):
        return True
    built = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > built for p in [src, *HEADERS])


def build(remarks: bool = False, cached: bool = False, out: str = LIB) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    todo = [s for s in SOURCES if not cached or _stale_object(s)]

    def compile_one(src):
        obj = _object(src)
        tmp = obj + f".tmp{os.getpid()}"
        cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", "-o", tmp, src]
        if remarks and src.endswith("ai.hip"):
            cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
        _run(cmd, remarks and src.endswith("ai.hip"))
        os.replace(tmp, obj)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(compile_one, todo))
    tmp = out + f".tmp{os.getpid()}"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
          *[_object(s) for s in SOURCES]], False)
    os.replace(tmp, out)
    return out


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    built = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > built for p in [*SOURCES, *HEADERS])


if __name__ == "__main__":
    print(build(remarks="--remarks" in sys.argv, cached="--cached" in sys.argv))
