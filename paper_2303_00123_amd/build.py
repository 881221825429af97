"""Build libqsv.so (the HIP library behind include/qsv.h) for gfx950.

Each source is compiled by hipcc into paper_2303_00123_amd/_build/ in
parallel, then linked into paper_2303_00123_amd/libqsv.so.  Run directly
(`python -m paper_2303_00123_amd.build`) or through __graft_entry__.build().
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqsv.so")
ARCH = os.environ.get("QSV_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "qsv_capi.cpp",
    "qsv_plan.cpp",
    "qsv_gates.hip",
    "qsv_reduce.hip",
    "qsv_tile.hip",
    "qsv_adjoint.hip",
    "qsv_batch.hip",
    "qsv_tune.cpp",
]

# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions.
# -simplifycfg-sink-common=false: the tile kernel's compile-time register
#   index maps live in switch cases; sinking their common code would turn the
#   constant indices into a runtime-selected one and push the per-thread
#   amplitude array out of registers into scratch memory.
# kernel-resource-usage remarks are parsed to reject any kernel that spills
# to scratch or overflows into accumulation registers (see _compile).
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Rpass-analysis=kernel-resource-usage",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *CFLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    usage = parse_resource_usage(r.stderr)
    spills = {k: v for k, v in usage.items() if v.get("ScratchSize [bytes/lane]", 0) > 0}
    if spills:
        raise RuntimeError(f"{src}: kernels use scratch memory: {sorted(spills)}")
    # No kernel here uses matrix instructions, so accumulation registers in
    # use mean the arrays overflowed 256 vector registers: the kernel then
    # runs one wave per SIMD.  That is accepted only where LDS already
    # limits it to one workgroup per CU (more than 80 KiB).
    overflow = {k for k, v in usage.items()
                if v.get("AGPRs", 0) > 0 and v.get("LDS Size [bytes/block]", 0) <= 80 * 1024}
    if overflow:
        raise RuntimeError(f"{src}: kernels overflow 256 vector registers: {sorted(overflow)}")
    with open(obj + ".usage.json", "w") as f:
        json.dump(usage, f, indent=1, sort_keys=True)
    return obj


def parse_resource_usage(text: str) -> dict:
    """Kernel name -> {field: int} from -Rpass-analysis=kernel-resource-usage."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([^:]+): (\d+) \[-Rpass-analysis", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = int(m.group(2))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
