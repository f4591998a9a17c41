"""Compile libvc.so (HIP, gfx950) in-tree with hipcc.

Each .hip source under csrc/ is compiled to an object in parallel (the
search worker once per degree-array type), then
linked into paper_2512_18334_amd/libvc.so.  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libvc.so")
BUILD_DIR = os.path.join(ROOT, "_build")
# (source, object name, extra flags); the search worker is built once per
# degree-array type, with its lists in LDS and in HBM, so the six
# instantiations compile in parallel
SOURCES = [("api.hip", "api", []), ("batch.hip", "batch", []), ("root.hip", "root", []),
           ("crown.hip", "crown", []), ("enum.hip", "enum", []),
           ("search.hip", "search", []), ("serve.hip", "serve", []),
           ("search_deg.hip", "search_d1", ["-DVC_DEG_BYTES=1"]),
           ("search_deg.hip", "search_d2", ["-DVC_DEG_BYTES=2"]),
           ("search_deg.hip", "search_d4", ["-DVC_DEG_BYTES=4"]),
           ("search_deg.hip", "search_d1h", ["-DVC_DEG_BYTES=1", "-DVC_HL=1"]),
           ("search_deg.hip", "search_d2h", ["-DVC_DEG_BYTES=2", "-DVC_HL=1"]),
           ("search_deg.hip", "search_d4h", ["-DVC_DEG_BYTES=4", "-DVC_HL=1"])]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libvc)")


def _compile(entry) -> str:
    src, name, extra = entry
    obj = os.path.join(BUILD_DIR, name + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if name.startswith("search_d"):
        # the search kernel's register use: a spill to scratch (the worker
        # object no longer kept in registers) costs far more than it looks
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if name.startswith("search_d"):
        _check_resources(name, r.stderr)
    return obj


SCRATCH_WARN = 64  # bytes per lane


def _check_resources(name: str, remarks: str) -> None:
    kernel, lines = None, []
    for line in remarks.splitlines():
        if "Function Name:" in line:
            kernel = line.split("Function Name:")[1].split()[0]
        elif kernel and "search_kernel" in kernel and "ScratchSize" in line:
            size = int(line.split("]:")[1].split()[0])
            lines.append(f"{name} {kernel} scratch {size} B/lane")
            if size > SCRATCH_WARN:
                print(f"warning: {kernel} ({name}) spills {size} bytes per lane to scratch")
    with open(os.path.join(BUILD_DIR, name + ".resources.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
