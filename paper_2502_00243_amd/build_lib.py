"""Builds libfpw.so (HIP kernels + host runtime) for gfx950 with hipcc.

Run as ``python -m paper_2502_00243_amd.build_lib``; ``__graft_entry__.build``
calls :func:`build`.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfpw.so")
ARCH = "gfx950"

SOURCES = ["fpw_batched.hip", "fpw_aux.hip", "fpw_shared.hip", "fpw_baseline.hip", "fpw_static.hip", "fpw_host.cpp"]

# Device code: no automatic fma contraction (the folds spell out every fused
# operation they want) and no packed-FP32 instructions.
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
COMMON_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the FPW library needs ROCm's hipcc to build")


def _compile_cmd(src: str, obj: str) -> list:
    cmd = [hipcc(), *COMMON_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip", *DEVICE_FLAGS]
    else:
        cmd[1:1] = ["-D__HIP_PLATFORM_AMD__"]
    return cmd


def build(verbose: bool = False) -> str:
    """Compiles every source (in parallel) and links libfpw.so next to this file; returns its path."""
    from concurrent.futures import ThreadPoolExecutor

    build_dir = os.path.join(CSRC, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, src + ".o") for src in SOURCES]
    cmds = [_compile_cmd(src, obj) for src, obj in zip(SOURCES, objs)]
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for src, r in zip(SOURCES, results):
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
