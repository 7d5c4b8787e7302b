"""Build the gfx950 shared library in-tree with hipcc (no JIT, no torch extension)."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcfr_mi355x.so")
SOURCES = ["flatten.cpp", "xplan.cpp", "host_layout.cpp", "partition_plan.cpp", "partition.cpp",
           "solver.cpp", "mlp_api.cpp", "kernels.hip", "xkernels.hip", "mlp.hip", "mlp_noalloc.hip"]

# Packed-fp32 instructions stay off: plain float code only.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libcfr_mi355x.so next to this file."""
    from concurrent.futures import ThreadPoolExecutor
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmds.append(([hipcc(), *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    if verbose:
        for cmd, _ in cmds:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1, 8)) as pool:
        for proc in pool.map(lambda c: subprocess.run(c[0]), cmds):
            if proc.returncode != 0:
                raise subprocess.CalledProcessError(proc.returncode, proc.args)
    objs = [obj for _, obj in cmds]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
