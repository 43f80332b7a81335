"""Build libpdhg.so for gfx950 with hipcc (in-tree; no GPU needed)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpdhg.so")
SOURCES = ["host_csr.cpp", "kernels.hip", "pdhg.cpp", "cpu_steps.cpp", "cpu_pdhg.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def build(verbose: bool = False, out: str = OUT, defines=(),
          bdir: str = None) -> str:
    """Compile every source and link the shared library at `out`.
    `defines` (e.g. ["PDHG_TILE64=1024"]) override build-time tile sizes."""
    objs = []
    bdir = bdir or os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        cmd = [HIPCC, *COMMON, *["-D" + d for d in defines], "-c", path,
               "-o", obj]
        cmd[1:1] = ["-x", "hip"] + DEVICE
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp,
           *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
