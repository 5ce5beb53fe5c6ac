"""Build the gfx950 library libgpe.so in-tree with hipcc (no JIT, no torch extension).

Each source is compiled to an object of its own, in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("kernels_plan.hip", "kernels_batch.hip", "kernels_adj.hip", "runtime.cpp", "batch.cpp", "noalloc.hip")]
OUT = os.path.join(HERE, "libgpe.so")
ARCH = os.environ.get("GPE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str = OUT, defines: tuple = ()) -> str:
    """Compile every source into `out`; `defines` (e.g. ("GPE_RADIX=16",)) select
    compile-time kernel variants for tuning runs."""
    srcs = [s for s in SRC if os.path.exists(s)]
    objdir = os.path.join(os.path.dirname(out) or ".", "_build", os.path.basename(out) + ".obj")
    os.makedirs(objdir, exist_ok=True)
    dflags = [f"-D{d}" for d in defines]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = ["hipcc", *FLAGS, *dflags, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = out + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    defs = tuple(a[2:] for a in sys.argv[1:] if a.startswith("-D"))
    outs = [a[len("--out="):] for a in sys.argv[1:] if a.startswith("--out=")]
    print(build(verbose="-v" in sys.argv, out=outs[0] if outs else OUT, defines=defs))
