"""Build libsqrtba.so (FP32) and libsqrtba64.so (FP64) for gfx950 in-tree with hipcc.

Both libraries come from the same sources; the FP64 one is compiled with
SQRTBA_FP64, which makes the element type of every kernel and buffer double.

    python -m paper_2103_01843_amd.build          # release build of both
    python -m paper_2103_01843_amd.build --check  # print the commands only
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsqrtba.so")
LIB64 = os.path.join(HERE, "libsqrtba64.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "learned.hip"), os.path.join(CSRC, "noalloc.hip"),
           os.path.join(CSRC, "api.cpp")]
ARCH = "gfx950"

# packed-FP32 instructions are disabled for every HIP file (numerical safety
# on this hardware generation); the host pass warns that it does not know the
# feature, which is harmless.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def command(out: str = LIB, fp64: bool = False):
    return [hipcc(), *FLAGS, *(["-DSQRTBA_FP64"] if fp64 else []), "-I", os.path.join(ROOT, "include"), *SOURCES,
            "-o", out]


def build(verbose: bool = True) -> str:
    """Compile both libraries (concurrently) and move them into place; returns the FP32 path."""
    jobs = []
    for lib, fp64 in ((LIB, False), (LIB64, True)):
        cmd = command(lib + ".tmp", fp64)
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((lib, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = []
    for lib, proc in jobs:
        _, err = proc.communicate()
        errs = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if proc.returncode != 0:
            failed.append(f"{os.path.basename(lib)}: hipcc failed ({proc.returncode}):\n{errs}")
        elif verbose and errs:
            print(errs, file=sys.stderr)
    if failed:
        raise RuntimeError("\n".join(failed))
    for lib, _ in jobs:
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    if "--check" in sys.argv:
        print(" ".join(command()))
        print(" ".join(command(LIB64, True)))
    else:
        build()
