"""Build ``libgna.so`` for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgna.so")
SOURCES = [os.path.join(CSRC, "gna.hip"), os.path.join(CSRC, "gna_pipe.hip")]
HEADERS = [os.path.join(CSRC, "gna_kernels.h"), os.path.join(ROOT, "include", "gna.h")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into ``libgna.so`` (always recompiles).

    The translation units are compiled in parallel into objects, then linked."""
    tmp = LIB + ".tmp"
    flags = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
             # packed FP32 VALU forms are kept out of generated code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = [os.path.join(HERE, "_" + os.path.splitext(os.path.basename(src))[0] + ".o") for src in SOURCES]
    procs = []
    for src, obj in zip(SOURCES, objs):
        cmd = [*flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    errs = []
    for pr in procs:
        _, err = pr.communicate()
        if pr.returncode != 0:
            errs.append("\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l))
    try:
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc link failed ({res.returncode}):\n{res.stderr}")
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
