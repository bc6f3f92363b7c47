"""Compile libthcsox for gfx950 with hipcc (in-tree shared library).

Each source is compiled to its own object in parallel (every kernel is launched
from the file that defines it, so no relocatable device code is needed), then
the objects are linked into paper_2404_17744_amd/libthcsox.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libthcsox.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["kernels.hip", "gemmk.hip", "astage_f16.hip", "astage_bf3.hip", "fused.hip", "fused_f16.hip", "fused_bf3.hip",
           "thcsox.hip", "dyson.hip", "loopctl.hip", "direct.hip", "mlp.hip", "irgrid.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")


def build(verbose: bool = False, out: str = LIB) -> str:
    """Compile every HIP source and link the shared library (default: the
    in-tree paper_2404_17744_amd/libthcsox.so)."""
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-c", "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = out + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
