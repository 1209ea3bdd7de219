"""Build libmclbm.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBS = {
    "libmclbm.so": ["api.cpp", "geometry.cpp", "kernels.hip", "remap.hip", "probe.hip", "thermal.hip"],
    "libwarmnet.so": ["warmnet.hip"],
}

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def _build_one(hipcc, out_name, sources, verbose, jobs):
    out = os.path.join(HERE, out_name)
    objs, procs = [], []
    for src in sources:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc] + [f for f in HIPCC_FLAGS if f != "-shared"] + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + cmd[1:]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(out + ".tmp", out)
    for o in objs:
        os.remove(o)
    return out


def build(verbose: bool = True, jobs: int = 4) -> list:
    """Compile every HIP library (always, also when up to date)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [_build_one(hipcc, name, srcs, verbose, jobs) for name, srcs in LIBS.items()]


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
