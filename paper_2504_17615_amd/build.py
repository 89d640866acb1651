"""Build steps for the native parts of the package.

* ``liblmgp.so``      — the HIP library (gfx950) behind ``include/lmgp.h``.
* ``libgraphgen.so``  — the seeded input generators (host C++).

Both are built in-tree so that they travel with the source tree.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblmgp.so")
GEN_SRC = os.path.join(PKG, "graphgen", "graphgen.cpp")
GEN_LIB = os.path.join(PKG, "graphgen", "libgraphgen.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LMGP_OFFLOAD_ARCH", "gfx950")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_graphgen() -> str:
    tmp = GEN_LIB + ".tmp"
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
          GEN_SRC, "-o", tmp])
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def hip_sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build_lib(jobs: int = 8) -> str:
    """Compile every HIP source for gfx950 and link liblmgp.so."""
    srcs = hip_sources()
    if not srcs:
        raise RuntimeError("no HIP sources found")
    objdir = os.path.join(ROOT, "_build", "lmgp")
    os.makedirs(objdir, exist_ok=True)
    flags = [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        # never emit packed-fp32 instructions (they are avoided on this target)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
    ]
    procs = []
    objs = []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = [HIPCC] + flags + ["-c", s, "-o", o]
        print("+", " ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            s0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"compile failed: {s0}")
    for s0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"compile failed: {s0}")
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


def build_all():
    build_graphgen()
    build_lib()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"all": build_all, "lib": build_lib, "graphgen": build_graphgen}[w]()
