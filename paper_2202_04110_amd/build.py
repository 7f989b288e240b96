"""Builds liblbp.so (HIP kernels for gfx950 + the C-ABI) in the package directory.

    python -m paper_2202_04110_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbp.so")
SOURCES = ["kernels.hip", "compile.cpp", "hostmem.cpp", "runtime.cpp", "api.cpp", "server.cpp"]
HEADERS = ["kernels.h", "compile.h", "hostmem.h", "lbp_internal.h", "runtime.h", "arena.h"]

# -ffp-contract=off: no implicit fused multiply-adds, so every element is
# computed with the same roundings in every kernel that inlines the same
# device function.  packed-fp32-ops is switched off for device code.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-D__HIP_PLATFORM_AMD__",
              "-I/opt/rocm/include"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build_library(out: str = LIB, jobs: int = 3) -> str:
    """Compiles every source and links liblbp.so; always rebuilds."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if src.endswith(".hip"):
            cmd = ["hipcc"] + HIP_FLAGS + ["-c", path, "-o", obj]
        else:
            cmd = ["g++"] + HOST_FLAGS + ["-c", path, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = []
    for cmd, p in procs:
        o, e = p.communicate()
        if p.returncode != 0:
            failed.append((cmd, o + e))
    if failed:
        for cmd, msg in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + msg)
        raise RuntimeError("liblbp build failed")
    tmp = out + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library())
