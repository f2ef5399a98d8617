"""Build the engine's shared library (HIP kernels for gfx950 + host C++).

    python -m paper_1412_3022_amd.build

Objects go to ``_build/`` at the repository root; the library to
``paper_1412_3022_amd/_lib/libpmrc.so``.  Host sources are compiled with g++
against the HIP headers, the kernel file with hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libpmrc.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["gf256.cpp", "construct.cpp", "program.cpp", "capi.cpp", "batch.cpp", "server.cpp", "bitslice.cpp",
                "gf16.cpp", "mfma.cpp", "bitslice16.cpp"]
HIP_SOURCES = ["kernels.hip", "gj.hip", "gf16.hip", "noalloc.hip", "mfma.hip"]

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
              "-I" + os.path.join(ROCM, "include"), "-I" + INCLUDE, "-pthread"]
# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I" + INCLUDE, "-I" + CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _jobs():
    out = []
    for src in HOST_SOURCES:
        path = os.path.join(CSRC, src)
        if os.path.exists(path):
            obj = os.path.join(BUILD, src + ".o")
            out.append((["g++"] + HOST_FLAGS + ["-c", path, "-o", obj], obj))
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        out.append(([HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj], obj))
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link the library.  Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = _jobs()
    procs = []
    for cmd, obj in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), cmd))
    failed = []
    for p, cmd in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines()
                         if "packed-fp32-ops" not in l and "unused during compilation" not in l)
        if p.returncode != 0:
            failed.append((cmd, text))
        elif text.strip() and verbose:
            print(text)
    if failed:
        for cmd, text in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + text + "\n")
        raise RuntimeError("build of the HIP engine failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + [o for _, o in jobs] + \
        ["-pthread", "-L" + os.path.join(ROCM, "lib"), "-lhiprtc"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
