"""Builds libfd.so (the gfx950 HIP kernels and the C ABI of include/fd.h)
and libfd_cpu.so (the host back-end: the same ABI over host memory with
OpenMP and AVX2/AVX-512, include/fd_cpu.h).

Run as ``python -m paper_2311_05038_amd.build``; the libraries are written
next to this file so that they travel with the source tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfd.so")
SOURCES = ["fd_kernels.hip", "fd_routines.hip", "fd_probe.hip", "fd_host.cpp", "fd_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    # packed FP32 instructions stay off: the kernels are plain scalar FP32
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source into one shared library (`out`).  `defines`
    (e.g. ["FD_3D_ZC=32"]) override the tile-shape defaults."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + \
        [os.path.join(CSRC, f) for f in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


CSRC_CPU = os.path.join(HERE, "csrc_cpu")
LIB_CPU = os.path.join(HERE, "libfd_cpu.so")
GXX = os.environ.get("CXX", "g++")
CPU_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra"]
# (source, instruction-set flags): each vector width in its own object, the
# choice made at run time from what the processor reports
CPU_SOURCES = [("fd_cpu.cpp", []), ("fd_cpu_avx2.cpp", ["-mavx2", "-mfma"]),
               ("fd_cpu_avx512.cpp", ["-mavx512f"])]


def build_cpu(verbose: bool = False, out: str = LIB_CPU, extra=()) -> str:
    """Compile the host back-end into one shared library (`out`); `extra`
    flags go to every compile and the link (e.g. sanitizers)."""
    tmp = out + ".tmp%d" % os.getpid()
    objs = []
    for src, isa in CPU_SOURCES:
        obj = "%s.%s.o" % (tmp, os.path.splitext(src)[0])
        cmd = [GXX] + CPU_FLAGS + list(extra) + isa + ["-c", os.path.join(CSRC_CPU, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    # -Bsymbolic: calls between the library's own entry points stay inside it
    # even when the GPU library (same symbol names) is loaded in the process
    cmd = [GXX, "-shared", "-fopenmp", "-Wl,-Bsymbolic"] + list(extra) + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    for o in objs:
        os.remove(o)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_cpu(verbose="-v" in sys.argv))
