"""Build step: compiles the HIP/C++ sources into ``libjdmi.so`` next to this file.

    python -m paper_math_0508111_amd.build

hipcc targets gfx950 only.  Object files go to ``_build/`` (not committed).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libjdmi.so")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    o = os.path.join(OBJ, "setup.o")
    _run(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, "setup.cpp"), "-o", o])
    objs.append(o)
    for src in ("kernels.hip", "jd.hip"):
        o = os.path.join(OBJ, src.replace(".hip", ".o"))
        _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
