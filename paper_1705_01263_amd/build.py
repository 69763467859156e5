"""Build libqpt.so for gfx950 in-tree (hipcc; no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqpt.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions stay off (the compiler must not form v_pk_* FP32 ops)
NO_PK_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    host_o = os.path.join(BUILD, "qpt_host.o")
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INC, "-I", CSRC, "-I", "/opt/rocm/include", "-Wall", "-Wno-unused-function"]
    # host builders: no contraction, so FP64 table construction is reproducible
    _run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-ffp-contract=off", *common, "-c",
          os.path.join(CSRC, "qpt_host.cpp"), "-o", host_o])
    objs = [host_o]
    for src in ("qpt_kernels.hip", "qpt_guide.hip", "qpt_build.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", *NO_PK_FP32, *common, "-c",
              os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    # -z defs: every symbol the library uses must resolve at link time
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
