"""Build the in-tree libraries.

librteom.so            the product: C ABI + engine + gfx950 HIP kernels.
librteom_hostcheck.so  test build of the same engine over host loops (tests/hostcheck/backend_host.cpp,
                       output in tests/_hostcheck/),
                       used only by CPU tests of the host logic; never loaded by the package.
kernel_probe           test program (tests/kernel_probe/) that checks the GEMM and permute
                       kernels of librteom.so against host loops; run by a GPU test.

Run ``python -m paper_2301_04249_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CXX_SOURCES = ["engine.cpp", "rteom.cpp"]
HIP_SOURCES = ["backend_hip.hip"]
# packed fp32 instructions off for all device code (build notes)
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_product(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    out = os.path.join(HERE, "librteom.so")
    tmp = out + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, out)
    return out


def build_hostcheck():
    outdir = os.path.join(ROOT, "tests", "_hostcheck")
    os.makedirs(outdir, exist_ok=True)
    out = os.path.join(outdir, "librteom_hostcheck.so")
    srcs = [os.path.join(CSRC, s) for s in ("engine.cpp", "rteom.cpp")]
    srcs.append(os.path.join(ROOT, "tests", "hostcheck", "backend_host.cpp"))
    _run(["g++", "-O2", "-g", "-std=c++17", "-fPIC", "-shared", "-DRTEOM_HOST_BACKEND", f"-I{CSRC}", *srcs,
          "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_probe():
    d = os.path.join(ROOT, "tests", "kernel_probe")
    out = os.path.join(d, "kernel_probe")
    _run([HIPCC, "-O2", "-std=c++17", os.path.join(d, "kernel_probe.cpp"), f"-L{HERE}", "-l:librteom.so",
          "-Wl,-rpath,$ORIGIN/../../paper_2301_04249_amd", "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def main():
    build_product()
    build_hostcheck()
    build_probe()


if __name__ == "__main__":
    sys.exit(main())
