"""Build ``libvcx.so`` (HIP for gfx950 + host C++) in the package directory.

    python -m paper_2201_01291_amd.build

Compiles every time it is called.  The library is loaded in-tree by the
ctypes binding (``paper_2201_01291_amd/vcx.py``).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvcx.so")
ARCH = os.environ.get("VCX_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain scalar FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fused multiply-adds only inside one source expression, so that a body
    # inlined into different kernels (single solve, batch) rounds the same way
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


# HIP translation units: the C ABI, one kernel-table unit per model (compiled
# in parallel), and the Poisson solve
HIP_SOURCES = ["vcx_capi.hip", "vcx_tab_gas2.hip", "vcx_tab_gas3.hip", "vcx_tab_dd.hip",
               "vcx_tab_ns.hip", "vcx_tab_quad.hip", "vcx_poisson.hip", "vcx_static.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="vcx_build_") as tmp:
        host_o = os.path.join(tmp, "vcx_mesh.o")
        serv_o = os.path.join(tmp, "vcx_server.o")
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        procs = [
            subprocess.Popen(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", *inc, "-c",
                              os.path.join(CSRC, "vcx_mesh.cpp"), "-o", host_o]),
            subprocess.Popen(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-pthread",
                              "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"), *inc,
                              "-c", os.path.join(CSRC, "vcx_server.cpp"), "-o", serv_o]),
        ]
        objs = [host_o, serv_o]
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            objs.append(obj)
            procs.append(subprocess.Popen(["hipcc", *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src),
                                           "-o", obj]))
        if verbose:
            print("compiling vcx_mesh.cpp, vcx_server.cpp (g++) and " + ", ".join(HIP_SOURCES) +
                  " (hipcc)", flush=True)
        rcs = [p.wait() for p in procs]
        if any(rcs):
            raise RuntimeError(f"compilation failed (exit codes {rcs})")
        tmp_lib = LIB + ".tmp"
        _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp_lib, *objs],
             verbose)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    print(LIB)
