"""Build libatlas_nabla.so in-tree for gfx950.

Host C++ (mesh builder, C ABI) is compiled with g++, the kernels with hipcc
for gfx950, and everything is linked by hipcc into
``paper_1908_07038_amd/lib/libatlas_nabla.so``.

The mesh builder is compiled without floating-point contraction and without
the compiler's sin/cos builtins, so node positions come out of the C library
exactly as written in the source.  Kernels are compiled with packed FP32
instructions disabled.

Usage: ``python -m paper_1908_07038_amd.build`` (or ``build()`` from Python).
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libatlas_nabla.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"


def _hipcc():
    p = os.path.join(ROCM, "bin", "hipcc")
    return p if os.path.exists(p) else shutil.which("hipcc")


def _commands():
    hipcc = _hipcc()
    if not hipcc:
        raise RuntimeError("hipcc not found (ROCm is required to build the library)")
    inc = ["-I", INCLUDE, "-I", CSRC]
    host = ["g++", "-std=c++17", "-O2", "-fPIC", "-Wall", "-Wno-unused-result",
            "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos",
            "-fno-builtin-sincos", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]
    dev = [hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # work-counter claims stay plain atomics whose result is read
           # late (no wave-level rewrite that waits for it at once)
           "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
           "-Wno-unused-command-line-argument"]
    objs = []
    cmds = []
    for src, base in (("mesh_build.cpp", host), ("remap_build.cpp", host), ("capi.cpp", host), ("kernels.hip", dev)):
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmds.append(base + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
    link = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs + \
        ["-Wl,--no-undefined", "-L", os.path.join(ROCM, "lib"), "-lamdhip64"]
    return cmds, link


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose=False):
    """Compile every source and (re)link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    cmds, link = _commands()
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for r, c in zip(ex.map(_run, cmds), cmds):
            if verbose:
                print(" ".join(c))
    _run(link)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
