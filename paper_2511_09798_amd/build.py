"""Build libmqhelm.so (the gfx950 HIP library behind include/mqhelm.h) in-tree.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled; the host objects are linked into one shared library
next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmqhelm.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["op_kernels.hip", "stored_kernels.hip", "gkb_kernels.hip", "proj_kernels.hip", "svd_kernels.hip",
           "mlp_kernels.hip", "full_kernels.hip", "block_kernels.hip", "band_kernels.hip", "capi.hip"]
# the measurement library beside it (reference kernels for the rooflines; not part of the method)
PEAK_SOURCES = ["peak_kernels.hip", "peak_capi.hip"]
PEAK_LIB = os.path.join(HERE, "libmqhpeak.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results straight into VGPRs (the product kernels read every
    # result with VALU instructions; the accumulator-register form would add
    # one move per value)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compile all sources (always) and link libmqhelm.so and the measurement library
    libmqhpeak.so; returns the solver library's path."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES + PEAK_SOURCES))
    _link(objs[: len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], PEAK_LIB)
    if verbose:
        print(f"built {LIB}")
        print(f"built {PEAK_LIB}")
    return LIB


SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer"]
SAN_DRIVER = os.path.join(ROOT, "tests", "host", "capi_san_main.cpp")
SAN_EXE = os.path.join(ROOT, "tests", "host", "capi_san")


def build_sanitized(verbose: bool = False) -> str:
    """A test executable that drives the C ABI (tests/host/capi_san_main.cpp) through the
    library's sources with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
    (device code is built as usual); returns its path."""
    objdir = os.path.join(OBJDIR, "san")
    os.makedirs(objdir, exist_ok=True)
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_FLAGS

    def comp(src):
        obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
        res = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"sanitized build failed for {src}:\n{res.stderr}")
        return obj

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [SAN_DRIVER]
    with cf.ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    tmp = SAN_EXE + ".tmp"
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN_FLAGS, *objs, "-o", tmp], capture_output=True,
                         text=True)
    if res.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{res.stderr}")
    os.replace(tmp, SAN_EXE)
    if verbose:
        print(f"built {SAN_EXE}")
    return SAN_EXE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
