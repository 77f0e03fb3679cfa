"""Build the HIP library libqhd.so for gfx950 (hipcc, in-tree).

Every source is compiled to an object of its own in parallel (objects under
_build/, which is not part of the product), then the objects are linked into
libqhd.so.  Kernels never reference device symbols of another source, so the
sources need no relocatable device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqhd.so")
OBJDIR = os.path.join(ROOT, "_build", "qhd")

SOURCES = ["qhd_api.cpp", "qhd_kernels.hip", "qhd_kernels_3d.hip", "qhd_kernels_mfma.hip", "qhd_kernels_resident.hip",
           "qhd_static.hip", "qhd_spectrum.cpp", "qhd_spectrum_kernels.hip", "sno.cpp",
           "sno_gemm.hip", "sno_kernels.hip", "rqp.cpp", "rqp_kernels.hip"]
HEADERS = ["line_fft.h", "qhd_internal.h", "pass_common.h", "sno_internal.h", "rqp_internal.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 VALU forms are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", h) for h in
                                                                  ("qhd.h", "qhd_sno.h", "qhd_rqp.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (always; the caller decides when) and link libqhd.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
