"""Build the HIP library libqhd.so for gfx950 (hipcc, in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqhd.so")

SOURCES = ["qhd_api.cpp", "qhd_kernels.hip", "qhd_kernels_3d.hip", "qhd_kernels_mfma.hip", "qhd_kernels_resident.hip", "qhd_spectrum.cpp", "qhd_spectrum_kernels.hip", "sno.cpp", "sno_gemm.hip", "sno_kernels.hip", "rqp.cpp", "rqp_kernels.hip"]
HEADERS = ["line_fft.h", "qhd_internal.h", "pass_common.h", "sno_internal.h", "rqp_internal.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 VALU forms are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", h) for h in ("qhd.h", "qhd_sno.h", "qhd_rqp.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + sources()
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
