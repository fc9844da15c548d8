"""Build liblf.so (HIP, gfx950) and the bw_ceiling benchmark in-tree with hipcc.

Usage: python -m paper_0911_5692_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblf.so")
BW_CEILING = os.path.join(PKG, "bw_ceiling")
SOURCES = ["lf_api.hip", "lf_kernels.hip", "lf_sweep.hip", "lf_sweep27.hip", "lf_slab7.hip", "lf_slab27.hip",
           "lf_adjoint.hip", "lf_fft.hip"]
LIBS = ["-L/opt/rocm/lib", "-lhipfft", "-lrocprofiler-sdk-roctx"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 arithmetic stays off: the compiler must not form v_pk_*_f32
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str, build_dir: str) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def _build_bw_ceiling() -> str:
    """The standalone streaming-ceiling benchmark (csrc/bw_ceiling.hip)."""
    tmp = BW_CEILING + ".tmp"
    subprocess.run([HIPCC, *[f for f in FLAGS if f != "-fPIC"], os.path.join(CSRC, "bw_ceiling.hip"), "-o", tmp],
                   check=True)
    os.replace(tmp, BW_CEILING)
    return BW_CEILING


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link liblf.so, and build the
    streaming-ceiling benchmark (always rebuilds)."""
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        bw = ex.submit(_build_bw_ceiling)
        objs = list(ex.map(lambda s: _compile(s, build_dir), SOURCES))
        bw.result()
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} and {BW_CEILING}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
