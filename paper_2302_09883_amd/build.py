"""Build liblbmz.so (HIP for gfx950) in the package directory.

Every translation unit is compiled by hipcc for gfx950 only, in parallel, then
linked into ``paper_2302_09883_amd/liblbmz.so``.  Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbmz.so")

SOURCES = [
    "lbmz_runtime.cpp",
    "lbmz_dense.hip",
    "lbmz_inst_f32_fv.hip",
    "lbmz_inst_f32_lbm.hip",
    "lbmz_inst_f64_fv.hip",
    "lbmz_inst_f64_lbm.hip",
    "lbmz_inst_f32_fv_q.hip",
    "lbmz_inst_f32_lbm_q.hip",
    "lbmz_inst_f32_euler.hip",
    "lbmz_net.hip",
    "lbmz_d3q19.hip",
    "lbmz_inst_f32_e4m3b_lbm.hip",
    "lbmz_inst_f32_e4m3b_fv.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-6000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, extra_flags=(), lib_path: str = LIB,
          build_dir: str = BUILD) -> str:
    """Compile every HIP source and link the shared library; returns its path.

    ``extra_flags`` are added to every hipcc compile (e.g. a profiling macro);
    ``lib_path`` / ``build_dir`` let such variants live outside the package.
    """
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, tuple(extra_flags)), SOURCES))
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, lib_path)
    if verbose:
        print(f"built {lib_path}", file=sys.stderr)
    return lib_path


if __name__ == "__main__":
    build()
