"""Builds libhomelbm.so (HIP for gfx950) in-tree.

    python -m paper_2602_05295_amd.build [-v]

Every source under csrc/ is compiled with hipcc for gfx950 only, with the
packed-FP32 instructions disabled, and linked into
paper_2602_05295_amd/libhomelbm.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build", "homelbm")
LIB = os.path.join(PKG, "libhomelbm.so")

SOURCES = ["lbm_api.hip", "lbm_fluid.hip", "lbm_boundary.hip", "lbm_aux.hip", "lbm_adjoint.hip",
           "lbm_batch.hip", "lbm_batch_api.hip", "lbm_mixed.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++20",
    "-fPIC",
    "-Wall",
    # no packed FP32 (v_pk_*_f32) anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
]


def _compile(src: str, verbose: bool, build_dir: str, extra: list) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, defines=None, lib_path: str = LIB) -> str:
    """Compiles and links the library.  defines: optional {"NAME": value}
    passed as -DNAME=value (tuning variants); lib_path: output file."""
    extra = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    tag = "_".join(f"{k}{v}" for k, v in sorted((defines or {}).items()))
    build_dir = os.path.join(BUILD_DIR, tag) if tag else BUILD_DIR
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir, extra), SOURCES))
    LIB_OUT = lib_path
    tmp = LIB_OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_OUT)
    return LIB_OUT


def dump_isa(out_dir: str) -> None:
    """Writes the gfx950 assembly of every source to out_dir (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    for src in SOURCES:
        out = os.path.join(out_dir, os.path.splitext(src)[0] + ".s")
        cmd = [HIPCC, *CFLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
