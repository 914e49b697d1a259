"""Build libfill.so (HIP, gfx950) in-tree.

Every source under csrc/ is compiled with hipcc for gfx950 into
_build/*.o (in parallel) and linked into libfill.so next to this file.
Usage: python paper_1109_0286_amd/build.py  (runs without importing the package).

build(variant=v, rows=r, lib=path) builds a candidate library in which every
FFT kernel uses radix-plan variant v and every row pass r times the default
rows per workgroup (the autotuner's candidates) instead of the tuned table.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfill.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["k_f64.hip", "k_f32.hip", "k_misc.hip", "k_adjoint.hip", "k_strips.hip", "k_block.hip", "fill_api.cpp",
           "strips.cpp", "block.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept off: some of their forms have given
    # wrong results on this chip, with no error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True, variant: int | None = None, lib: str = LIB, rows: int | None = None) -> str:
    tag = "" if variant is None else f"variant{variant}" + ("" if rows is None else f"_rows{rows}")
    build_dir = BUILD if variant is None else os.path.join(BUILD, tag)
    extra = () if variant is None else (f"-DFILL_FFT_FORCE_VARIANT={int(variant)}",)
    if rows is not None:
        extra = extra + (f"-DFILL_FFT_FORCE_ROWS={int(rows)}",)
    os.makedirs(build_dir, exist_ok=True)
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), SOURCES))
    tmp = lib + ".tmp"
    # rocSOLVER (with rocBLAS): the block preconditioner's dense inverses at set-up
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrocsolver", "-lrocblas"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build()
