"""Build libfsp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2405_02603_amd.build [--jobs N] [--debug]

Each .hip translation unit is compiled to an object in parallel, then linked
into ``paper_2405_02603_amd/libfsp.so``.  Always recompiles.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfsp.so")
ARCH = os.environ.get("FSP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "serve_engine.hip", "greens.hip", "solve_f32.hip", "solve_f64.hip", "solve_rows_f32.hip", "solve_rows_f64.hip",
           "solve_cols_f32.hip", "solve_cols_f64.hip", "solve_plane_f32.hip", "solve_plane_f64.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(debug: bool, defines=()):
    f = [f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
         # packed fp32 instructions stay off: only scalar/vector fp32 forms are emitted
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]
    f += ["-O1", "-g"] if debug else ["-O3"]
    f += [f"-D{d}" for d in defines]
    return f


def compile_one(src: str, debug: bool, defines=(), build_dir: str = BUILD) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *flags(debug, defines), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 4, debug: bool = False, verbose: bool = False, defines=(), out: str = LIB) -> str:
    build_dir = BUILD if out == LIB else os.path.join(BUILD, "alt")
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug, defines, build_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--define", action="append", default=[], help="extra preprocessor definition")
    ap.add_argument("--out", default=LIB, help="output library path")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug, verbose=True, defines=a.define, out=os.path.abspath(a.out))


if __name__ == "__main__":
    sys.exit(main())
