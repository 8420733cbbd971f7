"""Build the e3mi HIP library for gfx950, in-tree.

Steps: compile and run the Clebsch-Gordan table generator (host C++), then
compile every HIP translation unit with hipcc and link libe3mi.so next to
this file. Object files go to _build/ at the repository root.

    python -m paper_2605_22698_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libe3mi.so")
SOURCES = ["graph.hip", "tp.hip", "tps.hip", "radial.hip", "first.hip", "last.hip", "node.hip", "md.hip", "grad.hip", "coulomb.hip", "product.hip", "api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def generate_tables() -> str:
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "gen_tables")
    _run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(CSRC, "gen_tables.cpp")])
    out = os.path.join(CSRC, "cg_tables.inc")
    _run([exe, out])
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    generate_tables()
    hipcc = _hipcc()
    jobs = jobs or min(8, os.cpu_count() or 1)

    def compile_one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
