"""Compile the HIP library (libbsm.so) for gfx950, in-tree.

hipcc cross-compiles without a GPU.  Host-only planner sources are compiled with g++; the HIP
sources (kernels and the C ABI) with hipcc, the FP64/FP32 tile kernel once per instantiation so
that they compile in parallel; the objects are linked into one shared library next to this file.
Every build recompiles from scratch.
"""
from __future__ import annotations

import glob
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed FP32 instructions are kept out of every kernel
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


TILE_UNIT = "kernels_tile.hip"
B3_UNIT = "kernels_bf16x3.hip"


def tile_variant_ids(table="BSM_TILE_VARIANTS"):
    """Variant ids of a tile-variant table (BSM_TILE_VARIANTS, BSM_BF16_VARIANTS) in csrc/types.hpp."""
    text = open(os.path.join(CSRC, "types.hpp")).read()
    body = text[text.index(f"#define {table}(X)"):]
    body = body[:body.index("\n\n")]
    return [int(m) for m in re.findall(r"X\((\d+),", body)]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("command failed: " + " ".join(cmd))
    return out


def build(verbose: bool = False) -> str:
    if os.path.isdir(BUILD):
        shutil.rmtree(BUILD)
    os.makedirs(BUILD)
    jobs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        jobs.append((["g++"] + CXX_FLAGS + ["-c", src, "-o", obj], obj))
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        if os.path.basename(src) in (TILE_UNIT, B3_UNIT):
            continue
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        jobs.append(([HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj], obj))
    # the FP64/FP32 tile kernel: one translation unit per (form, variant, window kind)
    unit = os.path.join(CSRC, TILE_UNIT)
    for form in (0, 1):
        for vid in tile_variant_ids():
            for resume in (0, 1):
                obj = os.path.join(BUILD, f"tile_{form}_{vid}_{resume}.o")
                defs = [f"-DBSM_UNIT_FORM={form}", f"-DBSM_UNIT_ID={vid}", f"-DBSM_UNIT_RESUME={resume}"]
                jobs.append(([HIPCC] + HIP_FLAGS + defs + ["-c", unit, "-o", obj], obj))
    unit = os.path.join(CSRC, B3_UNIT)
    for vid in tile_variant_ids("BSM_BF16_VARIANTS"):
        for resume in (0, 1):
            obj = os.path.join(BUILD, f"tile_b3_{vid}_{resume}.o")
            defs = [f"-DBSM_B3_UNIT_ID={vid}", f"-DBSM_B3_UNIT_RESUME={resume}"]
            jobs.append(([HIPCC] + HIP_FLAGS + defs + ["-c", unit, "-o", obj], obj))
    # longest first: the tile units dominate
    jobs.sort(key=lambda j: 0 if os.path.basename(j[1]).startswith("tile_") else 1)
    # translation units compile independently (the tile kernels dominate; one per form)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for out in outs:
            if out:
                print(out)
    objs = [j[1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
