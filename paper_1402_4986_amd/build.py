"""Builds libidw.so for gfx950 in-tree with hipcc (parallel per translation unit).

Usage: python -m paper_1402_4986_amd.build [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libidw.so")
ARCH = "gfx950"

# Packed FP32 instructions are disabled on purpose (-packed-fp32-ops).
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
            "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]

LAYOUTS = [("soa", 0), ("aos", 1), ("aoas", 2), ("hybrid", 3), ("soaos", 4)]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


TUNING = os.path.join(HERE, "tuning", f"{ARCH}.json")


def tuned_defines(path: str = TUNING) -> list:
    """The autotuned batched-plan parameters (written by paper_1402_4986_amd.autotune) as
    compile-time defaults of the library; none when the table is absent."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return []
    out = []
    for key, macro in (("batch_chunk", "IDW_TUNED_BATCH_CHUNK"), ("batch_workgroups", "IDW_TUNED_BATCH_WORKGROUPS")):
        v = int(t.get(key, 0))
        if v > 0:
            out.append(f"-D{macro}={v}")
    return out


def _units():
    units = []
    for name, idx in LAYOUTS:
        units.append((os.path.join(CSRC, "idw_layout.hip"), os.path.join(BUILD, f"idw_layout_{name}.o"),
                      [f"-DIDW_LAYOUT={idx}", f"-DIDW_LAYOUT_NAME={name}"]))
    for src in ("idw_common.hip", "idw_batched.hip", "idw_api.cpp"):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        extra = ["-x", "hip"] if src.endswith(".cpp") else []
        if src == "idw_batched.hip":
            extra = extra + tuned_defines()
        units.append((os.path.join(CSRC, src), obj, extra))
    return units


def _compile(hipcc, src, obj, extra):
    cmd = [hipcc] + HIPFLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every translation unit and link libidw.so; returns the library path."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, hipcc, *u) for u in units]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    build(ap.parse_args().j)
