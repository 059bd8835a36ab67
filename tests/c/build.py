"""Builds the plain C client of libidw (tests/c/idw_c_client) with gcc: include/idw.h and
the HIP runtime headers, linked against the in-tree libidw.so and libamdhip64 (rpath to
both, so it runs from the tree on any box)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "idw_c_client.c")
EXE = os.path.join(HERE, "idw_c_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out: str = EXE) -> list:
    pkg = os.path.join(ROOT, "paper_1402_4986_amd")
    return ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", SRC, "-o", out,
            f"-L{pkg}", "-lidw", f"-L{ROCM}/lib", "-lamdhip64",
            "-Wl,-rpath,$ORIGIN/../../paper_1402_4986_amd", f"-Wl,-rpath,{ROCM}/lib"]


def build(out: str = EXE) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(command(tmp))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
