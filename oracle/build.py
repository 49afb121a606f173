"""Build the CPU oracle (plain C, gcc) into ``oracle/liboracle.so``."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build() -> str:
    src = os.path.join(_HERE, "hyb_oracle.c")
    out = lib_path()
    tmp = out + ".tmp"
    # Plain IEEE double: no fast-math, no FMA contraction.  OpenMP runs the
    # FDM rows over z planes (same result for any thread count).
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
