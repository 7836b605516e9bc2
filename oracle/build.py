"""Compile the CPU oracle (test infrastructure) into two shared libraries.

``liboracle_f64.so`` computes in double (the reference precision) and
``liboracle_f32.so`` is the same source in float, used where a float decision
must be compared in float.  Both are built with ``-ffp-contract=off`` so no
multiply-add is fused.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bpsf_oracle.c")
VARIANTS = {"f64": ("double", "_f64"), "f32": ("float", "_f32")}


def lib_path(prec: str) -> str:
    return os.path.join(HERE, f"liboracle_{prec}.so")


def build(force: bool = True, src: str = SRC, out_dir: str = HERE, extra_defines=(),
          variants=("f64", "f32")) -> dict:
    out = {}
    for prec in variants:
        real, suffix = VARIANTS[prec]
        dst = os.path.join(out_dir, f"liboracle_{prec}.so")
        if not force and os.path.exists(dst) and os.path.getmtime(dst) >= os.path.getmtime(src):
            out[prec] = dst
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wno-unused-function", f"-DREAL={real}", f"-DSUFFIX={suffix}",
               *[f"-D{d}" for d in extra_defines], src, "-o", dst + ".tmp", "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(dst + ".tmp", dst)
        out[prec] = dst
    return out


if __name__ == "__main__":
    print(build())
