"""Build ``libbpsf.so`` (HIP, gfx950) in-tree with hipcc.

The kernels are compiled with ``-ffp-contract=off`` (no fused multiply-add,
so float arithmetic matches a plain C evaluation of the same expressions) and
``-fno-honor-nans`` (no NaN can reach the message arithmetic; this lets min and
max take their operands without canonicalization). The host runtime is
compiled without ``-fno-honor-nans`` because it validates user input.
Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbpsf.so")
PROBE_LIB = os.path.join(HERE, "liblds_probe.so")
ARCH = os.environ.get("BPSF_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-variable",
          "-Wno-unused-but-set-variable"]
# units of libbpsf.so (lds_probe.hip builds liblds_probe.so on its own)
UNITS = [("bpsf_kernels.hip", ["-fno-honor-nans"]), ("bpsf_wide.hip", ["-fno-honor-nans"]),
         ("bpsf_sparse.hip", ["-fno-honor-nans"]), ("bpsf_sparse_layout.hip", []), ("bpsf_api.hip", []),
         ("bpsf_server.hip", [])]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".h"))] + [os.path.join(os.path.dirname(HERE), "include", "bpsf.h")]


def _wait(proc_cmd) -> None:
    proc, cmd = proc_cmd
    if proc.wait() != 0:
        raise subprocess.CalledProcessError(proc.returncode, cmd)


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    # the LDS bandwidth probe: a library of its own (include/lds_probe.h)
    probe_cmd = ["hipcc", *COMMON, "-shared", os.path.join(CSRC, "lds_probe.hip"), "-o", PROBE_LIB + ".tmp"]
    if verbose:
        print(" ".join(probe_cmd), flush=True)
    procs.append((subprocess.Popen(probe_cmd), probe_cmd))
    # the units compile in parallel (at most four at a time)
    for src, extra in UNITS:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = ["hipcc", *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        if len(procs) >= 4:
            _wait(procs.pop(0))
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for pr in procs:
        _wait(pr)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
