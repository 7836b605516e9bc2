"""Python access to ``liblds_probe.so`` (include/lds_probe.h): the measured
LDS bandwidth of the device, the roofline the decoder's message traffic is
compared with. Importing loads the library and raises if it is missing."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblds_probe.so")

READ, WRITE = 0, 1
WIDTHS = (4, 8, 16)


def _load():
    import torch  # noqa: F401  (one HIP runtime in the process, torch's)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2507_00254_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    lib.lds_probe_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_double), C.POINTER(C.c_float)]
    return lib


LIB = _load()


def run(kind: int, width: int, blocks_per_cu: int = 8, iters: int = 4096, stream=None) -> dict:
    """One timed probe launch: LDS bytes per second and its duration."""
    import torch
    st = torch.cuda.current_stream() if stream is None else stream
    bps = C.c_double(0.0)
    ms = C.c_float(0.0)
    rc = LIB.lds_probe_run(kind, width, blocks_per_cu, iters, C.c_void_p(st.cuda_stream), C.byref(bps),
                           C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"lds_probe_run({kind}, {width}, {blocks_per_cu}, {iters}) failed: {rc}")
    return {"kind": "read" if kind == READ else "write", "width": width, "blocks_per_cu": blocks_per_cu,
            "iters": iters, "GBps": bps.value / 1e9, "ms": ms.value}


def measure(blocks=(2, 4, 8), iters: int = 16384) -> dict:
    """Every kind and width at a few occupancies; the peak is the largest
    rate seen (the most generous denominator for the decoder)."""
    rows = [run(kind, w, b, iters) for kind in (READ, WRITE) for w in WIDTHS for b in blocks]
    best = max(rows, key=lambda r: r["GBps"])
    return {"peak_GBps": best["GBps"], "peak_at": {k: best[k] for k in ("kind", "width", "blocks_per_cu")},
            "rows": rows}
