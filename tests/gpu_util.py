"""Helpers shared by the GPU tests: seeded inputs, a GPU decode through the C
ABI, the oracle on the same inputs, and comparisons."""
from __future__ import annotations

import numpy as np

from oracle.oracle import OracleLib, Params
from workloads import codes, shots

_O = OracleLib()


def inputs(code_name: str, p: float, n: int, tag: int = 0):
    code = codes.get_code(code_name)
    key = shots.stream_key(shots.MASTER_SEED, 500 + tag, code.n, int(round(p * 100000)))
    err, syn = shots.make_shots(code.hx, p, n, key)
    return code, err, syn


def oracle_params(max_iter=100, cand_max_iter=20, k=6, cand_mode=0, w_max=1, select_mode=0, alpha=0.625,
                  flags=0) -> Params:
    return Params(max_iter=max_iter, cand_max_iter=cand_max_iter, k=k, cand_mode=cand_mode, w_max=w_max,
                  select_mode=select_mode, alpha=alpha, flags=flags)


def gpu_decode(h, syn, priors, prm: Params, precision: str = "f32", handle=None):
    import torch
    from paper_2507_00254_amd import bpsf as B
    own = handle is None
    if own:
        handle = B.bpsf_load_code(h)
    try:
        m, n = h.shape
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, prm.cand_mode, prm.w_max, prm.select_mode,
                           prm.alpha, prm.flags, B.PREC_FP64 if precision == "f64" else B.PREC_FP32)
        s = torch.from_numpy(np.ascontiguousarray(syn, dtype=np.uint8)).cuda()
        corr = torch.full((len(syn), n), 7, dtype=torch.uint8, device="cuda")
        conv = torch.full((len(syn),), 7, dtype=torch.uint8, device="cuda")
        it = torch.full((len(syn),), -1, dtype=torch.int32, device="cuda")
        pri = np.broadcast_to(np.asarray(priors, np.float64), (n,))
        B.bpsf_decode(handle, s, pri, bp, corr, conv, it)
        torch.cuda.synchronize()
        st = B.bpsf_last_stats(handle)
        return {"correction": corr.cpu().numpy(), "converged": conv.cpu().numpy(),
                "iterations": it.cpu().numpy(), "stats": st}
    finally:
        if own:
            B.bpsf_free_code(handle)


def oracle_decode(h, syn, priors, prm: Params, precision: str = "f64", threads: int = 8):
    return _O.bpsf_batch(h, syn, priors, prm, prec=precision, threads=threads)


def mismatches(g, o):
    bad = np.zeros(len(o["converged"]), bool)
    bad |= (g["correction"] != o["correction"]).any(axis=1)
    bad |= g["converged"] != o["converged"]
    bad |= g["iterations"] != o["iterations"]
    return np.nonzero(bad)[0]


def wilson(k: int, n: int, z: float = 1.959963984540054):
    if n == 0:
        return 0.0, 1.0
    ph = k / n
    den = 1 + z * z / n
    cen = (ph + z * z / (2 * n)) / den
    half = z * np.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return cen - half, cen + half
