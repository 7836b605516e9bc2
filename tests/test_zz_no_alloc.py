"""bpsf_decode_noalloc (scratch in the library's fixed device array) against
bpsf_decode on the same inputs: two calls in a row, the second smaller (and
taking the small-call kernel family, whose records are longer), a wide code,
and a call too large for the fixed array, which is refused before any work."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu


def _both(B, handle, syn, n_bits, pri, bp):
    import torch
    s = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
    out = {}
    for mode in (False, True):
        corr = torch.full((len(syn), n_bits), 7, dtype=torch.uint8, device="cuda")
        conv = torch.full((len(syn),), 7, dtype=torch.uint8, device="cuda")
        it = torch.full((len(syn),), -1, dtype=torch.int32, device="cuda")
        B.bpsf_decode(handle, s, pri, bp, corr, conv, it, noalloc=mode)
        torch.cuda.synchronize()
        out[mode] = {"correction": corr.cpu().numpy(), "converged": conv.cpu().numpy(),
                     "iterations": it.cpu().numpy(), "stats": B.bpsf_last_stats(handle)}
    return out[False], out[True]


def test_noalloc_equals_decode_two_calls():
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs("bb144", 0.05, 20_000, tag=51)
    pri = np.full(code.n, 0.05)
    bp = B.make_params(precision=B.PREC_FP32)
    h = B.bpsf_load_code(code.hx)
    try:
        for n in (20_000, 3_000):
            print(f"[[144]] {n} shots", flush=True)
            ref, got = _both(B, h, syn[:n], code.n, pri, bp)
            assert len(U.mismatches(got, ref)) == 0
            # the fixed scratch keeps no trial corrections: its last phase
            # re-runs the winners that the other call copies
            assert ref["stats"]["rerun_iterations"] == 0 and got["stats"]["rerun_iterations"] > 0
            same = {k: v for k, v in got["stats"].items() if k != "rerun_iterations"}
            assert same == {k: v for k, v in ref["stats"].items() if k != "rerun_iterations"}
            assert got["stats"]["failed_shots"] > 0 and got["stats"]["errors"] == 0
    finally:
        B.bpsf_free_code(h)


def test_noalloc_wide_code():
    from paper_2507_00254_amd import bpsf as B
    h = codes.phenomenological(codes.bb144().hx, 12)
    _, syn = shots.make_shots(h, 0.005, 300, shots.stream_key(shots.MASTER_SEED, 52))
    pri = np.full(h.shape[1], 0.005)
    bp = B.make_params(max_iter=200, cand_max_iter=30, k=8, precision=B.PREC_FP32)
    handle = B.bpsf_load_code(h)
    try:
        print("phenomenological 300 shots", flush=True)
        ref, got = _both(B, handle, syn, h.shape[1], pri, bp)
        assert len(U.mismatches(got, ref)) == 0
        assert got["stats"] == ref["stats"] and got["stats"]["failed_shots"] > 0
    finally:
        B.bpsf_free_code(handle)


def test_noalloc_refuses_oversized_calls():
    import torch
    from paper_2507_00254_amd import bpsf as B
    code = codes.bb144()
    n = 200_000   # 272 bytes of scratch per shot: about 52 MiB, above the 32 MiB array
    handle = B.bpsf_load_code(code.hx)
    try:
        s = torch.zeros((n, 72), dtype=torch.uint8, device="cuda")
        corr = torch.full((n, code.n), 7, dtype=torch.uint8, device="cuda")
        conv = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        with pytest.raises(B.BpsfError, match="fixed scratch") as ei:
            B.bpsf_decode(handle, s, np.full(code.n, 0.05), B.make_params(), corr, conv, it, noalloc=True)
        assert ei.value.code == B.BPSF_EINVAL
        torch.cuda.synchronize()
        assert int(conv.max().item()) == 7 and int(conv.min().item()) == 7   # nothing was enqueued
    finally:
        B.bpsf_free_code(handle)
