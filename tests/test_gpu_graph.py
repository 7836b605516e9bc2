"""bpsf_decode and bpsf_mix_decode captured in a HIP graph: every replay, with
new inputs copied in and other eager work between replays, gives the eager
results (the calls enqueue kernels only once shapes, priors and parameters
have been seen)."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu


def test_decode_graph_replays():
    import torch
    from paper_2507_00254_amd import bpsf as B
    code, _, syn_all = U.inputs("bb144", 0.05, 4 * 2048, tag=30)
    prm = U.oracle_params(k=6)
    bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
    pri = np.full(code.n, 0.05)
    n = 2048
    h = B.bpsf_load_code(code.hx)
    try:
        s = torch.from_numpy(syn_all[:n].copy()).cuda()
        corr = torch.zeros((n, code.n), dtype=torch.uint8, device="cuda")
        conv = torch.zeros(n, dtype=torch.uint8, device="cuda")
        it = torch.zeros(n, dtype=torch.int32, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            B.bpsf_decode(h, s, pri, bp, corr, conv, it, side)       # warm: tables and scratch in place
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            B.bpsf_decode(h, s, pri, bp, corr, conv, it, torch.cuda.current_stream())
        for r in range(4):
            batch = syn_all[r * n:(r + 1) * n]
            s.copy_(torch.from_numpy(batch).cuda())
            junk = torch.randn(1 << 20, device="cuda").sum()        # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = {"correction": corr.cpu().numpy(), "converged": conv.cpu().numpy(), "iterations": it.cpu().numpy()}
            o = U.oracle_decode(code.hx, batch, 0.05, prm, precision="f32")
            print(f"replay {r}: {len(U.mismatches(got, o))} mismatches {float(junk):.1f}", flush=True)
            assert len(U.mismatches(got, o)) == 0
    finally:
        B.bpsf_free_code(h)


def test_mix_graph_replays():
    import torch
    from paper_2507_00254_amd import bpsf as B
    hs = [codes.get_code(nm).hx for nm in ("bb72", "bb144", "bb288")]
    p = 0.05
    prm = U.oracle_params(k=6)
    bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
    pri = [np.full(h.shape[1], p) for h in hs]
    handles = [B.bpsf_load_code(h) for h in hs]
    mix = B.bpsf_mix_create(handles)
    try:
        batches = [shots.mixed_batch(hs, p, 400, shots.stream_key(shots.MASTER_SEED, 940 + r)) for r in range(3)]
        n = len(batches[0][0])
        d_sc = torch.from_numpy(batches[0][0]).cuda()
        d_syn = torch.from_numpy(batches[0][1]).cuda()
        corr = torch.zeros((n, 288), dtype=torch.uint8, device="cuda")
        conv = torch.zeros(n, dtype=torch.uint8, device="cuda")
        it = torch.zeros(n, dtype=torch.int32, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            B.bpsf_mix_decode(mix, d_sc, d_syn, pri, bp, corr, conv, it, side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            B.bpsf_mix_decode(mix, d_sc, d_syn, pri, bp, corr, conv, it, torch.cuda.current_stream())
        for r, (sc, syn, _, _) in enumerate(batches):
            d_sc.copy_(torch.from_numpy(sc).cuda())
            d_syn.copy_(torch.from_numpy(syn).cuda())
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for c, h in enumerate(hs):
                sel = np.nonzero(sc == c)[0]
                got = {"correction": corr.cpu().numpy()[sel, :h.shape[1]], "converged": conv.cpu().numpy()[sel],
                       "iterations": it.cpu().numpy()[sel]}
                o = U.oracle_decode(h, syn[sel, :h.shape[0]], p, prm, precision="f32")
                assert len(U.mismatches(got, o)) == 0, (r, c)
            print(f"mix replay {r} ok", flush=True)
    finally:
        B.bpsf_mix_free(mix)
        for x in handles:
            B.bpsf_free_code(x)
