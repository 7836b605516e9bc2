"""Launch shapes: every decodes-per-wave and grid size gives bit-identical
results and work counts, and the autotuner picks one of them."""
import numpy as np
import pytest

from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,p", [("bb72", 0.06), ("bb144", 0.05), ("bb288", 0.04)])
def test_every_tile_gives_the_same_results(name, p):
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs(name, p, 1500, tag=20)
    prm = U.oracle_params(k=6)
    h = B.bpsf_load_code(code.hx)
    try:
        opts = B.bpsf_tile_options(h)
        assert opts and opts == sorted(opts, reverse=True) and all(64 % d == 0 for d in opts)
        assert len(set(opts)) == len(opts)      # each D once, whichever families fit it
        ref = U.gpu_decode(code.hx, syn, p, prm, handle=h)
        o = U.oracle_decode(code.hx, syn, p, prm, precision="f32")
        assert len(U.mismatches(ref, o)) == 0
        for d in opts:
            for w in (0, 1, 3):
                print(f"{name} D={d} W={w}", flush=True)
                B.bpsf_set_tile(h, d, w)
                g = U.gpu_decode(code.hx, syn, p, prm, handle=h)
                assert len(U.mismatches(g, ref)) == 0, (d, w)
                assert g["stats"] == ref["stats"], (d, w)
        with pytest.raises(B.BpsfError):
            B.bpsf_set_tile(h, 32, 0)        # 2 lanes per decode: no family fits
    finally:
        B.bpsf_free_code(h)


def test_autotune_picks_a_listed_tile_and_keeps_results():
    import torch
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs("bb144", 0.03, 20000, tag=21)
    prm = U.oracle_params(k=6)
    h = B.bpsf_load_code(code.hx)
    try:
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
        s = torch.from_numpy(syn).cuda()
        t = B.bpsf_autotune(h, s, np.full(code.n, 0.03), bp, reps=2)
        print(t, flush=True)
        assert t["decodes_per_wave"] in B.bpsf_tile_options(h)
        assert t["waves_per_cu"] >= 1 and t["ms"] > 0 and t["candidates"] >= len(B.bpsf_tile_options(h))
        g = U.gpu_decode(code.hx, syn[:3000], 0.03, prm, handle=h)
        o = U.oracle_decode(code.hx, syn[:3000], 0.03, prm, precision="f32")
        assert len(U.mismatches(g, o)) == 0
    finally:
        B.bpsf_free_code(h)


def test_small_and_large_calls_agree():
    """A call of more than 4096 x D shots (D: the small family's decodes per
    wave for the code) runs the large family at its most decodes per wave,
    smaller calls the family with the fewest items per lane (and calls of at
    most 512 x D shots take D tasks at a time): the same shots decoded both
    ways give identical results, equal to the oracle's."""
    from paper_2507_00254_amd import bpsf as B
    for name, p in (("bb144", 0.05), ("bb288", 0.04), ("bb72", 0.06)):
        code, _, syn = U.inputs(name, p, 18000, tag=22)
        prm = U.oracle_params(k=6)
        h = B.bpsf_load_code(code.hx)
        try:
            print(f"{name}: one call of 18000, then 1500-shot and 300-shot calls", flush=True)
            big = U.gpu_decode(code.hx, syn, p, prm, handle=h)
            cuts = list(range(0, 9000, 1500)) + list(range(9000, 18000, 300)) + [18000]
            parts = [U.gpu_decode(code.hx, syn[a:b], p, prm, handle=h) for a, b in zip(cuts[:-1], cuts[1:])]
            for f in ("correction", "converged", "iterations"):
                assert np.array_equal(big[f], np.concatenate([q[f] for q in parts])), (name, f)
            o = U.oracle_decode(code.hx, syn[:1500], p, prm, precision="f32")
            assert len(U.mismatches(parts[0], o)) == 0, name
        finally:
            B.bpsf_free_code(h)
