"""Layered BP schedule (BPSF_FLAG_LAYERED): exact parity with the oracle's
layered schedule in both precisions, on every one-wave code family, per
iteration (traces) and under the options; the calls that do not take it
report BPSF_ENOTSUP."""
import numpy as np
import pytest

from oracle.oracle import LAYERED
from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,p,k,n", [("bb72", 0.06, 6, 2000), ("bb144", 0.05, 6, 2000), ("bb288", 0.04, 6, 800),
                                        ("gb254", 0.05, 6, 800), ("cbb126", 0.05, 6, 1000)])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_layered_parity(name, p, k, n, precision):
    code, _, syn = U.inputs(name, p, n, tag=70)
    prm = U.oracle_params(k=k, flags=LAYERED)
    g = U.gpu_decode(code.hx, syn, p, prm, precision=precision)
    o = U.oracle_decode(code.hx, syn, p, prm, precision=precision)
    bad = U.mismatches(g, o)
    print(f"layered {name} p={p} {precision}: failed {g['stats']['failed_shots']} mismatches {len(bad)}", flush=True)
    assert len(bad) == 0
    assert g["stats"]["errors"] == 0
    assert g["stats"]["main_iterations"] == int(o["main_iterations"].sum())
    assert g["stats"]["failed_shots"] > 0          # the trials ran


def test_layered_differs_from_flooding():
    """The flag reaches the kernels: on shots where BP struggles the two
    schedules take different iteration counts."""
    code, _, syn = U.inputs("bb144", 0.05, 500, tag=71)
    lay = U.gpu_decode(code.hx, syn, 0.05, U.oracle_params(k=0, flags=LAYERED))
    flo = U.gpu_decode(code.hx, syn, 0.05, U.oracle_params(k=0))
    assert (lay["iterations"] != flo["iterations"]).any()
    # layered BP converges in fewer iterations on average
    assert lay["iterations"].mean() < flo["iterations"].mean()


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name", ["bb144", "gb254"])
def test_layered_traces_exact(name, precision):
    from oracle.oracle import OracleLib
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs(name, 0.06, 40, tag=72)
    O = OracleLib()
    prm = U.oracle_params(k=0, max_iter=30, alpha=0.0, flags=LAYERED)
    handle = B.bpsf_load_code(code.hx)
    try:
        bp = B.make_params(max_iter=30, k=0, alpha=0.0, flags=B.FLAG_LAYERED,
                           precision=B.PREC_FP64 if precision == "f64" else B.PREC_FP32)
        for i in range(len(syn)):
            o = O.bp(code.hx, syn[i], 0.06, prm, max_iter=30, prec=precision, trace=True)
            g = B.bpsf_bp_trace(handle, syn[i], np.full(code.n, 0.06), bp)
            assert g["iterations"] == o["iterations"] and g["converged"] == o["converged"], i
            assert np.array_equal(g["hard"], o["hard"]), i
            assert np.array_equal(g["trace_lout"], o["trace_lout"]), i
            assert np.array_equal(g["trace_c2v"], o["trace_c2v"]), i
    finally:
        B.bpsf_free_code(handle)


@pytest.mark.parametrize("opts", [dict(k=6, alpha=0.0), dict(k=6, select_mode=1), dict(k=8, cand_mode=1, w_max=2),
                                  dict(k=6, select_mode=1, flags=4), dict(k=4, flags=2), dict(k=6, flags=1),
                                  dict(k=0)])
def test_layered_options(opts):
    code, _, syn = U.inputs("bb72", 0.07, 1500, tag=73)
    o_flags = opts.pop("flags", 0)
    prm = U.oracle_params(flags=LAYERED | o_flags, **opts)
    g = U.gpu_decode(code.hx, syn, 0.07, prm)
    o = U.oracle_decode(code.hx, syn, 0.07, prm, precision="f32")
    assert len(U.mismatches(g, o)) == 0


def test_layered_nonuniform_priors_and_launch_shapes():
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs("bb144", 0.05, 1200, tag=74)
    pri = np.random.default_rng(11).uniform(0.02, 0.08, code.n)
    prm = U.oracle_params(k=6, flags=LAYERED)
    o = U.oracle_decode(code.hx, syn, pri, prm, precision="f32")
    h = B.bpsf_load_code(code.hx)
    try:
        for D in B.bpsf_tile_options(h):
            B.bpsf_set_tile(h, D, 0)
            g = U.gpu_decode(code.hx, syn, pri, prm, handle=h)
            assert len(U.mismatches(g, o)) == 0, D
    finally:
        B.bpsf_free_code(h)


def test_layered_edge_batches():
    """One shot, an all-zero batch, and a batch whose size is not a multiple of
    anything the launch uses."""
    code, _, syn = U.inputs("bb288", 0.05, 333, tag=75)
    prm = U.oracle_params(k=6, flags=LAYERED)
    for s in (syn[:1], np.zeros((17, code.hx.shape[0]), np.uint8), syn):
        g = U.gpu_decode(code.hx, s, 0.05, prm)
        o = U.oracle_decode(code.hx, s, 0.05, prm, precision="f32")
        assert len(U.mismatches(g, o)) == 0


def test_layered_not_supported_elsewhere():
    import torch
    from paper_2507_00254_amd import bpsf as B
    h72 = codes.get_code("bb72").hx
    a = B.bpsf_load_code(h72)
    wide = B.bpsf_load_code(codes.phenomenological(h72, 4))
    try:
        bp = B.make_params(100, 20, 4, alpha=0.625, flags=B.FLAG_LAYERED, precision=B.PREC_FP32)
        # a wide code
        m2, n2 = codes.phenomenological(h72, 4).shape
        s = torch.zeros((4, m2), dtype=torch.uint8, device="cuda")
        corr = torch.zeros((4, n2), dtype=torch.uint8, device="cuda")
        conv = torch.zeros(4, dtype=torch.uint8, device="cuda")
        it = torch.zeros(4, dtype=torch.int32, device="cuda")
        with pytest.raises(B.BpsfError) as ei:
            B.bpsf_decode(wide, s, np.full(n2, 0.01), bp, corr, conv, it)
        assert ei.value.code == B.BPSF_ENOTSUP
        # a mixed-code call
        mix = B.bpsf_mix_create([a])
        try:
            sc = torch.zeros(4, dtype=torch.int32, device="cuda")
            s1 = torch.zeros((4, 36), dtype=torch.uint8, device="cuda")
            c1 = torch.zeros((4, 72), dtype=torch.uint8, device="cuda")
            with pytest.raises(B.BpsfError) as ei:
                B.bpsf_mix_decode(mix, sc, s1, [np.full(72, 0.05)], bp, c1, conv, it)
            assert ei.value.code == B.BPSF_ENOTSUP
        finally:
            B.bpsf_mix_free(mix)
        # the request loop
        with pytest.raises(B.BpsfError) as ei:
            B.Server([a], [np.full(72, 0.05)], bp, lanes=1, max_batch_shots=64)
        assert ei.value.code == B.BPSF_ENOTSUP
    finally:
        B.bpsf_free_code(wide)
        B.bpsf_free_code(a)


def test_layered_f32_against_f64():
    """Float GPU messages against the double oracle under the layered
    schedule: the bar of the flooding schedule (identical corrections on at
    least 99.99% of shots, the LER inside the oracle's 95% interval)."""
    from tests.test_gpu_statistical import _logical_failures
    code, err, syn = U.inputs("bb144", 0.03, 20000, tag=76)
    prm = U.oracle_params(k=6, flags=LAYERED)
    o = U.oracle_decode(code.hx, syn, 0.03, prm, precision="f64")
    g = U.gpu_decode(code.hx, syn, 0.03, prm, precision="f32")
    same = (g["correction"] == o["correction"]).all(axis=1) & (g["converged"] == o["converged"])
    print(f"identical shots {same.mean():.6f} ({(~same).sum()} differ)", flush=True)
    assert same.mean() >= 0.9999
    fo = _logical_failures(code, err, o)
    fg = _logical_failures(code, err, g)
    lo, hi = U.wilson(int(fo.sum()), len(syn))
    assert lo <= fg.mean() <= hi
