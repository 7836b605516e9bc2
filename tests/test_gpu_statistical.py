"""Float GPU messages against the double oracle.

The bar: identical corrections on at least 99.99% of shots at every
configuration point, every converged output solving its syndrome, and a
logical error rate inside the oracle's 95% Wilson interval on the same shots.
Per-iteration marginals and c2v messages stay within 1e-4 relative error (mixed criterion, see _close) until the two
precisions first take different hard decisions.
"""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, gf2

pytestmark = pytest.mark.gpu


def _logical_failures(code, err, res):
    lx = gf2.logical_basis(code.hx, code.hz)
    resid = (err ^ res["correction"]).astype(np.int64)
    flips = ((resid @ lx.T.astype(np.int64)) & 1).any(axis=1)
    return (res["converged"] == 0) | flips


# Float GPU and double oracle on the same seeded shots, decoded once per point
# and shared by the tests below (the configuration sizes: 2x10^5 shots per
# point; [[144]] at p = 0.03, the benchmark point, runs 10^6 shots in
# test_gpu_fullsize).
_RUNS = {}


def _run(code_name, p, n, k):
    key = (code_name, p, n, k)
    if key not in _RUNS:
        print(f"case {code_name} p={p} n={n} k={k}", flush=True)
        code, err, syn = U.inputs(code_name, p, n, tag=11)
        prm = U.oracle_params(k=k)
        o = U.oracle_decode(code.hx, syn, p, prm, precision="f64", threads=16)
        g = U.gpu_decode(code.hx, syn, p, prm, precision="f32")
        same = (g["correction"] == o["correction"]).all(axis=1) & (g["converged"] == o["converged"])
        print(f"  identical shots {same.mean():.6f} ({(~same).sum()} differ)", flush=True)
        _RUNS.clear()       # keep one point's arrays at a time
        _RUNS[key] = (code, err, syn, prm, o, g, same)
    return _RUNS[key]


# The configuration points run with float messages: [[144]] over the error
# rates of the float-message configuration and the codes of the five-code
# batch at p = 0.03. [[72,12,6]] misses the bar in float: its first BP
# oscillates without converging on about 3.6% of shots, and on about one in
# nine of those 100 iterations of oscillation amplify the float-vs-double
# rounding into a different hard decision (0.39% of shots differ, every one
# with a capped double first BP; the logical error rate stays inside the
# interval, and the double GPU path is bit-exact, test_config1_double_is_exact).
CONFIG_POINTS = [
    ("bb144", 0.01, 200_000, 6), ("bb144", 0.02, 200_000, 6), ("bb144", 0.05, 200_000, 6),
    ("bb90", 0.03, 200_000, 6), ("bb108", 0.03, 200_000, 6), ("bb288", 0.03, 200_000, 6),
    pytest.param("bb72", 0.03, 200_000, 6, marks=pytest.mark.xfail(
        strict=True, reason="[[72,12,6]] in float: 0.39% of shots differ from the double oracle, all on "
                            "first BPs that oscillate to the iteration cap")),
]


@pytest.mark.parametrize("code_name,p,n,k", CONFIG_POINTS)
def test_fp32_agrees_with_fp64_oracle(code_name, p, n, k):
    """>= 99.99% of shots identical (correction and converged flag)."""
    *_, same = _run(code_name, p, n, k)
    assert same.mean() >= 0.9999


# the configuration points, and [[72]] at p = 0.05 (reported, not a
# configuration point: that workload specifies double messages)
@pytest.mark.parametrize("code_name,p,n,k", [tuple(pt.values) if hasattr(pt, "marks") else pt
                                             for pt in CONFIG_POINTS] + [("bb72", 0.05, 20_000, 4)])
def test_fp32_logical_error_rate_and_divergence(code_name, p, n, k):
    """The logical error rate lies in the oracle's Wilson 95% interval on the
    same shots, every converged output solves its syndrome, and every shot
    that differs is one whose double first BP ran to the iteration cap."""
    code, err, syn, prm, o, g, same = _run(code_name, p, n, k)
    assert (o["main_iterations"][~same] == prm.max_iter).all()
    sg = (g["correction"].astype(np.int64) @ code.hx.T.astype(np.int64)) & 1
    assert (sg[g["converged"] == 1] == syn[g["converged"] == 1]).all()
    fo = _logical_failures(code, err, o)
    fg = _logical_failures(code, err, g)
    lo, hi = U.wilson(int(fo.sum()), n)
    ler = fg.mean()
    print(f"  LER gpu {ler:.3e} oracle {fo.mean():.3e} CI [{lo:.3e}, {hi:.3e}]", flush=True)
    assert lo <= ler <= hi


def test_config1_double_is_exact():
    """[[72,12,6]], p = 0.05, 10^4 shots, double messages, |Phi| = 4 (16 trials
    of 20 iterations): the double GPU path equals the double oracle on every
    shot (correction, converged, iterations), and so does the logical error
    rate with its Wilson interval."""
    code, err, syn = U.inputs("bb72", 0.05, 10_000, tag=31)
    prm = U.oracle_params(k=4)
    o = U.oracle_decode(code.hx, syn, 0.05, prm, precision="f64", threads=16)
    g = U.gpu_decode(code.hx, syn, 0.05, prm, precision="f64")
    assert len(U.mismatches(g, o)) == 0
    assert g["stats"]["failed_shots"] == int(((o["winner"] >= 0) | (o["converged"] == 0)).sum()) > 0
    fo = _logical_failures(code, err, o)
    lo, hi = U.wilson(int(fo.sum()), len(syn))
    print(f"  LER {fo.mean():.4e} CI [{lo:.4e}, {hi:.4e}]", flush=True)
    assert lo <= _logical_failures(code, err, g).mean() <= hi


def _phen_failures(h_code, rounds, err, res):
    """Phenomenological shots: a failure when the decoder did not converge, or
    the data residual folded over the rounds flips a logical operator."""
    n = h_code.hx.shape[1]
    resid = (err ^ res["correction"])[:, :rounds * n].reshape(len(err), rounds, n)
    folded = np.bitwise_xor.reduce(resid, axis=1).astype(np.int64)
    lx = gf2.logical_basis(h_code.hx, h_code.hz)
    return (res["converged"] == 0) | ((folded @ lx.T.astype(np.int64)) & 1).any(axis=1)


@pytest.mark.parametrize("p,n", [(0.002, 100_000), (0.005, 50_000)])
def test_phenomenological_fp32_against_fp64_oracle(p, n):
    """The phenomenological configuration ([[144]] over 12 rounds, 864 x 2592,
    200 first-BP iterations, |Phi| = 8: 256 trials of 30 iterations) in float
    against the double oracle: >= 99.99% identical shots, failed first BPs
    present, logical error rate inside the interval."""
    from workloads import shots
    c = codes.bb144()
    h = codes.phenomenological(c.hx, 12)
    err, syn = shots.make_shots(h, p, n, shots.stream_key(shots.MASTER_SEED, 41, h.shape[1], int(round(p * 1e5))))
    prm = U.oracle_params(max_iter=200, cand_max_iter=30, k=8)
    print(f"phen p={p} n={n}", flush=True)
    g = U.gpu_decode(h, syn, p, prm, precision="f32")
    print(f"  gpu done: {g['stats']['failed_shots']} failed first BPs", flush=True)
    o = U.oracle_decode(h, syn, p, prm, precision="f64", threads=16)
    same = (g["correction"] == o["correction"]).all(axis=1) & (g["converged"] == o["converged"])
    print(f"  identical shots {same.mean():.6f} ({(~same).sum()} differ)", flush=True)
    assert same.mean() >= 0.9999
    assert g["stats"]["failed_shots"] == int(((o["winner"] >= 0) | (o["converged"] == 0)).sum()) > 0
    assert g["stats"]["errors"] == 0
    fo = _phen_failures(c, 12, err, o)
    fg = _phen_failures(c, 12, err, g)
    lo, hi = U.wilson(int(fo.sum()), n)
    print(f"  LER gpu {fg.mean():.3e} oracle {fo.mean():.3e} CI [{lo:.3e}, {hi:.3e}]", flush=True)
    assert lo <= fg.mean() <= hi


def _close(g, o, lmin, rel=1e-4):
    """|g - o| <= rel * max(|o|, min channel LLR): relative for messages of
    channel size and above, absolute at that scale for near-zero ones."""
    return np.abs(g.astype(np.float64) - o) <= rel * np.maximum(np.abs(o), lmin)


@pytest.mark.parametrize("code_name,p", [("bb144", 0.05), ("bb72", 0.08), ("bb288", 0.04)])
def test_llr_messages_within_1e4(code_name, p):
    from oracle.oracle import OracleLib
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs(code_name, p, 400, tag=12)
    O = OracleLib()
    prm = U.oracle_params(k=0, max_iter=60)
    lmin = float(np.log((1 - p) / p))
    handle = B.bpsf_load_code(code.hx)
    worst, compared, fails = 0.0, 0, 0
    try:
        bp = B.make_params(max_iter=60, k=0, alpha=0.625, precision=B.PREC_FP32)
        # include shots where BP struggles: they exercise long message histories
        for i in range(0, len(syn), 10):
            o = O.bp(code.hx, syn[i], p, prm, max_iter=60, trace=True)
            g = B.bpsf_bp_trace(handle, syn[i], np.full(code.n, p), bp)
            fails += int(not o["converged"])
            its = min(o["iterations"], g["iterations"])
            for t in range(its):
                if not np.array_equal(o["trace_hard"][t], (g["trace_lout"][t] <= 0).astype(np.uint8)):
                    break   # the precisions took different decisions: later messages differ legitimately
                ok_l = _close(g["trace_lout"][t], o["trace_lout"][t], lmin)
                ok_c = _close(g["trace_c2v"][t], o["trace_c2v"][t], lmin)
                assert ok_l.all() and ok_c.all(), (i, t)
                big = np.abs(o["trace_lout"][t]) >= 1e-3 * lmin
                if big.any():
                    worst = max(worst, float(np.max(np.abs(g["trace_lout"][t][big] - o["trace_lout"][t][big])
                                                    / np.abs(o["trace_lout"][t][big]))))
                compared += 1
    finally:
        B.bpsf_free_code(handle)
    print(f"  compared {compared} iterations ({fails} failing shots); worst relative marginal error {worst:.2e}")
    assert compared > 0 and fails > 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_traces_exact_in_same_precision(prec):
    from oracle.oracle import OracleLib
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs("bb144", 0.06, 60, tag=13)
    O = OracleLib()
    prm = U.oracle_params(k=0, max_iter=40, alpha=0.0)
    handle = B.bpsf_load_code(code.hx)
    try:
        bp = B.make_params(max_iter=40, k=0, alpha=0.0,
                           precision=B.PREC_FP64 if prec == "f64" else B.PREC_FP32)
        for i in range(len(syn)):
            o = O.bp(code.hx, syn[i], 0.06, prm, max_iter=40, prec=prec, trace=True)
            g = B.bpsf_bp_trace(handle, syn[i], np.full(code.n, 0.06), bp)
            assert g["iterations"] == o["iterations"] and g["converged"] == o["converged"]
            assert np.array_equal(g["hard"], o["hard"])
            assert np.array_equal(g["trace_lout"], o["trace_lout"])
            assert np.array_equal(g["trace_c2v"], o["trace_c2v"])
    finally:
        B.bpsf_free_code(handle)
