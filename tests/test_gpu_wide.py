"""Codes too large for one wave, with irregular weights: the phenomenological
space-time matrices (one decode per workgroup of three waves). Exact parity
with the oracle under the workload's parameters and under the options."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots, trials

pytestmark = pytest.mark.gpu


def _phen(base, rounds):
    return codes.phenomenological(codes.get_code(base).hx, rounds)


def _inputs(h, p, n, tag):
    _, syn = shots.make_shots(h, p, n, shots.stream_key(shots.MASTER_SEED, 980 + tag, h.shape[1], int(p * 1e5)))
    return syn


@pytest.mark.parametrize("p,n", [(0.002, 600), (0.005, 600)])
def test_phenomenological_r12_parity(p, n):
    h = _phen("bb144", 12)
    assert h.shape == (864, 2592)
    syn = _inputs(h, p, n, 0)
    prm = U.oracle_params(max_iter=200, cand_max_iter=30, k=8)
    g = U.gpu_decode(h, syn, p, prm)
    o = U.oracle_decode(h, syn, p, prm, precision="f32")
    bad = U.mismatches(g, o)
    print(f"phen R=12 p={p}: failed {g['stats']['failed_shots']} mismatches {len(bad)}", flush=True)
    assert len(bad) == 0
    assert g["stats"]["errors"] == 0
    assert g["stats"]["main_iterations"] == int(o["main_iterations"].sum())


@pytest.mark.parametrize("opts", [dict(k=6), dict(k=6, select_mode=1), dict(k=5, cand_mode=1, w_max=2),
                                  dict(k=4, flags=2), dict(k=0), dict(k=6, alpha=0.0), dict(k=6, flags=1)])
def test_small_phenomenological_options(opts):
    h = _phen("bb72", 4)
    p = 0.01
    syn = _inputs(h, p, 800, 1)
    kw = dict(max_iter=60, cand_max_iter=15)
    kw.update(opts)
    prm = U.oracle_params(**kw)
    g = U.gpu_decode(h, syn, p, prm)
    o = U.oracle_decode(h, syn, p, prm, precision="f32")
    assert len(U.mismatches(g, o)) == 0, opts


def test_nonuniform_priors_and_sampled_pruned_trials():
    h = _phen("bb72", 4)
    rng = np.random.default_rng(9)
    pri = rng.uniform(0.003, 0.02, h.shape[1])
    syn = _inputs(h, 0.012, 700, 2)
    prm = U.oracle_params(max_iter=80, cand_max_iter=20, k=8)
    g = U.gpu_decode(h, syn, pri, prm)
    o = U.oracle_decode(h, syn, pri, prm, precision="f32")
    assert len(U.mismatches(g, o)) == 0
    from tests.test_gpu_trials import _decode_table
    from oracle import oracle as O
    masks = trials.sample_trial_table(8, 4, 5, shots.stream_key(shots.MASTER_SEED, 985), len(syn))
    prm1 = U.oracle_params(max_iter=80, cand_max_iter=20, k=8, select_mode=1)
    full = _decode_table(h, syn, 0.012, prm1, masks)
    pruned = _decode_table(h, syn, 0.012, prm1, masks, flags=4)
    o1 = O.bpsf_batch(h, syn, 0.012, prm1, prec="f32", threads=8, masks=masks)
    assert len(U.mismatches(full, o1)) == 0 and len(U.mismatches(pruned, o1)) == 0
    assert pruned["stats"]["trial_iterations"] <= full["stats"]["trial_iterations"]


def test_double_precision_or_refused():
    from paper_2507_00254_amd import bpsf as B
    h = _phen("bb72", 4)
    syn = _inputs(h, 0.01, 400, 3)
    prm = U.oracle_params(max_iter=60, cand_max_iter=15, k=6)
    try:
        g = U.gpu_decode(h, syn, 0.01, prm, precision="f64")
    except B.BpsfError as e:
        assert e.code == B.BPSF_ENOTSUP
        pytest.skip("double messages of this wide family exceed the device's LDS per workgroup")
    o = U.oracle_decode(h, syn, 0.01, prm, precision="f64")
    assert len(U.mismatches(g, o)) == 0


def test_wide_codes_do_not_mix_and_have_no_tiles():
    from paper_2507_00254_amd import bpsf as B
    hw = B.bpsf_load_code(_phen("bb72", 4))
    hb = B.bpsf_load_code(codes.get_code("bb72").hx)
    try:
        assert B.bpsf_tile_options(hw) == []
        assert B.bpsf_code_info(hw)["row_weight"] == 8 and B.bpsf_code_info(hw)["col_weight"] == 3
        with pytest.raises(B.BpsfError):
            B.bpsf_mix_create([hb, hw])
    finally:
        B.bpsf_free_code(hw)
        B.bpsf_free_code(hb)


@pytest.mark.parametrize("n", [1, 2, 3, 7])
def test_ragged_calls_alone_equal_the_batch(n):
    """Calls of a few shots (fewer workgroups than the grid holds; the first
    task of a workgroup is its block index) give each shot the result it gets
    in a batch, and the oracle's. Failing shots are included (p = 0.03)."""
    h = _phen("bb72", 4)
    p = 0.03
    syn = _inputs(h, p, 40, 2)
    prm = U.oracle_params(max_iter=60, cand_max_iter=15, k=6)
    full = U.gpu_decode(h, syn, p, prm)
    assert full["stats"]["failed_shots"] > 0
    for i in range(0, 40 - n + 1, 9):
        part = U.gpu_decode(h, syn[i:i + n], p, prm)
        for f in ("correction", "converged", "iterations"):
            assert np.array_equal(part[f], full[f][i:i + n]), (n, i, f)
    o = U.oracle_decode(h, syn, p, prm, precision="f32")
    assert len(U.mismatches(full, o)) == 0
