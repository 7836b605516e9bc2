"""Caller trial lists (sampled subsets per weight, shared or per shot) and
pruning under lowest-index selection: exact parity with the oracle, and
pruning changes no result while running fewer trial iterations."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots, trials

pytestmark = pytest.mark.gpu


def _decode_table(h, syn, p, prm, masks, flags=0):
    import torch
    from paper_2507_00254_amd import bpsf as B
    handle = B.bpsf_load_code(h)
    try:
        d_masks = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
        B.bpsf_set_trial_table(handle, d_masks)
        q = U.oracle_params(max_iter=prm.max_iter, cand_max_iter=prm.cand_max_iter, k=prm.k, cand_mode=2,
                            select_mode=prm.select_mode, alpha=prm.alpha, flags=prm.flags | flags)
        return U.gpu_decode(h, syn, p, q, handle=handle)
    finally:
        B.bpsf_free_code(handle)


def test_generated_list_as_table_matches_generated_mode():
    code, _, syn = U.inputs("bb144", 0.05, 2000, tag=70)
    from paper_2507_00254_amd import bpsf as B
    prm = U.oracle_params(k=6)
    ref = U.gpu_decode(code.hx, syn, 0.05, prm)
    tab = B.bpsf_num_trials(B.make_params(k=6))
    got = _decode_table(code.hx, syn, 0.05, prm, tab)
    assert len(U.mismatches(got, ref)) == 0
    # the generated mode leaves out the empty trial of every failed shot (it
    # repeats the failed first BP); the caller's list runs it to its cap
    extra = {"trial_iterations": prm.cand_max_iter * ref["stats"]["failed_shots"]}
    assert ref["stats"]["failed_shots"] > 0
    for f, v in ref["stats"].items():
        assert got["stats"][f] == v + extra.get(f, 0), f


@pytest.mark.parametrize("select", [0, 1])
@pytest.mark.parametrize("per_shot", [False, True])
def test_sampled_lists_match_oracle(select, per_shot):
    name, p, n = "bb144", 0.06, 1500
    code, _, syn = U.inputs(name, p, n, tag=71)
    prm = U.oracle_params(k=8, cand_max_iter=20, select_mode=select)
    key = shots.stream_key(shots.MASTER_SEED, 971)
    masks = trials.sample_trial_table(8, 4, 5, key, n) if per_shot else trials.sample_trial_list(8, 4, 5, key)
    got = _decode_table(code.hx, syn, p, prm, masks)
    from oracle import oracle as O
    o = O.bpsf_batch(code.hx, syn, p, prm, prec="f32", threads=8, masks=masks)
    bad = U.mismatches(got, o)
    print(f"select={select} per_shot={per_shot}: failed {got['stats']['failed_shots']} mismatches {len(bad)}",
          flush=True)
    assert len(bad) == 0


@pytest.mark.parametrize("per_shot", [False, True])
def test_pruning_keeps_results_and_saves_work(per_shot):
    name, p, n = "bb144", 0.07, 2000
    code, _, syn = U.inputs(name, p, n, tag=72)
    prm = U.oracle_params(k=8, select_mode=1)
    key = shots.stream_key(shots.MASTER_SEED, 972)
    masks = trials.sample_trial_table(8, 5, 6, key, n) if per_shot else trials.sample_trial_list(8, 5, 6, key)
    full = _decode_table(code.hx, syn, p, prm, masks)
    pruned = _decode_table(code.hx, syn, p, prm, masks, flags=4)
    assert len(U.mismatches(pruned, full)) == 0
    print(f"trial iterations: {full['stats']['trial_iterations']} -> {pruned['stats']['trial_iterations']}",
          flush=True)
    assert pruned["stats"]["trial_iterations"] < full["stats"]["trial_iterations"]
    from oracle import oracle as O
    o = O.bpsf_batch(code.hx, syn, p, prm, prec="f32", threads=8, masks=masks)
    assert len(U.mismatches(pruned, o)) == 0
    # the oracle stops at the first success in trial order: no parallel run does less
    assert pruned["stats"]["trial_iterations"] >= int(o["trial_iterations"].sum())


def test_prune_needs_first_selection_and_table_needs_a_list():
    from paper_2507_00254_amd import bpsf as B
    h = B.bpsf_load_code(codes.get_code("bb72").hx)
    try:
        code, _, syn = U.inputs("bb72", 0.05, 8, tag=73)
        with pytest.raises(B.BpsfError):
            U.gpu_decode(code.hx, syn, 0.05, U.oracle_params(k=4, select_mode=0, flags=4), handle=h)
        with pytest.raises(B.BpsfError):
            U.gpu_decode(code.hx, syn, 0.05, U.oracle_params(k=4, cand_mode=2), handle=h)
    finally:
        B.bpsf_free_code(h)
