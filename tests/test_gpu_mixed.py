"""Shots of several codes decoded in one call (bpsf_mix_*): every shot's result
equals the single-code call's and the oracle's, per-code work counters add
up to the single-code calls', and rows, padding and bad code indices are
handled as the header states."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu

NAMES = ["bb72", "bb90", "bb108", "bb144", "bb288"]


def _mix_decode(hs, shot_code, syn, priors, prm, precision="f32", corr_stride=None):
    import torch
    from paper_2507_00254_amd import bpsf as B
    handles = [B.bpsf_load_code(h) for h in hs]
    mix = B.bpsf_mix_create(handles)
    try:
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, prm.cand_mode, prm.w_max, prm.select_mode,
                           prm.alpha, prm.flags, B.PREC_FP64 if precision == "f64" else B.PREC_FP32)
        n = len(shot_code)
        width = corr_stride or max(h.shape[1] for h in hs)
        sc = torch.from_numpy(np.ascontiguousarray(shot_code, dtype=np.int32)).cuda()
        s = torch.from_numpy(np.ascontiguousarray(syn, dtype=np.uint8)).cuda()
        corr = torch.full((n, width), 7, dtype=torch.uint8, device="cuda")
        conv = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        B.bpsf_mix_decode(mix, sc, s, priors, bp, corr, conv, it)
        torch.cuda.synchronize()
        st, bad = B.bpsf_mix_last_stats(mix, len(hs))
        return {"correction": corr.cpu().numpy(), "converged": conv.cpu().numpy(),
                "iterations": it.cpu().numpy(), "stats": st, "bad": bad}
    finally:
        B.bpsf_mix_free(mix)
        for h in handles:
            B.bpsf_free_code(h)


def _per_code(out, shot_code, c, n_bits):
    sel = np.nonzero(shot_code == c)[0]
    return {"correction": out["correction"][sel, :n_bits], "converged": out["converged"][sel],
            "iterations": out["iterations"][sel]}, sel


# 2500 shots run the small family's tiles, 5000 the large families'
@pytest.mark.parametrize("precision,per", [("f32", 500), ("f64", 500), ("f32", 1000)])
def test_mixed_five_codes_match_single_calls_and_oracle(precision, per):
    p = 0.05
    hs = [codes.get_code(n).hx for n in NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, per, shots.stream_key(shots.MASTER_SEED, 900))
    prm = U.oracle_params(k=6)
    print(f"mixed {precision} {len(sc)} shots", flush=True)
    out = _mix_decode(hs, sc, syn, [np.full(h.shape[1], p) for h in hs], prm, precision)
    assert out["bad"] == 0
    for c, h in enumerate(hs):
        g, sel = _per_code(out, sc, c, h.shape[1])
        s_c = syn[sel, :h.shape[0]]
        one = U.gpu_decode(h, s_c, p, prm, precision=precision)
        assert len(U.mismatches(g, one)) == 0, NAMES[c]
        o = U.oracle_decode(h, s_c, p, prm, precision=precision)
        assert len(U.mismatches(g, o)) == 0, NAMES[c]
        # padding after the code's N bits is left alone
        assert (out["correction"][sel, h.shape[1]:] == 7).all()
        st = out["stats"][c]
        for f in ("main_iterations", "trial_iterations", "failed_shots", "converged_trials"):
            assert st[f] == one["stats"][f], (NAMES[c], f)
        # the winners of the kept records are copied, the others decoded again
        # (which records a code's failed shots get depends on the order the
        # waves reach them): at most every winner's trial iterations
        won = o["winner"] >= 0
        assert 0 <= st["rerun_iterations"] <= int((o["iterations"] - o["main_iterations"])[won].sum()), NAMES[c]
        assert one["stats"]["rerun_iterations"] == 0
        assert st["errors"] == 0


def test_mixed_kept_corrections_run_out():
    """More failed shots than the kept records of a mixed call hold: the
    winners of the first records are copied, the rest decoded again, and
    every shot equals the single-code call's (which keeps all of its
    records)."""
    p = 0.08
    hs = [codes.get_code(n).hx for n in NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, 3000, shots.stream_key(shots.MASTER_SEED, 905))
    prm = U.oracle_params(k=8)          # 256 trials: a few thousand records fill the kept region
    print(f"mixed f32 {len(sc)} shots", flush=True)
    out = _mix_decode(hs, sc, syn, [np.full(h.shape[1], p) for h in hs], prm)
    assert out["bad"] == 0
    failed = rerun = 0
    for c, h in enumerate(hs):
        g, sel = _per_code(out, sc, c, h.shape[1])
        one = U.gpu_decode(h, syn[sel, :h.shape[0]], p, prm)
        assert len(U.mismatches(g, one)) == 0, NAMES[c]
        st = out["stats"][c]
        for f in ("main_iterations", "trial_iterations", "failed_shots", "converged_trials", "errors"):
            assert st[f] == one["stats"][f], (NAMES[c], f)
        assert one["stats"]["rerun_iterations"] == 0
        failed += st["failed_shots"]
        rerun += st["rerun_iterations"]
    print(f"failed shots {failed}, re-run iterations {rerun}", flush=True)
    assert rerun > 0


def test_mixed_call_above_the_small_form():
    """A mixed call of more than 65536 shots runs the large form of the mixed
    kernel (every chunk from the counters, no kept corrections): every shot
    equals the single-code call's, the work counters too, and every winner is
    decoded again."""
    p = 0.03
    hs = [codes.get_code(n).hx for n in NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, 14000, shots.stream_key(shots.MASTER_SEED, 906))
    assert len(sc) > 65536
    prm = U.oracle_params(k=6)
    print(f"mixed f32 {len(sc)} shots", flush=True)
    out = _mix_decode(hs, sc, syn, [np.full(h.shape[1], p) for h in hs], prm)
    assert out["bad"] == 0
    for c, h in enumerate(hs):
        g, sel = _per_code(out, sc, c, h.shape[1])
        one = U.gpu_decode(h, syn[sel, :h.shape[0]], p, prm)
        assert len(U.mismatches(g, one)) == 0, NAMES[c]
        st = out["stats"][c]
        for f in ("main_iterations", "trial_iterations", "failed_shots", "converged_trials", "errors"):
            assert st[f] == one["stats"][f], (NAMES[c], f)
        assert st["failed_shots"] > 0 and st["rerun_iterations"] > 0 and one["stats"]["rerun_iterations"] == 0


def test_mixed_first_success_with_pruning():
    """First success with pruning in one mixed call (trial tasks of every
    code taken trial index first): every shot equals the oracle's, which
    keeps the lowest successful trial; pruning runs fewer trial iterations
    than the unpruned mixed call."""
    p = 0.06
    hs = [codes.get_code(n).hx for n in NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, 600, shots.stream_key(shots.MASTER_SEED, 903))
    pri = [np.full(h.shape[1], p) for h in hs]
    full = _mix_decode(hs, sc, syn, pri, U.oracle_params(k=6, select_mode=1))
    pruned = _mix_decode(hs, sc, syn, pri, U.oracle_params(k=6, select_mode=1, flags=4))
    assert full["bad"] == 0 and pruned["bad"] == 0
    saved = 0
    for c, h in enumerate(hs):
        g, sel = _per_code(pruned, sc, c, h.shape[1])
        o = U.oracle_decode(h, syn[sel, :h.shape[0]], p, U.oracle_params(k=6, select_mode=1), precision="f32")
        assert len(U.mismatches(g, o)) == 0, NAMES[c]
        f, _ = _per_code(full, sc, c, h.shape[1])
        assert len(U.mismatches(g, f)) == 0, NAMES[c]
        sp, sf = pruned["stats"][c], full["stats"][c]
        assert sp["failed_shots"] == sf["failed_shots"] > 0 and sp["errors"] == 0
        assert sp["trial_iterations"] <= sf["trial_iterations"]
        saved += sf["trial_iterations"] - sp["trial_iterations"]
    print(f"trial iterations saved by pruning: {saved}", flush=True)
    assert saved > 0


def test_mixed_missing_code_and_bad_indices():
    p = 0.06
    hs = [codes.get_code(n).hx for n in ("bb72", "bb144", "bb288")]
    sc, syn, _, _ = shots.mixed_batch(hs, p, 300, shots.stream_key(shots.MASTER_SEED, 901))
    sc = sc.copy()
    sc[sc == 1] = 0                      # no bb144 shot at all
    bad_at = np.array([3, 50, 777])
    sc[bad_at] = [-1, 3, 1 << 20]        # out of range: skipped
    prm = U.oracle_params(k=6)
    out = _mix_decode(hs, sc, syn, [np.full(h.shape[1], p) for h in hs], prm)
    assert out["bad"] == len(bad_at)
    assert (out["correction"][bad_at] == 7).all() and (out["converged"][bad_at] == 7).all()
    assert (out["iterations"][bad_at] == -1).all()
    assert out["stats"][1]["main_iterations"] == 0 and out["stats"][1]["failed_shots"] == 0
    for c in (0, 2):
        h = hs[c]
        g, sel = _per_code(out, sc, c, h.shape[1])
        o = U.oracle_decode(h, syn[sel, :h.shape[0]], p, prm, precision="f32")
        assert len(U.mismatches(g, o)) == 0


def test_mixed_single_code_and_nonuniform_priors():
    """One code in a mix, then two codes one of whose priors vary per bit (the
    launch then takes the per-bit LLR path for both)."""
    h72, h144 = codes.get_code("bb72").hx, codes.get_code("bb144").hx
    rng = np.random.default_rng(3)
    pri144 = rng.uniform(0.01, 0.08, h144.shape[1])
    sc, syn, _, _ = shots.mixed_batch([h72, h144], 0.05, 400, shots.stream_key(shots.MASTER_SEED, 902))
    prm = U.oracle_params(k=5)
    out = _mix_decode([h72, h144], sc, syn, [np.full(72, 0.05), pri144], prm)
    for c, (h, pri) in enumerate(((h72, 0.05), (h144, pri144))):
        g, sel = _per_code(out, sc, c, h.shape[1])
        o = U.oracle_decode(h, syn[sel, :h.shape[0]], pri, prm, precision="f32")
        assert len(U.mismatches(g, o)) == 0
    only = np.zeros(257, np.int32)
    _, s1 = shots.make_shots(h144, 0.05, 257, shots.stream_key(shots.MASTER_SEED, 903))
    out1 = _mix_decode([h144], only, s1, [np.full(144, 0.05)], prm)
    o1 = U.oracle_decode(h144, s1, 0.05, prm, precision="f32")
    assert len(U.mismatches(out1, o1)) == 0


def test_mixed_rejects_bad_arguments():
    import torch
    from paper_2507_00254_amd import bpsf as B
    h72 = codes.get_code("bb72").hx
    a = B.bpsf_load_code(h72)
    try:
        with pytest.raises(B.BpsfError):
            B.bpsf_mix_create([a, a])                       # repeated handle
        mix = B.bpsf_mix_create([a])
        try:
            bp = B.make_params(100, 20, 4, 0, 1, 0, 0.625, 0, B.PREC_FP32)
            sc = torch.zeros(4, dtype=torch.int32, device="cuda")
            s = torch.zeros((4, 30), dtype=torch.uint8, device="cuda")      # stride < M = 36
            corr = torch.zeros((4, 72), dtype=torch.uint8, device="cuda")
            conv = torch.zeros(4, dtype=torch.uint8, device="cuda")
            it = torch.zeros(4, dtype=torch.int32, device="cuda")
            with pytest.raises(B.BpsfError):
                B.bpsf_mix_decode(mix, sc, s, [np.full(72, 0.05)], bp, corr, conv, it)
        finally:
            B.bpsf_mix_free(mix)
    finally:
        B.bpsf_free_code(a)


def test_grouped_call_matches_listed_call():
    """bpsf_mix_decode_grouped on the shots sorted by code gives each shot the
    result bpsf_mix_decode gives it in interleaved order."""
    import torch
    from paper_2507_00254_amd import bpsf as B
    p = 0.05
    hs = [codes.get_code(n).hx for n in NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, 300, shots.stream_key(shots.MASTER_SEED, 904))
    sc = sc.copy()
    sc[np.isin(np.arange(len(sc)), [5, 6])] = 2     # uneven counts
    prm = U.oracle_params(k=6)
    listed = _mix_decode(hs, sc, syn, [np.full(h.shape[1], p) for h in hs], prm)
    order = np.argsort(sc, kind="stable")
    counts = np.bincount(sc, minlength=len(hs))
    handles = [B.bpsf_load_code(h) for h in hs]
    mix = B.bpsf_mix_create(handles)
    try:
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
        s = torch.from_numpy(np.ascontiguousarray(syn[order])).cuda()
        corr = torch.full((len(sc), 288), 7, dtype=torch.uint8, device="cuda")
        conv = torch.zeros(len(sc), dtype=torch.uint8, device="cuda")
        it = torch.zeros(len(sc), dtype=torch.int32, device="cuda")
        B.bpsf_mix_decode_grouped(mix, counts, s, [np.full(h.shape[1], p) for h in hs], bp, corr, conv, it)
        torch.cuda.synchronize()
        st, _ = B.bpsf_mix_last_stats(mix, len(hs))
        assert np.array_equal(corr.cpu().numpy(), listed["correction"][order])
        assert np.array_equal(conv.cpu().numpy(), listed["converged"][order])
        assert np.array_equal(it.cpu().numpy(), listed["iterations"][order])
        assert st == listed["stats"]
    finally:
        B.bpsf_mix_free(mix)
        for h in handles:
            B.bpsf_free_code(h)


def test_grouped_call_with_one_code_present():
    """A grouped call whose shots are all of one code (the single-code kernels
    run on the mix's scratch) matches the oracle."""
    import torch
    from paper_2507_00254_amd import bpsf as B
    p = 0.06
    hs = [codes.get_code(n).hx for n in NAMES]
    h = hs[4]
    _, syn = shots.make_shots(h, p, 700, shots.stream_key(shots.MASTER_SEED, 905))
    prm = U.oracle_params(k=6)
    handles = [B.bpsf_load_code(x) for x in hs]
    mix = B.bpsf_mix_create(handles)
    try:
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
        pad = np.zeros((700, 144), np.uint8)
        pad[:, :h.shape[0]] = syn
        s = torch.from_numpy(pad).cuda()
        corr = torch.full((700, 288), 7, dtype=torch.uint8, device="cuda")
        conv = torch.zeros(700, dtype=torch.uint8, device="cuda")
        it = torch.zeros(700, dtype=torch.int32, device="cuda")
        B.bpsf_mix_decode_grouped(mix, [0, 0, 0, 0, 700], s, [np.full(x.shape[1], p) for x in hs], bp, corr, conv, it)
        torch.cuda.synchronize()
        st, _ = B.bpsf_mix_last_stats(mix, len(hs))
        got = {"correction": corr.cpu().numpy()[:, :288], "converged": conv.cpu().numpy(), "iterations": it.cpu().numpy()}
        o = U.oracle_decode(h, syn, p, prm, precision="f32")
        assert len(U.mismatches(got, o)) == 0
        assert st[4]["failed_shots"] == int(((o["winner"] >= 0) | (o["converged"] == 0)).sum())
        assert all(st[c]["main_iterations"] == 0 for c in range(4))
    finally:
        B.bpsf_mix_free(mix)
        for x in handles:
            B.bpsf_free_code(x)


def test_reserved_mix_small_calls_keep_corrections():
    """After bpsf_mix_reserve, grouped small calls of growing size (each
    keeping its trials' corrections) give every shot the single-code call's
    result, and no winner is decoded again."""
    import torch
    from paper_2507_00254_amd import bpsf as B
    p = 0.05
    hs = [codes.get_code(n).hx for n in ("bb72", "bb144", "bb288")]
    prm = U.oracle_params(k=6)
    handles = [B.bpsf_load_code(h) for h in hs]
    mix = B.bpsf_mix_create(handles)
    try:
        bp = B.make_params(prm.max_iter, prm.cand_max_iter, prm.k, alpha=prm.alpha, precision=B.PREC_FP32)
        B.bpsf_mix_reserve(mix, 900, bp)
        pri = [np.full(h.shape[1], p) for h in hs]
        for r, per in enumerate((40, 120, 300)):
            sc, syn, _, _ = shots.mixed_batch(hs, p, per, shots.stream_key(shots.MASTER_SEED, 907, r))
            order = np.argsort(sc, kind="stable")
            counts = np.bincount(sc, minlength=len(hs))
            s = torch.from_numpy(np.ascontiguousarray(syn[order])).cuda()
            n = len(sc)
            corr = torch.full((n, 288), 7, dtype=torch.uint8, device="cuda")
            conv = torch.zeros(n, dtype=torch.uint8, device="cuda")
            it = torch.zeros(n, dtype=torch.int32, device="cuda")
            B.bpsf_mix_decode_grouped(mix, counts, s, pri, bp, corr, conv, it)
            torch.cuda.synchronize()
            st, _ = B.bpsf_mix_last_stats(mix, len(hs))
            got = {"correction": corr.cpu().numpy(), "converged": conv.cpu().numpy(), "iterations": it.cpu().numpy()}
            row = 0
            for c, h in enumerate(hs):
                g = {k: v[row:row + counts[c]] for k, v in got.items()}
                g["correction"] = g["correction"][:, :h.shape[1]]
                one = U.gpu_decode(h, syn[order][row:row + counts[c], :h.shape[0]], p, prm)
                assert len(U.mismatches(g, one)) == 0, (per, c)
                assert st[c]["failed_shots"] == one["stats"]["failed_shots"] and st[c]["rerun_iterations"] == 0
                row += counts[c]
    finally:
        B.bpsf_mix_free(mix)
        for h in handles:
            B.bpsf_free_code(h)
