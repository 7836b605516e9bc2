"""Checks that pin the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` takes an :class:`oracle.oracle.OracleLib` and raises
``AssertionError`` when the oracle disagrees. They run against the real oracle
(``test_oracle_pins.py``, all must pass) and against copies with planted
mistakes (``test_oracle_mutants.py``, each mutant must fail at least one), so
they are kept small and fast.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

from oracle.oracle import (ALL_SUBSETS, FIRST, FORCE_PP, LAYERED, MIN_WEIGHT, NO_EARLY_STOP, SUM_PRODUCT,
                           WEIGHT_LE, Params)
from workloads import codes, shots

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ------------------------------------------------------------------ helpers --

def random_tree(rng, n_vars: int):
    """Tanner graph that is a tree, every check of degree >= 2: each new check
    hangs off an existing variable and brings 1-3 new variables."""
    edges = []          # (check, var)
    nv, nc = 1, 0
    while nv < n_vars:
        anchor = int(rng.integers(0, nv))
        new = int(min(rng.integers(1, 4), n_vars - nv))
        edges.append((nc, anchor))
        for j in range(new):
            edges.append((nc, nv + j))
        nv += new
        nc += 1
    h = np.zeros((nc, nv), np.uint8)
    for c, v in edges:
        h[c, v] = 1
    return h


def all_vectors(n: int) -> np.ndarray:
    return ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)


def feasible(h, s):
    x = all_vectors(h.shape[1])
    syn = (x.astype(np.int64) @ h.T.astype(np.int64)) & 1
    return x[(syn == s[None, :]).all(axis=1)]


def llr(p):
    return np.log((1.0 - p) / p)


def syndrome(h, e):
    return ((h.astype(np.int64) @ np.asarray(e, np.int64)) & 1).astype(np.uint8)


# --------------------------------------------------------------------- pins --

def pin_tree_min_sum(O):
    """On a cycle-free Tanner graph, min-sum with alpha = 1 run past the graph
    diameter yields the max-marginal LLR: the cheapest solution of He = s with
    e_v = 1 minus the cheapest with e_v = 0, cost = sum of channel LLRs."""
    rng = np.random.default_rng(11)
    for trial in range(6):
        h = random_tree(rng, int(rng.integers(5, 12)))
        m, n = h.shape
        p = rng.uniform(0.02, 0.4, n)
        L = llr(p)
        e = (rng.random(n) < 0.3).astype(np.uint8)
        s = syndrome(h, e)
        sol = feasible(h, s)
        cost = sol @ L
        want = np.array([cost[sol[:, v] == 1].min() - cost[sol[:, v] == 0].min() for v in range(n)])
        r = O.bp(h, s, p, Params(alpha=1.0, flags=NO_EARLY_STOP), max_iter=2 * (m + n))
        assert np.allclose(r["lout"], want, rtol=1e-10, atol=1e-10), (trial, r["lout"], want)


def pin_tree_sum_product(O):
    """On a tree, the sum-product rule (the oracle's tanh mode) gives the exact
    posterior LLR log P(e_v = 0 | s) / P(e_v = 1 | s), found by enumeration.
    This pins the variable-node side shared with min-sum."""
    rng = np.random.default_rng(12)
    for trial in range(5):
        h = random_tree(rng, int(rng.integers(5, 11)))
        m, n = h.shape
        p = rng.uniform(0.05, 0.4, n)
        e = (rng.random(n) < 0.3).astype(np.uint8)
        s = syndrome(h, e)
        sol = feasible(h, s)
        logw = sol @ np.log(p) + (1 - sol) @ np.log(1 - p)
        w = np.exp(logw - logw.max())
        want = np.array([math.log(w[sol[:, v] == 0].sum() / w[sol[:, v] == 1].sum()) for v in range(n)])
        r = O.bp(h, s, p, Params(alpha=1.0, flags=NO_EARLY_STOP, rule=SUM_PRODUCT), max_iter=2 * (m + n))
        assert np.allclose(r["lout"], want, rtol=1e-9, atol=1e-9), (trial, r["lout"], want)


def pin_first_iteration_closed_form(O):
    """Weight-one error on a column-weight-3 code whose columns share at most
    one check: after iteration 1 every message into a variable is +-alpha*L, so
    l_out = L (1 + alpha (3 - 2u)) with u the number of unsatisfied checks of
    the variable (3 at the error, 1 at neighbours, 0 elsewhere); BP stops at
    iteration 1 with the error itself."""
    for code in (codes.bb72(), codes.bb144()):
        h = code.hx
        n = h.shape[1]
        p = 0.05
        L = llr(p)
        for alpha, a_eff in ((0.625, 0.625), (0.0, 0.5)):   # 0.0 selects adaptive 1 - 2^-i
            for v in (0, 17, n // 2 + 5, n - 1):
                e = np.zeros(n, np.uint8)
                e[v] = 1
                s = syndrome(h, e)
                u = (h[s == 1].sum(axis=0)).astype(np.int64)
                want = L * (1.0 + a_eff * (3 - 2 * u))
                r = O.bp(h, s, p, Params(alpha=alpha, flags=NO_EARLY_STOP), max_iter=1)
                assert np.allclose(r["lout"], want, rtol=1e-12, atol=0), (code.name, v, alpha)
                r = O.bp(h, s, p, Params(alpha=alpha), max_iter=50)
                assert r["converged"] == 1 and r["iterations"] == 1, (code.name, v, r["iterations"])
                assert np.array_equal(r["hard"], e)
        if code.name == "bb72":
            # the worked number: p = 0.05, alpha = 0.625 -> -0.875 ln 19 at the flipped bit
            r = O.bp(h, syndrome(h, np.eye(n, dtype=np.uint8)[3]), p, Params(alpha=0.625, flags=NO_EARLY_STOP),
                     max_iter=1)
            assert abs(r["lout"][3] - (-0.875 * math.log(19.0))) < 1e-12


def pin_zero_syndrome(O):
    """s = 0 with p < 1/2: every marginal is L (1 + 3 alpha) > 0, so the zero
    correction is returned after one iteration."""
    for code in (codes.bb72(), codes.bb90()):
        h = code.hx
        m, n = h.shape
        r = O.bpsf_detail(h, np.zeros(m, np.uint8), 0.03, Params())
        assert r["converged"] == 1 and r["iterations"] == 1 and not r["correction"].any()


def pin_half_prior(O):
    """p = 1/2 gives L = 0, every message 0 and l_out = 0, which the hard
    decision rule maps to 1 ("0 if l_out > 0, 1 otherwise"). With even row
    weight the all-ones vector satisfies s = 0, so BP stops at iteration 1."""
    h = codes.bb72().hx
    m, n = h.shape
    r = O.bp(h, np.zeros(m, np.uint8), 0.5, Params(), max_iter=5)
    assert r["converged"] == 1 and r["iterations"] == 1 and r["hard"].all()


def _small_codes():
    hamming = np.array([[1, 0, 1, 0, 1, 0, 1], [0, 1, 1, 0, 0, 1, 1], [0, 0, 0, 1, 1, 1, 1]], np.uint8)
    rng = np.random.default_rng(5)
    rand = np.zeros((5, 10), np.uint8)
    for v in range(10):
        rand[rng.choice(5, size=2, replace=False), v] = 1
    rep = (np.eye(4, 5, dtype=np.uint8) | np.eye(4, 5, k=1, dtype=np.uint8))   # repetition code, a path
    return [hamming, rand, rep]


def pin_ml_identity(O):
    """With Phi = all bits, all 2^N trial vectors, minimum-weight selection and
    post-processing forced, the ML error t* is a trial whose flipped syndrome
    is 0 (converges at once to 0), so the result has the brute-force minimum
    weight of Eq. (MLD_classical), and equals t* when that is unique."""
    rng = np.random.default_rng(7)
    for h in _small_codes():
        m, n = h.shape
        for _ in range(4):
            e = (rng.random(n) < 0.25).astype(np.uint8)
            s = syndrome(h, e)
            sol = feasible(h, s)
            wts = sol.sum(axis=1)
            wmin = wts.min()
            prm = Params(max_iter=8, cand_max_iter=8, k=n, cand_mode=ALL_SUBSETS, select_mode=MIN_WEIGHT,
                         flags=FORCE_PP)
            r = O.bpsf_detail(h, s, 0.1, prm)
            assert r["converged"] == 1
            assert np.array_equal(syndrome(h, r["correction"]), s)
            assert int(r["correction"].sum()) == wmin, (r["correction"].sum(), wmin)
            if (wts == wmin).sum() == 1:
                assert np.array_equal(r["correction"], sol[wts == wmin][0])


def _shots(code, p, n, tag):
    key = shots.stream_key(shots.MASTER_SEED, 900 + tag, code.n, int(p * 10000))
    return shots.make_shots(code.hx, p, n, key)


def pin_converged_invariant(O):
    """Every output flagged converged satisfies H e = s; every other output is
    the first BP's final hard decision."""
    for code, p in ((codes.bb72(), 0.08), (codes.bb144(), 0.06)):
        _, syn = _shots(code, p, 150, 1)
        prm = Params(max_iter=30, cand_max_iter=10, k=4)
        r = O.bpsf_batch(code.hx, syn, p, prm)
        got = (r["correction"].astype(np.int64) @ code.hx.T.astype(np.int64)) & 1
        ok = (got == syn).all(axis=1)
        assert ok[r["converged"] == 1].all()
        assert not ok[r["converged"] == 0].any()
        for i in np.nonzero(r["converged"] == 0)[0][:5]:
            b = O.bp(code.hx, syn[i], p, prm, max_iter=prm.max_iter)
            assert np.array_equal(b["hard"], r["correction"][i])


def pin_flip_counts(O):
    """Oscillation counts equal the number of changes in the recorded per-
    iteration hard decisions (starting from the all-zero vector), and Phi is
    the top-|Phi| of those counts by (count desc, index asc)."""
    code = codes.bb144()
    p = 0.07
    _, syn = _shots(code, p, 80, 2)
    prm = Params(max_iter=40, cand_max_iter=8, k=6)
    seen_fail = 0
    for i in range(len(syn)):
        b = O.bp(code.hx, syn[i], p, prm, max_iter=prm.max_iter, trace=True)
        th = b["trace_hard"].astype(np.int32)
        prev = np.vstack([np.zeros((1, th.shape[1]), np.int32), th[:-1]])
        assert np.array_equal((th != prev).sum(axis=0), b["flips"]), i
        if not b["converged"]:
            seen_fail += 1
            d = O.bpsf_detail(code.hx, syn[i], p, prm)
            assert np.array_equal(d["flips"], b["flips"])
            order = sorted(range(code.n), key=lambda v: (-int(b["flips"][v]), v))
            assert list(d["phi"]) == order[:prm.k], (list(d["phi"]), order[:prm.k])
        if seen_fail >= 4:
            break
    assert seen_fail >= 1


def pin_empty_trial(O):
    """The empty trial vector leaves s unchanged, so with the same damping and
    no more iterations it replays a prefix of the failed first BP and cannot
    converge."""
    code = codes.bb72()
    p = 0.1
    _, syn = _shots(code, p, 200, 3)
    prm = Params(max_iter=30, cand_max_iter=12, k=3)
    fails = 0
    for i in range(len(syn)):
        d = O.bpsf_detail(code.hx, syn[i], p, prm)
        if d["main_converged"]:
            continue
        fails += 1
        assert d["trial_converged"][0] == 0 and d["trial_iterations"][0] == prm.cand_max_iter
        if fails >= 3:
            break
    assert fails >= 1


def pin_trials_independent(O):
    """Algorithm 1 decodes every trial syndrome s' = s + t H^T with its own
    BP(s'): for every trial vector of a failed shot, the trial's recorded
    outcome (converged, iterations, weight of e' + t) equals a separate plain
    BP run on s' from fresh messages, undone by t. A trial that inherited any
    state of the first BP or of the previous trial (messages, the damping
    schedule) would differ from the separate run."""
    cases = ((codes.bb72(), 0.1, Params(max_iter=30, cand_max_iter=12, k=4)),
             (codes.bb144(), 0.07, Params(max_iter=25, cand_max_iter=15, k=5)),
             (codes.bb144(), 0.07, Params(max_iter=25, cand_max_iter=15, k=4, alpha=0.0)))
    for code, p, prm in cases:
        h = code.hx
        _, syn = _shots(code, p, 200, 6)
        masks = O.trial_masks(prm)
        seen = 0
        for i in range(len(syn)):
            d = O.bpsf_detail(h, syn[i], p, prm)
            if d["main_converged"]:
                continue
            phi = [int(v) for v in d["phi"]]
            for ti, mask in enumerate(masks):
                t = np.zeros(code.n, np.uint8)
                for j in range(prm.k):
                    if (int(mask) >> j) & 1:
                        t[phi[j]] = 1
                b = O.bp(h, syn[i] ^ syndrome(h, t), p, prm, max_iter=prm.cand_max_iter)
                assert d["trial_converged"][ti] == b["converged"], (code.name, i, ti)
                assert d["trial_iterations"][ti] == b["iterations"], (code.name, i, ti)
                want_w = int((b["hard"] ^ t).sum()) if b["converged"] else -1
                assert d["trial_weight"][ti] == want_w, (code.name, i, ti)
            seen += 1
            if seen >= 3:
                break
        assert seen >= 1, code.name


def pin_trial_vectors(O):
    """Trial enumeration: all 2^k subsets (bit j <-> Phi[j]), or the
    combinations of weight 1..w_max in order; the iteration budgets printed in
    Section V-A follow from |Phi| trials of weight one."""
    assert list(O.trial_masks(Params(k=4, cand_mode=ALL_SUBSETS))) == list(range(16))
    k, w = 6, 3
    want = [sum(1 << j for j in comb) for r in range(1, w + 1) for comb in itertools.combinations(range(k), r)]
    assert list(O.trial_masks(Params(k=k, cand_mode=WEIGHT_LE, w_max=w))) == want
    with open(os.path.join(GOLDEN, "trial_budgets.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            phi, wmax, per_bp, total = map(int, line.split())
            n = len(O.trial_masks(Params(k=phi, cand_mode=WEIGHT_LE, w_max=wmax)))
            assert per_bp * (n + 1) == total


def pin_trial_results(O):
    """Each successful trial's undone output solves the original syndrome; the
    minimum-weight mode keeps the lightest (lowest index on ties) and the
    first-success mode the lowest successful index."""
    code = codes.bb144()
    p = 0.07
    _, syn = _shots(code, p, 120, 4)
    prm = Params(max_iter=25, cand_max_iter=15, k=5)
    checked = 0
    for i in range(len(syn)):
        d = O.bpsf_detail(code.hx, syn[i], p, prm)
        if d["main_converged"] or not d["trial_converged"].any():
            continue
        ok = np.nonzero(d["trial_converged"])[0]
        wts = d["trial_weight"][ok]
        best = ok[np.argmin(wts)]
        assert d["winner"] == best and d["correction"].sum() == wts.min()
        assert d["iterations"] == d["main_iterations"] + d["trial_iterations"][best]
        f = O.bpsf_detail(code.hx, syn[i], p, Params(max_iter=25, cand_max_iter=15, k=5, select_mode=FIRST))
        assert f["winner"] == ok[0]
        checked += 1
        if checked >= 3:
            break
    assert checked >= 1


def pin_scale_invariance(O):
    """Min-sum is positively homogeneous: priors with doubled LLR give exactly
    doubled messages up to rounding and the same decoding decisions."""
    code = codes.bb144()
    p = 0.03
    p2 = p * p / (p * p + (1 - p) * (1 - p))
    _, syn = _shots(code, p, 60, 5)
    prm = Params(max_iter=40, cand_max_iter=10, k=4)
    a = O.bpsf_batch(code.hx, syn, p, prm)
    b = O.bpsf_batch(code.hx, syn, p2, prm)
    for key in ("correction", "converged", "iterations", "winner"):
        assert np.array_equal(a[key], b[key]), key
    for i in range(5):
        x = O.bp(code.hx, syn[i], p, prm, max_iter=10, trace=True)
        y = O.bp(code.hx, syn[i], p2, prm, max_iter=10, trace=True)
        assert np.allclose(2 * x["trace_lout"], y["trace_lout"], rtol=1e-12, atol=1e-12)


def pin_layered_tree(O):
    """The layered schedule has the same fixed point on a tree: min-sum with
    alpha = 1 run long enough yields the max-marginal LLR."""
    rng = np.random.default_rng(13)
    for trial in range(6):
        h = random_tree(rng, int(rng.integers(5, 12)))
        m, n = h.shape
        p = rng.uniform(0.02, 0.4, n)
        L = llr(p)
        e = (rng.random(n) < 0.3).astype(np.uint8)
        s = syndrome(h, e)
        sol = feasible(h, s)
        cost = sol @ L
        want = np.array([cost[sol[:, v] == 1].min() - cost[sol[:, v] == 0].min() for v in range(n)])
        r = O.bp(h, s, p, Params(alpha=1.0, flags=NO_EARLY_STOP | LAYERED), max_iter=2 * (m + n))
        assert np.allclose(r["lout"], want, rtol=1e-10, atol=1e-10), (trial, r["lout"], want)


def pin_layered_chain(O):
    """A worked sweep. Checks {0,1}, {1,2}, {2,3}: check 2 shares no bit with
    check 0, so the layers are {0, 2} then {1}. With every message positive
    and s = (0, 1, 0), one sweep gives, by hand (a = alpha, L = channel LLRs):
    checks 0 and 2 add a*L1, a*L0 and a*L3, a*L2 to the posteriors of bits
    0, 1 and 2, 3; check 1 then reads bits 1 and 2 at L1 + a*L0 and
    L2 + a*L3 and subtracts a times the other one (its syndrome bit is 1).
    Flooding, index order or any other order give different numbers."""
    h = np.array([[1, 1, 0, 0], [0, 1, 1, 0], [0, 0, 1, 1]], np.uint8)
    p = np.array([0.1, 0.2, 0.25, 0.3])
    L = llr(p)
    a = 0.75
    b1 = L[1] + a * L[0]
    b2 = L[2] + a * L[3]
    want = np.array([L[0] + a * L[1], b1 - a * b2, b2 - a * b1, L[3] + a * L[2]])
    r = O.bp(h, np.array([0, 1, 0], np.uint8), p, Params(alpha=a, flags=NO_EARLY_STOP | LAYERED), max_iter=1)
    assert np.allclose(r["lout"], want, rtol=1e-12, atol=1e-12), (r["lout"], want)


def pin_layered_ml_identity(O):
    """The ML identity of pin_ml_identity holds with the layered schedule."""
    rng = np.random.default_rng(17)
    for h in _small_codes():
        m, n = h.shape
        for _ in range(3):
            e = (rng.random(n) < 0.25).astype(np.uint8)
            s = syndrome(h, e)
            sol = feasible(h, s)
            wmin = sol.sum(axis=1).min()
            prm = Params(max_iter=8, cand_max_iter=8, k=n, cand_mode=ALL_SUBSETS, select_mode=MIN_WEIGHT,
                         flags=FORCE_PP | LAYERED)
            r = O.bpsf_detail(h, s, 0.1, prm)
            assert r["converged"] == 1 and np.array_equal(syndrome(h, r["correction"]), s)
            assert int(r["correction"].sum()) == wmin


def pin_wide_trial_masks(O):
    """64-bit caller lists: a list widened from 32 bits gives the 32-bit
    results; with |Phi| = 40, Phi is the first BP's 40 most-flipped bits by a
    plain sort of its flip counts, and the single-bit trial 1 << 35 is plain
    BP on s + H[:, Phi[35]] with that bit undone."""
    h = codes.get_code("bb72").hx
    _, syn = shots.make_shots(h, 0.08, 200, shots.stream_key(shots.MASTER_SEED, 973))
    prm = Params(k=5, cand_mode=1, w_max=2)
    tab = O.trial_masks(prm)
    ref = O.bpsf_batch(h, syn, 0.08, prm, threads=4, masks=tab)
    got = O.bpsf_batch(h, syn, 0.08, prm, threads=4, masks=tab.astype(np.uint64))
    for f in ("correction", "converged", "iterations", "winner", "main_iterations", "trial_iterations"):
        assert np.array_equal(got[f], ref[f]), f
    big = Params(k=40, cand_max_iter=20)
    res = O.bpsf_batch(h, syn, 0.08, big, threads=4, masks=np.array([1 << 35], np.uint64))
    failed = np.nonzero(res["main_iterations"] == big.max_iter)[0]
    assert len(failed) > 3
    for i in failed[:8]:
        flips = O.bpsf_detail(h, syn[i], 0.08, Params(k=1))["flips"]
        order = sorted(range(len(flips)), key=lambda v: (-int(flips[v]), v))
        assert list(res["phi"][i]) == order[:40]
        v = int(res["phi"][i][35])
        b = O.bp(h, syn[i] ^ h[:, v], 0.08, big, max_iter=big.cand_max_iter)
        want = b["hard"].copy()
        want[v] ^= 1
        if b["converged"]:
            assert res["converged"][i] == 1 and np.array_equal(res["correction"][i], want)
        else:
            assert res["converged"][i] == 0


PINS = [pin_tree_min_sum, pin_tree_sum_product, pin_first_iteration_closed_form, pin_zero_syndrome,
        pin_half_prior, pin_ml_identity, pin_converged_invariant, pin_flip_counts, pin_empty_trial,
        pin_trials_independent,
        pin_trial_vectors, pin_trial_results, pin_scale_invariance, pin_layered_tree, pin_layered_chain,
        pin_layered_ml_identity, pin_wide_trial_masks]
