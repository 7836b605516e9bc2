"""Every decoder option against the float oracle, exact on every shot."""
import numpy as np
import pytest

from tests import gpu_util as U

pytestmark = pytest.mark.gpu

CASES = {
    "weight_le_1": dict(k=8, cand_mode=1, w_max=1),
    "weight_le_3": dict(k=8, cand_mode=1, w_max=3),
    "first_success": dict(k=6, select_mode=1),
    "adaptive_alpha": dict(k=6, alpha=0.0),
    "no_early_stop": dict(k=4, max_iter=25, flags=1),
    "force_pp": dict(k=4, max_iter=30, cand_max_iter=10, flags=2),
    "plain_bp": dict(k=0),
    "one_iteration": dict(k=4, max_iter=1, cand_max_iter=1),
    "k10_all_subsets": dict(k=10, max_iter=40, cand_max_iter=10),
    "k16_weight_le_2": dict(k=16, cand_mode=1, w_max=2, max_iter=40),
    "long_trials": dict(k=3, cand_max_iter=300, max_iter=60),
}


@pytest.mark.parametrize("name", list(CASES))
def test_mode_exact(name):
    kw = CASES[name]
    code_name, p, n = ("bb72", 0.09, 800) if kw.get("k", 6) >= 10 else ("bb144", 0.06, 1500)
    print(f"case {name} {code_name} p={p} n={n} {kw}", flush=True)
    code, _, syn = U.inputs(code_name, p, n, tag=3)
    prm = U.oracle_params(**kw)
    o = U.oracle_decode(code.hx, syn, p, prm, precision="f32")
    g = U.gpu_decode(code.hx, syn, p, prm, precision="f32")
    bad = U.mismatches(g, o)
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]}"
    assert g["stats"]["errors"] == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_nonuniform_priors(prec):
    code, _, syn = U.inputs("bb144", 0.05, 1500, tag=4)
    rng = np.random.default_rng(3)
    pri = rng.uniform(0.01, 0.1, code.n)
    prm = U.oracle_params(k=6)
    o = U.oracle_decode(code.hx, syn, pri, prm, precision=prec)
    g = U.gpu_decode(code.hx, syn, pri, prm, precision=prec)
    assert len(U.mismatches(g, o)) == 0


def test_priors_above_half():
    """p > 1/2 gives negative channel LLRs (legitimate); results still match."""
    code, _, syn = U.inputs("bb72", 0.05, 600, tag=5)
    pri = np.full(code.n, 0.05)
    pri[::7] = 0.6
    prm = U.oracle_params(k=4)
    o = U.oracle_decode(code.hx, syn, pri, prm, precision="f32")
    g = U.gpu_decode(code.hx, syn, pri, prm, precision="f32")
    assert len(U.mismatches(g, o)) == 0
