"""GPU path (through the C ABI) against the CPU oracle on identical seeded inputs.

Same-precision runs must agree exactly (corrections, converged flags and
iteration counts): both sides evaluate the same expressions in the same order
without fused multiply-add. Float GPU messages against the double oracle are
held to the decision-level bar (>= 99.99% identical shots) and the LER bar.
"""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import gf2

pytestmark = pytest.mark.gpu


def _report(name, g, o, bad):
    if len(bad):
        i = bad[0]
        print(f"{name}: {len(bad)} mismatching shots; first {i}: gpu conv={g['converged'][i]} it={g['iterations'][i]} "
              f"oracle conv={o['converged'][i]} it={o['iterations'][i]}", flush=True)


@pytest.mark.parametrize("code_name,p,k,n", [
    ("bb144", 0.03, 6, 3000),
    ("bb144", 0.07, 6, 1500),
    ("bb72", 0.05, 4, 3000),
    ("bb72", 0.10, 4, 1500),
    ("bb90", 0.05, 6, 1500),
    ("bb108", 0.05, 6, 1500),
    ("bb288", 0.05, 6, 1000),
])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_exact_parity_same_precision(code_name, p, k, n, prec):
    print(f"case {code_name} p={p} k={k} n={n} {prec}", flush=True)
    code, err, syn = U.inputs(code_name, p, n, tag=1)
    prm = U.oracle_params(k=k)
    o = U.oracle_decode(code.hx, syn, p, prm, precision=prec)
    g = U.gpu_decode(code.hx, syn, p, prm, precision=prec)
    bad = U.mismatches(g, o)
    _report(code_name, g, o, bad)
    assert len(bad) == 0
    # work counters agree with the oracle's iteration counts
    assert g["stats"]["main_iterations"] == int(o["main_iterations"].sum())
    # (the empty trial of every failed shot is not run: cand_max_iter iterations each)
    failed = int(((o["winner"] >= 0) | (o["converged"] == 0)).sum())
    assert g["stats"]["trial_iterations"] == int(o["trial_iterations"].sum()) - prm.cand_max_iter * failed
    assert g["stats"]["errors"] == 0
