"""The benchmark's launch configuration at full size (10^6 shots of
[[144,12,12]] at p = 0.03): sampled shots against the oracle one by one, and
properties that hold for every shot."""
import numpy as np
import pytest

from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def test_bench_configuration_full_size():
    import torch
    from paper_2507_00254_amd import bpsf as B
    code, err, syn = U.inputs("bb144", 0.03, 1_000_000, tag=21)
    prm = U.oracle_params(k=6)
    g = U.gpu_decode(code.hx, syn, 0.03, prm, precision="f32")
    st = g["stats"]
    # every converged output solves its syndrome (checked on the GPU)
    H = torch.from_numpy(code.hx.T.astype(np.float32)).cuda()
    s = torch.from_numpy(syn).cuda()
    ok = torch.ones(len(syn), dtype=torch.bool, device="cuda")
    conv = torch.from_numpy(g["converged"]).cuda().bool()
    for a in range(0, len(syn), 200_000):
        e = torch.from_numpy(g["correction"][a:a + 200_000]).cuda().float()
        sy = (e @ H).remainder(2).to(torch.uint8)
        ok[a:a + 200_000] = (sy == s[a:a + 200_000]).all(dim=1)
    assert bool((ok == conv).all().item()), "converged flag must equal H e == s"
    # sampled shots, every failed-first-BP shot among them included
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(syn), 3000, replace=False))
    hard = np.nonzero(g["iterations"] > 100)[0]
    idx = np.unique(np.concatenate([idx, hard[:500]]))
    o = U.oracle_decode(code.hx, syn[idx], 0.03, prm, precision="f32")
    sub = {k2: v[idx] for k2, v in g.items() if k2 != "stats"}
    assert len(U.mismatches(sub, o)) == 0
    assert st["errors"] == 0 and st["failed_shots"] > 0
    # work counters are consistent with the per-shot outputs
    assert st["main_iterations"] >= len(syn)
