"""The benchmark's workload at full size: the same 10^6 seeded shots of
[[144,12,12]] at p = 0.03 the benchmark decodes, in its launch configuration,
against the oracle on every shot: exactly against the float oracle, >= 99.99%
against the double oracle with the logical error rate inside its interval,
and the kernels' work counters equal to the oracle's iteration sums (the
counts the benchmark's roofline divides by)."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, gf2, shots

pytestmark = pytest.mark.gpu

N_SHOTS = 1_000_000


def test_bench_configuration_full_size():
    import torch
    code = codes.bb144()
    err, syn = shots.headline_shots(code.hx, 0.03, N_SHOTS)
    prm = U.oracle_params(k=6)
    g = U.gpu_decode(code.hx, syn, 0.03, prm, precision="f32")
    st = g["stats"]
    print(f"gpu: {st}", flush=True)
    # every converged output solves its syndrome (checked on the GPU)
    H = torch.from_numpy(code.hx.T.astype(np.float32)).cuda()
    s = torch.from_numpy(syn).cuda()
    ok = torch.ones(len(syn), dtype=torch.bool, device="cuda")
    for a in range(0, len(syn), 200_000):
        e = torch.from_numpy(g["correction"][a:a + 200_000]).cuda().float()
        sy = (e @ H).remainder(2).to(torch.uint8)
        ok[a:a + 200_000] = (sy == s[a:a + 200_000]).all(dim=1)
    conv = torch.from_numpy(g["converged"]).cuda().bool()
    assert bool((ok == conv).all().item()), "converged flag must equal H e == s"
    # every shot against the float oracle, exactly
    o32 = U.oracle_decode(code.hx, syn, 0.03, prm, precision="f32", threads=16)
    bad = U.mismatches(g, o32)
    print(f"float oracle: {len(bad)} mismatches", flush=True)
    assert len(bad) == 0
    # the work counters are the oracle's iteration sums
    won = o32["winner"] >= 0
    assert st["errors"] == 0
    assert st["failed_shots"] == int(((o32["winner"] >= 0) | (o32["converged"] == 0)).sum()) > 0
    assert st["main_iterations"] == int(o32["main_iterations"].sum())
    # the oracle also runs the empty trial of every failed shot (cand_max_iter iterations each)
    assert st["trial_iterations"] == int(o32["trial_iterations"].sum()) - prm.cand_max_iter * st["failed_shots"]
    # every failed shot's trials kept their corrections (25k records x 63
    # trials x 8 lanes x 4 B fit the 256 MiB buffer): the last phase copied
    # the winners' instead of re-running them; the winners' iteration counts
    # are in the per-shot iterations compared above
    assert st["rerun_iterations"] == 0 and int(won.sum()) > 0
    # every shot against the double oracle
    o64 = U.oracle_decode(code.hx, syn, 0.03, prm, precision="f64", threads=16)
    same = (g["correction"] == o64["correction"]).all(axis=1) & (g["converged"] == o64["converged"])
    print(f"double oracle: identical {same.mean():.6f} ({(~same).sum()} differ)", flush=True)
    assert same.mean() >= 0.9999
    lx = gf2.logical_basis(code.hx, code.hz)

    def fails(r):
        resid = (err ^ r["correction"]).astype(np.int64)
        return (r["converged"] == 0) | ((resid @ lx.T.astype(np.int64)) & 1).any(axis=1)

    fo, fg = fails(o64), fails(g)
    lo, hi = U.wilson(int(fo.sum()), len(syn))
    print(f"LER gpu {fg.mean():.4e} oracle {fo.mean():.4e} CI [{lo:.4e}, {hi:.4e}]", flush=True)
    assert lo <= fg.mean() <= hi
