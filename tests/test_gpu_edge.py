"""Edge cases, error paths and determinism of the GPU path."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu


def _run(code, syn, p, **kw):
    prm = U.oracle_params(**kw)
    return U.oracle_decode(code.hx, syn, p, prm, precision="f32"), U.gpu_decode(code.hx, syn, p, prm, precision="f32")


@pytest.mark.parametrize("n", [1, 2, 7, 9, 15, 17, 63, 65])
def test_ragged_shot_counts(n):
    code, _, syn = U.inputs("bb144", 0.06, n, tag=6)
    o, g = _run(code, syn, 0.06, k=6)
    assert len(U.mismatches(g, o)) == 0


def test_zero_shots():
    import torch
    from paper_2507_00254_amd import bpsf as B
    code = codes.bb72()
    h = B.bpsf_load_code(code.hx)
    try:
        e = torch.empty((0, code.hx.shape[0]), dtype=torch.uint8, device="cuda")
        c = torch.empty((0, code.n), dtype=torch.uint8, device="cuda")
        v = torch.empty((0,), dtype=torch.uint8, device="cuda")
        i = torch.empty((0,), dtype=torch.int32, device="cuda")
        B.bpsf_decode(h, e, np.full(code.n, 0.05), B.make_params(), c, v, i)
        torch.cuda.synchronize()
    finally:
        B.bpsf_free_code(h)


def test_zero_syndromes():
    code = codes.bb288()
    syn = np.zeros((300, code.hx.shape[0]), np.uint8)
    o, g = _run(code, syn, 0.03, k=6)
    assert len(U.mismatches(g, o)) == 0
    assert not g["correction"].any() and g["converged"].all() and (g["iterations"] == 1).all()


def test_dense_random_syndromes():
    """Syndromes of no low-weight error: BP mostly fails and every trial runs."""
    code = codes.bb72()
    syn = shots.random_syndromes(code.hx.shape[0], 200, shots.stream_key(9, 9), 0.5)
    o, g = _run(code, syn, 0.05, k=5, max_iter=50)
    assert len(U.mismatches(g, o)) == 0
    assert g["converged"].mean() < 1.0


def test_bad_arguments():
    from paper_2507_00254_amd import bpsf as B
    code = codes.bb72()
    h = B.bpsf_load_code(code.hx)
    try:
        import torch
        s = torch.zeros((4, code.hx.shape[0]), dtype=torch.uint8, device="cuda")
        c = torch.empty((4, code.n), dtype=torch.uint8, device="cuda")
        v = torch.empty((4,), dtype=torch.uint8, device="cuda")
        i = torch.empty((4,), dtype=torch.int32, device="cuda")
        bad_priors = np.full(code.n, 0.05)
        bad_priors[3] = 0.0
        with pytest.raises(B.BpsfError) as ei:
            B.bpsf_decode(h, s, bad_priors, B.make_params(), c, v, i)
        assert ei.value.code == B.BPSF_EINVAL
        bad_priors[3] = np.nan
        with pytest.raises(B.BpsfError):
            B.bpsf_decode(h, s, bad_priors, B.make_params(), c, v, i)
        with pytest.raises(B.BpsfError):
            B.bpsf_decode(h, s, np.full(code.n, 0.05), B.make_params(k=17), c, v, i)
        with pytest.raises(B.BpsfError):
            B.bpsf_decode(h, s, np.full(code.n, 0.05), B.make_params(max_iter=0), c, v, i)
        # a valid call still works afterwards
        B.bpsf_decode(h, s, np.full(code.n, 0.05), B.make_params(), c, v, i)
        torch.cuda.synchronize()
        assert not c.any().item() and v.all().item()
    finally:
        B.bpsf_free_code(h)




def test_deterministic_and_batch_independent():
    """A shot decodes to the same result alone, in a batch, and on repeat."""
    code, _, syn = U.inputs("bb144", 0.07, 1024, tag=7)
    prm = U.oracle_params(k=6)
    full = U.gpu_decode(code.hx, syn, 0.07, prm)
    again = U.gpu_decode(code.hx, syn, 0.07, prm)
    assert len(U.mismatches(full, again)) == 0
    rng = np.random.default_rng(1)
    pick = rng.choice(len(syn), 12, replace=False)
    for i in pick:
        one = U.gpu_decode(code.hx, syn[i:i + 1], 0.07, prm)
        assert np.array_equal(one["correction"][0], full["correction"][i])
        assert one["converged"][0] == full["converged"][i] and one["iterations"][0] == full["iterations"][i]
    # a shuffled batch gives the same per-shot results
    perm = rng.permutation(len(syn))
    sh = U.gpu_decode(code.hx, syn[perm], 0.07, prm)
    assert np.array_equal(sh["correction"], full["correction"][perm])
    assert np.array_equal(sh["iterations"], full["iterations"][perm])


def test_new_priors_wait_for_queued_decodes():
    """Two decodes on one handle and one side stream, enqueued back to back
    with different non-uniform priors: the second call's LLR tables must not
    reach the first call's kernels. Each result equals the oracle's with its
    own priors."""
    import torch
    from paper_2507_00254_amd import bpsf as B
    code, _, syn = U.inputs("bb144", 0.05, 8192, tag=14)
    rng = np.random.default_rng(14)
    pri = [rng.uniform(0.02, 0.07, code.n), rng.uniform(0.03, 0.09, code.n)]
    prm = U.oracle_params(k=6)
    want = [U.oracle_decode(code.hx, syn, x, prm, precision="f32") for x in pri]
    h = B.bpsf_load_code(code.hx)
    try:
        st = torch.cuda.Stream()
        bp = B.make_params(precision=B.PREC_FP32)
        with torch.cuda.stream(st):
            s = torch.from_numpy(syn).cuda()
            outs = [(torch.empty((len(syn), code.n), dtype=torch.uint8, device="cuda"),
                     torch.empty((len(syn),), dtype=torch.uint8, device="cuda"),
                     torch.empty((len(syn),), dtype=torch.int32, device="cuda")) for _ in pri]
        for x, o in zip(pri, outs):
            B.bpsf_decode(h, s, x, bp, *o, stream=st)
        st.synchronize()
        for o, w in zip(outs, want):
            got = {"correction": o[0].cpu().numpy(), "converged": o[1].cpu().numpy(), "iterations": o[2].cpu().numpy()}
            assert len(U.mismatches(got, w)) == 0
        assert (want[0]["correction"] != want[1]["correction"]).any()   # the priors change the result
    finally:
        B.bpsf_free_code(h)
