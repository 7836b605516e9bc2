"""The request loop (bpsf_server_*): every request's result equals the same
shots decoded alone, in batched and per-request mode, under a burst and under
an open-loop replay; argument errors are reported."""
import numpy as np
import pytest

from tests import gpu_util as U
from workloads import codes, shots

pytestmark = pytest.mark.gpu

NAMES = ["bb72", "bb90", "bb108", "bb144", "bb288"]
P = 0.05


def _requests(n_req, seed, max_n=256):
    rng = np.random.default_rng(seed)
    hs = [codes.get_code(nm).hx for nm in NAMES]
    code = rng.integers(0, len(hs), n_req)
    size = rng.integers(1, max_n + 1, n_req)
    syns = []
    for i in range(n_req):
        _, s = shots.make_shots(hs[code[i]], P, int(size[i]), shots.stream_key(shots.MASTER_SEED, 950, seed, i))
        syns.append(s)
    return hs, code, syns


def _server(hs, batching=True, lanes=2, cap=4096, budget=0):
    from paper_2507_00254_amd import bpsf as B
    handles = [B.bpsf_load_code(h) for h in hs]
    prm = B.make_params(100, 20, 6, alpha=0.625, precision=B.PREC_FP32)
    srv = B.Server(handles, [np.full(h.shape[1], P) for h in hs], prm, lanes=lanes, max_batch_shots=cap,
                   batching=batching, device_budget_bytes=budget)
    return B, handles, srv


def _close(B, handles, srv):
    srv.close()
    for h in handles:
        B.bpsf_free_code(h)


def _alone(hs, code, syns):
    prm = U.oracle_params(k=6)
    out = []
    for c, s in zip(code, syns):
        g = U.gpu_decode(hs[c], s, P, prm)
        out.append((g["correction"], g["converged"], g["iterations"]))
    return out


def test_burst_results_equal_alone_and_oracle():
    hs, code, syns = _requests(120, 1)
    alone = _alone(hs, code, syns)
    prm = U.oracle_params(k=6)
    for i in range(0, 120, 12):   # the oracle on a sample of requests
        o = U.oracle_decode(hs[code[i]], syns[i], P, prm, precision="f32")
        assert np.array_equal(alone[i][0], o["correction"]) and np.array_equal(alone[i][2], o["iterations"])
    for batching in (True, False):
        B, handles, srv = _server(hs, batching=batching, lanes=2 if batching else 1)
        try:
            reqs = [srv.submit(int(c), s) for c, s in zip(code, syns)]
            for i, (rid, corr, conv, it) in enumerate(reqs):
                lat = srv.wait(rid)
                assert lat >= 0
                assert np.array_equal(corr, alone[i][0]), (batching, i)
                assert np.array_equal(conv, alone[i][1]) and np.array_equal(it, alone[i][2]), (batching, i)
            cnt = srv.counters()
            print(batching, cnt, flush=True)
            assert cnt["requests_done"] == len(reqs)
            if batching:
                assert cnt["batches"] < len(reqs)      # requests were batched together
            else:
                assert cnt["batches"] == len(reqs)
        finally:
            _close(B, handles, srv)


def test_open_loop_replay_and_poll():
    hs, code, syns = _requests(200, 2)
    alone = _alone(hs, code, syns)
    arrival = np.cumsum(np.random.default_rng(5).exponential(2e-4, len(code)))
    B, handles, srv = _server(hs)
    try:
        lat, wall, outs = srv.replay(arrival, code, syns)
        print(f"p50 {np.percentile(lat, 50) * 1e6:.0f} us p99 {np.percentile(lat, 99) * 1e6:.0f} us wall {wall:.3f} s",
              flush=True)
        assert np.all(np.isfinite(lat)) and np.all(lat > 0) and wall >= arrival[-1]
        for i, (corr, conv, it) in enumerate(outs):
            assert np.array_equal(corr, alone[i][0]) and np.array_equal(conv, alone[i][1])
            assert np.array_equal(it, alone[i][2])
        # poll sees submitted requests once they are done
        rid, _, _, _ = srv.submit(int(code[0]), syns[0])
        srv.wait(rid)
        rid2, _, _, _ = srv.submit(int(code[1]), syns[1])
        seen = []
        for _ in range(2000):
            seen += srv.poll()
            if rid2 in seen:
                break
            import time
            time.sleep(1e-3)
        assert rid2 in seen
        srv.wait(rid2)
    finally:
        _close(B, handles, srv)


def test_server_rejects_bad_requests():
    hs, code, syns = _requests(2, 3)
    B, handles, srv = _server(hs, cap=128)
    try:
        with pytest.raises(B.BpsfError):
            srv.submit(7, syns[0])                                   # no such code
        with pytest.raises(B.BpsfError):
            srv.submit(0, np.zeros((129, hs[0].shape[0]), np.uint8))  # above the batch budget
        with pytest.raises(B.BpsfError):
            srv.wait(12345)                                          # unknown id
    finally:
        _close(B, handles, srv)
    with pytest.raises(B.BpsfError):
        _server(hs, batching=False, lanes=2)                         # per-request mode runs one lane


@pytest.mark.parametrize("batching", [True, False])
def test_small_memory_budget_queues_requests(batching):
    """A device budget that holds one request of this size at a time: a burst
    of such requests on two lanes queues for memory (the second lane waits
    until the first batch returns its region), every result still equals the
    shots decoded alone, the pool never holds more than its budget, and a
    request larger than the pool can ever hold is refused at submit."""
    budget = 768 * 1024
    hs = [codes.get_code(nm).hx for nm in NAMES]
    B, handles, srv = _server(hs, batching=batching, lanes=2 if batching else 1, cap=4096, budget=budget)
    try:
        mem = srv.memory()
        print(f"pool {mem}", flush=True)
        assert mem["budget"] == budget and 16 <= mem["max_request"] < 4096
        n = max(1, (mem["max_request"] * 3) // 5)     # two of these never fit the pool together
        rng = np.random.default_rng(9)
        code = rng.integers(0, len(hs), 16)
        syns = [shots.make_shots(hs[c], P, n, shots.stream_key(shots.MASTER_SEED, 951, i))[1]
                for i, c in enumerate(code)]
        alone = _alone(hs, code, syns)
        reqs = [srv.submit(int(c), s) for c, s in zip(code, syns)]
        for i, (rid, corr, conv, it) in enumerate(reqs):
            srv.wait(rid)
            assert np.array_equal(corr, alone[i][0]) and np.array_equal(conv, alone[i][1]), i
            assert np.array_equal(it, alone[i][2]), i
        mem = srv.memory()
        cnt = srv.counters()
        print(f"after: {mem} {cnt}", flush=True)
        assert cnt["requests_done"] == len(reqs) and cnt["batches"] == len(reqs)   # one request per batch
        assert 0 < mem["peak"] <= budget and mem["in_use"] == 0
        if batching:
            assert mem["waited_for_memory"] > 0
        with pytest.raises(B.BpsfError) as ei:
            srv.submit(0, np.zeros((mem["max_request"] + 1, hs[0].shape[0]), np.uint8))
        assert ei.value.code == B.BPSF_EINVAL
    finally:
        _close(B, handles, srv)
