"""The C ABI on the CPU: the library loads, exports every declared entry
point, and rejects bad input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpsf.h")


@pytest.fixture(scope="module")
def B():
    lib = os.path.join(ROOT, "paper_2507_00254_amd", "libbpsf.so")
    if not os.path.exists(lib):
        from paper_2507_00254_amd import build
        build.build()
    from paper_2507_00254_amd import bpsf
    return bpsf


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bpsf_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("bpsf_load_code", "bpsf_decode", "bpsf_free_code", "bpsf_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(B):
    for name in declared_functions():
        assert hasattr(B.LIB, name), name


def test_params_layout(B):
    assert C.sizeof(B.bpsf_params) == 40
    assert B.bpsf_params.alpha.offset == 24
    assert C.sizeof(B.bpsf_stats) == 48
    assert C.sizeof(B.bpsf_tuning) == 16


def test_trial_enumeration_matches_oracle(B):
    from oracle.oracle import OracleLib, Params
    O = OracleLib()
    for k, mode, w in [(4, 0, 1), (6, 0, 1), (8, 1, 1), (8, 1, 3), (16, 1, 2), (12, 1, 12)]:
        mine = B.bpsf_num_trials(B.make_params(k=k, cand_mode=mode, w_max=w))
        ref = O.trial_masks(Params(k=k, cand_mode=mode, w_max=w))
        assert np.array_equal(mine, ref), (k, mode, w)


@pytest.mark.parametrize("bad", [dict(max_iter=0), dict(max_iter=256), dict(k=17), dict(k=-1),
                                 dict(cand_mode=2), dict(cand_mode=1, w_max=0), dict(cand_mode=1, k=3, w_max=4),
                                 dict(select_mode=5), dict(alpha=-1.0), dict(alpha=float("nan")),
                                 dict(alpha=float("inf")), dict(flags=16), dict(precision=2),
                                 dict(cand_max_iter=0), dict(cand_max_iter=4096)])
def test_parameter_validation(B, bad):
    with pytest.raises(B.BpsfError) as ei:
        B.bpsf_num_trials(B.make_params(**bad))
    assert ei.value.code == B.BPSF_EINVAL
    assert B.LIB.bpsf_last_error().decode()


@pytest.mark.parametrize("case", ["unsorted", "out_of_range", "bad_rowptr", "empty"])
def test_load_code_rejects_malformed(B, case):
    if case == "unsorted":
        h = ([0, 2], [1, 0], 1, 2)
    elif case == "out_of_range":
        h = ([0, 2], [0, 5], 1, 2)
    elif case == "bad_rowptr":
        h = ([1, 2], [0, 1], 1, 2)
    else:
        h = ([0], [], 0, 3)
    with pytest.raises(B.BpsfError) as ei:
        B.bpsf_load_code(h)
    assert ei.value.code == B.BPSF_EINVAL


def test_load_code_refuses_untiled_shapes(B):
    # irregular, and a column of weight 12: no family takes it (checked before any device call)
    h = np.zeros((12, 13), np.uint8)
    h[:, 0] = 1
    for i in range(12):
        h[i, 1 + i] = 1
    with pytest.raises(B.BpsfError) as ei:
        B.bpsf_load_code(h)
    assert ei.value.code == B.BPSF_ENOTSUP
    # a check of weight 1
    h1 = np.zeros((2, 4), np.uint8)
    h1[0, 0] = 1
    h1[1, 1:4] = 1
    with pytest.raises(B.BpsfError) as ei:
        B.bpsf_load_code(h1)
    assert ei.value.code == B.BPSF_ENOTSUP


def test_null_handles(B):
    assert B.LIB.bpsf_decode(None, None, None, 0, None, None, None, None, None) == B.BPSF_EINVAL
    assert B.LIB.bpsf_code_info(None, None, None, None, None, None) == B.BPSF_EINVAL
    B.LIB.bpsf_free_code(None)


# ---- argument checks of the binding (before any library call) --------------

FAKE = 0x1234   # a handle the checks never pass to the library


def _fake_code(B, monkeypatch, m=72, n=144):
    real = B.bpsf_code_info
    monkeypatch.setattr(B, "bpsf_code_info",
                        lambda h: {"M": m, "N": n, "edges": 3 * n, "row_weight": 6, "col_weight": 3}
                        if h == FAKE else real(h))


def _decode_args(shots=4, m=72, n=144, **over):
    import torch
    a = {"syndromes": torch.zeros((shots, m), dtype=torch.uint8),
         "priors": np.full(n, 0.03),
         "corrections": torch.zeros((shots, n), dtype=torch.uint8),
         "converged": torch.zeros((shots,), dtype=torch.uint8),
         "iterations": torch.zeros((shots,), dtype=torch.int32)}
    a.update(over)
    return a


@pytest.mark.parametrize("case,what", [
    ("syn_dtype", "syndromes must be torch.uint8"), ("syn_width", "M = 72"), ("syn_rank", "dimension"),
    ("corr_width", "N = 144"), ("corr_rows", "rows for 4 shots"), ("conv_short", "at least 4"),
    ("iter_dtype", "iterations must be torch.int32"), ("priors_len", "N = 144 probabilities"),
    ("host_tensors", "CUDA"),
])
def test_decode_rejects_bad_tensors(B, monkeypatch, case, what):
    import torch
    _fake_code(B, monkeypatch)
    over = {
        "syn_dtype": {"syndromes": torch.zeros((4, 72), dtype=torch.int32)},
        "syn_width": {"syndromes": torch.zeros((4, 71), dtype=torch.uint8)},
        "syn_rank": {"syndromes": torch.zeros((4 * 72,), dtype=torch.uint8)},
        "corr_width": {"corrections": torch.zeros((4, 72), dtype=torch.uint8)},
        "corr_rows": {"corrections": torch.zeros((3, 144), dtype=torch.uint8)},
        "conv_short": {"converged": torch.zeros((3,), dtype=torch.uint8)},
        "iter_dtype": {"iterations": torch.zeros((4,), dtype=torch.int64)},
        "priors_len": {"priors": np.full(72, 0.03)},
        "host_tensors": {},
    }[case]
    a = _decode_args(**over)
    with pytest.raises(B.BpsfArgumentError, match=what) as ei:
        B.bpsf_decode(FAKE, a["syndromes"], a["priors"], B.make_params(), a["corrections"], a["converged"],
                      a["iterations"])
    assert ei.value.code == B.BPSF_EINVAL and isinstance(ei.value, ValueError)


@pytest.mark.parametrize("case,what", [
    ("code_dtype", "shot_code must be torch.int32"), ("syn_width", "largest M = 72"),
    ("corr_width", "at least 144 bits"), ("n_priors", "one priors array per code"),
    ("priors_len", r"priors\[1\]"), ("iter_short", "at least 4"), ("host_tensors", "CUDA"),
])
def test_mix_decode_rejects_bad_tensors(B, monkeypatch, case, what):
    import torch
    mix = 0x777
    monkeypatch.setitem(B._MIX_SHAPES, mix, [(36, 72), (72, 144)])
    sc = torch.zeros((4,), dtype=torch.int32)
    syn = torch.zeros((4, 72), dtype=torch.uint8)
    pri = [np.full(72, 0.03), np.full(144, 0.03)]
    corr = torch.zeros((4, 144), dtype=torch.uint8)
    conv = torch.zeros((4,), dtype=torch.uint8)
    it = torch.zeros((4,), dtype=torch.int32)
    if case == "code_dtype":
        sc = sc.long()
    elif case == "syn_width":
        syn = torch.zeros((4, 36), dtype=torch.uint8)
    elif case == "corr_width":
        corr = torch.zeros((4, 72), dtype=torch.uint8)
    elif case == "n_priors":
        pri = pri[:1]
    elif case == "priors_len":
        pri = [pri[0], np.full(72, 0.03)]
    elif case == "iter_short":
        it = torch.zeros((3,), dtype=torch.int32)
    with pytest.raises(B.BpsfArgumentError, match=what):
        B.bpsf_mix_decode(mix, sc, syn, pri, B.make_params(), corr, conv, it)
    if case == "iter_short":
        with pytest.raises(B.BpsfArgumentError, match=what):
            B.bpsf_mix_decode_grouped(mix, [2, 2], syn, pri, B.make_params(), corr, conv, it)
    with pytest.raises(B.BpsfArgumentError, match="unknown mix"):
        B.bpsf_mix_decode(0x778, torch.zeros((4,), dtype=torch.int32), syn, pri, B.make_params(), corr, conv, it)


def test_server_checks_request_shapes(B):
    srv = B.Server.__new__(B.Server)        # no library server behind it: only the checks run
    srv._shapes = [(36, 72), (72, 144)]
    assert srv._syndromes(1, np.zeros((3, 72), np.uint8)).shape == (3, 72)
    with pytest.raises(B.BpsfArgumentError, match=r"\[n, 36\]"):
        srv._syndromes(0, np.zeros((3, 72), np.uint8))
    with pytest.raises(B.BpsfArgumentError):
        srv._syndromes(1, np.zeros(72, np.uint8))
