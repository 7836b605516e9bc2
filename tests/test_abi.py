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
