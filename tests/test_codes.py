"""Code constructions against the paper's printed values (Appendix A)."""
import os

import numpy as np
import pytest

from workloads import codes, gf2, shots

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table():
    rows = []
    with open(os.path.join(GOLDEN, "code_tables.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            fam, l, m, a, b, n, k, d = line.split()
            rows.append((fam, int(l), int(m), a, b, int(n), int(k), int(d)))
    return rows


def test_shift_matrix_worked_example():
    want = np.loadtxt(os.path.join(GOLDEN, "shift_matrix_s3.txt"), dtype=np.uint8)
    assert np.array_equal(codes.shift_matrix(3), want)


@pytest.mark.parametrize("row", _table(), ids=lambda r: f"{r[0]}{r[5]}")
def test_code_table(row):
    fam, l, m, a, b, n, k, d = row
    if fam == "bb":
        at = [tuple(map(int, t.split(","))) for t in a.split("+")]
        bt = [tuple(map(int, t.split(","))) for t in b.split("+")]
        c = codes.bb_code(l, m, at, bt)
    elif fam == "cbb":
        c = codes.coprime_bb_code(l, m, [int(t) for t in a.split("+")], [int(t) for t in b.split("+")])
    else:
        c = codes.gb_code(l, [int(t) for t in a.split("+")], [int(t) for t in b.split("+")])
    assert c.n == n
    # CSS condition H_X H_Z^T = 0 (Section II-A) and the printed number of logical qubits.
    assert not ((c.hx.astype(np.int64) @ c.hz.T.astype(np.int64)) & 1).any()
    assert gf2.code_dimension(c.hx, c.hz) == k


@pytest.mark.parametrize("name,k", [("bb90", 8), ("bb108", 8)])
def test_extra_bb_codes(name, k):
    c = codes.get_code(name)
    assert gf2.code_dimension(c.hx, c.hz) == k
    assert set(c.hx.sum(axis=1)) == {6} and set(c.hx.sum(axis=0)) == {3}


def test_bb_columns_share_at_most_one_check():
    for name in ("bb72", "bb90", "bb108", "bb144", "bb288"):
        h = codes.get_code(name).hx.astype(np.int64)
        ov = h.T @ h
        np.fill_diagonal(ov, 0)
        assert ov.max() <= 1, name


def test_phenomenological_shape():
    h = codes.phenomenological(codes.bb144().hx, 12)
    assert h.shape == (864, 2592)
    assert int(h.sum()) == 6840
    rw = h.sum(axis=1)
    assert set(rw[:72]) == {7} and set(rw[72:]) == {8}
    cw = h.sum(axis=0)
    assert set(cw[:1728]) == {3} and set(cw[1728:2592 - 72]) == {2} and set(cw[2592 - 72:]) == {1}


def test_csr_roundtrip():
    h = codes.bb144().hx
    rp, ci = codes.csr(h)
    back = np.zeros_like(h)
    for r in range(h.shape[0]):
        back[r, ci[rp[r]:rp[r + 1]]] = 1
        assert np.all(np.diff(ci[rp[r]:rp[r + 1]]) > 0)
    assert np.array_equal(back, h)


def test_shots_are_partition_invariant():
    h = codes.bb72().hx
    key = shots.stream_key(1, 2, 3)
    e1, s1 = shots.make_shots(h, 0.05, 1000, key)
    e2, s2 = shots.make_shots(h, 0.05, 400, key, shot_start=600)
    assert np.array_equal(e1[600:], e2) and np.array_equal(s1[600:], s2)
    assert np.array_equal(s1, (e1.astype(np.int64) @ h.T.astype(np.int64)) & 1)
    rate = e1.mean()
    assert abs(rate - 0.05) < 0.005


def test_logical_basis_size():
    c = codes.bb144()
    lx = gf2.logical_basis(c.hx, c.hz)
    assert lx.shape == (12, 144)
    assert not ((lx.astype(np.int64) @ c.hz.T.astype(np.int64)) & 1).any()
