"""The sparse family's LDS layout (host only, no device): the tables
represent the caller's matrix exactly, every check reads each of its cells
once and otherwise only +inf pad cells of its own half-wave, column slots
keep the order the bit phase's sums need, and on the circuit-level matrix of
[[144,12,12]] every half-wave's row reads at every position hit 32 distinct
LDS banks (the layout's purpose; it changes no result)."""
import numpy as np
import pytest

from workloads import circuit, codes

BANKS = 32


@pytest.fixture(scope="module")
def B():
    from paper_2507_00254_amd import bpsf
    return bpsf


@pytest.fixture(scope="module")
def dem144():
    c = codes.bb144()
    return circuit.build_dem(c.hx, c.hz, 12, 0.001).h.astype(np.uint8)


def _random_sparse(seed, m=900, n=6000):
    """An irregular matrix of the sparse family's shape range: columns of
    weight 2..6, rows of weight at least two."""
    rng = np.random.default_rng(seed)
    h = np.zeros((m, n), np.uint8)
    for v in range(n):
        h[rng.choice(m, size=int(rng.integers(2, 7)), replace=False), v] = 1
    return h[h.sum(1) >= 2]


def _column_slots(L):
    start = (L["bits"] & 0xFFFF).astype(np.int64)
    w = (L["bits"] >> 16).astype(np.int64)
    return start, w


def _check_tables(h, L):
    m, n = h.shape
    cells, dv, T, cpt, wmax = L["cells"], L["DVMAX"], L["T"], L["CPT"], L["WMAX"]
    start, w = _column_slots(L)
    cperm, rperm = L["cperm"].astype(np.int64), L["rperm"].astype(np.int64)
    assert sorted(cperm.tolist()) == list(range(n)) and sorted(rperm.tolist()) == list(range(m))
    # internal numbering by weight: the bit phase's waves see near-equal weights
    assert (np.diff(w) >= 0).all() and (np.diff(h.sum(1)[rperm]) >= 0).all()
    assert (w == h.sum(0)[cperm]).all()
    # slots: consecutive, odd lengths (one padding cell after an even column)
    length = np.diff(np.append(start, cells))
    assert start[0] == 0 and ((length == w) | (length == w + 1)).all()
    assert (length % 2 == 1).all()
    # cell -> (internal check); column cells in the caller's check order
    rinv = np.empty(m, np.int64)
    rinv[rperm] = np.arange(m)
    owner = np.full(cells, -1, np.int64)
    for s in range(n):
        rows = np.nonzero(h[:, cperm[s]])[0]            # ascending caller checks
        owner[start[s]:start[s] + w[s]] = rinv[rows]
    # every internal check reads each of its cells exactly once, pads otherwise
    roff, rw = L["roff"].astype(np.int64), L["rw"].astype(np.int64)
    for ri in range(m):
        wave = ri // 64
        rb = rw[wave * 64:min(m, wave * 64 + 64)].max()
        pos = roff[ri, :rb]
        real = pos[pos < cells]
        assert sorted(real.tolist()) == sorted(np.nonzero(owner == ri)[0].tolist()), ri
        pad = pos[pos >= cells] - (cells + dv)
        assert (pad >= 0).all()
        lane, slot = pad // cpt, pad % cpt
        # a pad of a thread of the same half-wave, for the same check slot
        assert ((lane // 32) == (ri % T) // 32).all() and (slot == ri // T).all(), ri
        assert rw[ri] >= h[rperm[ri]].sum() and rw[ri] <= wmax
    # the tables give back H
    h2 = np.zeros_like(h)
    for ri in range(m):
        for cell in roff[ri, :rw[ri]]:
            if cell < cells:
                s = np.searchsorted(start, cell, side="right") - 1
                h2[rperm[ri], cperm[s]] ^= 1
    assert (h2 == h).all()


def _bank_excess(L, m):
    """Extra cycles of the check phase's reads: over every wave, position and
    half-wave, the largest number of distinct addresses in one bank, less one."""
    cells, dv, T, cpt = L["cells"], L["DVMAX"], L["T"], L["CPT"]
    roff, rw = L["roff"].astype(np.int64), L["rw"].astype(np.int64)
    extra = 0
    for w0 in range(0, m, 64):
        rb = rw[w0:min(m, w0 + 64)].max()
        for j in range(rb):
            for h0 in (w0, w0 + 32):
                addr = {int(roff[ri, j]) if ri < m else cells + dv + (ri % T) * cpt + ri // T
                        for ri in range(h0, h0 + 32)}
                extra += np.bincount([a % BANKS for a in addr], minlength=BANKS).max() - 1
    return extra


def test_layout_of_the_circuit_level_matrix(B, dem144):
    L = B.bpsf_sparse_layout(dem144)
    assert L is not None and L["family"] == 0
    _check_tables(dem144, L)
    print({k: L[k] for k in ("cells", "overflow", "extra_positions", "folded")})
    assert L["folded"] == 0
    # the row reads of every half-wave hit distinct banks, except where the
    # last, partly empty half-wave's idle lanes hold banks
    assert _bank_excess(L, dem144.shape[0]) <= 64
    # a few positions more than the waves' largest weights, not many
    assert L["extra_positions"] <= dem144.shape[0] // 32


def test_layout_of_random_irregular_matrices(B):
    for seed in (1, 2):
        h = _random_sparse(seed)
        L = B.bpsf_sparse_layout(h)
        assert L is not None
        _check_tables(h, L)


def test_layout_with_rows_of_the_largest_weight(B):
    """Rows of weight WMAX leave no spare position: where a group's bank
    loads exceed it, cells fold into positions that share a bank (a slower
    read, never a wrong one); the tables stay exact."""
    rng = np.random.default_rng(5)
    m, n = 64, 768
    cols = np.tile(np.arange(n), 5)[:48 * m]
    rng.shuffle(cols)
    h = np.zeros((m, n), np.uint8)
    for r in range(m):
        h[r, np.unique(cols[r * 48:(r + 1) * 48])] = 1
        while h[r].sum() < 48:
            h[r, rng.integers(n)] = 1
    h = h[:, h.sum(0) > 0]
    L = B.bpsf_sparse_layout(h)
    assert L is not None and L["WMAX"] == 48
    assert L["folded"] > 0
    _check_tables(h, L)


def test_layout_is_deterministic(B, dem144):
    a, b = B.bpsf_sparse_layout(dem144), B.bpsf_sparse_layout(dem144)
    for k in ("roff", "rw", "bits", "cperm", "rperm"):
        assert np.array_equal(a[k], b[k])


def test_other_families_have_no_sparse_layout(B):
    assert B.bpsf_sparse_layout(codes.bb144().hx) is None
    with pytest.raises(B.BpsfError):
        B.bpsf_sparse_layout(np.zeros((2, 3), np.uint8))   # checks of weight 0
