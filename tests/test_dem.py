"""The circuit-level detector error model (workloads.circuit) against an
independent state-vector simulation of the same noisy circuit, and its
structure on the [[144,12,12]] code (Section V: about 8,000 mechanisms for
d = 12 rounds)."""
import numpy as np
import pytest

from workloads import circuit, codes, gf2, shots


# ------------------------------------------------- state-vector simulation --

class StateVector:
    """Pure state of n qubits as a (2,)*n complex array; qubit q is axis q."""

    def __init__(self, n, rng):
        self.n = n
        self.s = np.zeros((2,) * n, complex)
        self.s[(0,) * n] = 1.0
        self.rng = rng

    def _sl(self, q, v):
        idx = [slice(None)] * self.n
        idx[q] = v
        return tuple(idx)

    def x(self, q):
        self.s = np.flip(self.s, axis=q).copy()

    def z(self, q):
        self.s[self._sl(q, 1)] *= -1.0

    def h(self, q):
        a, b = self.s[self._sl(q, 0)].copy(), self.s[self._sl(q, 1)].copy()
        self.s[self._sl(q, 0)] = (a + b) / np.sqrt(2.0)
        self.s[self._sl(q, 1)] = (a - b) / np.sqrt(2.0)

    def cx(self, c, t):
        sub = self.s[self._sl(c, 1)]
        self.s[self._sl(c, 1)] = np.flip(sub, axis=t if t < c else t - 1).copy()

    def mz(self, q):
        p1 = float(np.sum(np.abs(self.s[self._sl(q, 1)]) ** 2))
        if p1 < 1e-12:
            m = 0
        elif p1 > 1 - 1e-12:
            m = 1
        else:
            m = int(self.rng.random() < p1)
        self.s[self._sl(q, 1 - m)] = 0.0
        self.s /= np.sqrt(np.sum(np.abs(self.s) ** 2))
        return m

    def pauli(self, q, x, z):
        if z:
            self.z(q)
        if x:
            self.x(q)


def simulate(circ, fault=None, seed=0):
    """Measurement records of one run of the circuit, with an optional fault
    (op index, when, [(qubit, x, z)]) applied."""
    nq = circ.n_data + circ.n_x + circ.n_z
    sv = StateVector(nq, np.random.default_rng(seed))
    rec = np.zeros(circ.n_rec, np.uint8)

    def apply_fault(i, when):
        if fault is not None and fault[0] == i and fault[1] == when:
            for q, x, z in fault[2]:
                sv.pauli(q, x, z)

    for i, op in enumerate(circ.ops):
        apply_fault(i, 0)
        if op.kind in ("R0", "RX"):
            for q in op.a:
                if sv.mz(int(q)):
                    sv.x(int(q))
                if op.kind == "RX":
                    sv.h(int(q))
        elif op.kind == "CX":
            for c, t in zip(op.a, op.b):
                sv.cx(int(c), int(t))
        elif op.kind == "MZ":
            for q, r in zip(op.a, op.rec):
                rec[r] = sv.mz(int(q))
        elif op.kind == "MX":
            for q, r in zip(op.a, op.rec):
                sv.h(int(q))
                rec[r] = sv.mz(int(q))
                sv.h(int(q))
        apply_fault(i, 1)
    return rec


def detectors_from_records(circ, rec, hz, lz):
    det = []
    for r in range(circ.rounds):
        cur = rec[circ.zrec[r]]
        det.append(cur ^ rec[circ.zrec[r - 1]] if r > 0 else cur)
    last = rec[circ.zrec[circ.rounds - 1]].copy()
    for c in range(hz.shape[0]):
        last[c] ^= np.bitwise_xor.reduce(rec[circ.drec[np.nonzero(hz[c])[0]]])
    det.append(last)
    obs = np.array([np.bitwise_xor.reduce(rec[circ.drec[np.nonzero(l)[0]]]) for l in lz], np.uint8)
    return np.concatenate(det), obs


STEANE = np.array([[0, 0, 0, 1, 1, 1, 1], [0, 1, 1, 0, 0, 1, 1], [1, 0, 1, 0, 1, 0, 1]], np.uint8)
CODE422 = np.array([[1, 1, 1, 1]], np.uint8)


@pytest.mark.parametrize("name,hx,hz,rounds", [("422", CODE422, CODE422, 2), ("steane", STEANE, STEANE, 2)])
def test_fault_propagation_matches_state_vector(name, hx, hz, rounds):
    circ = circuit.memory_circuit(hx, hz, rounds)
    faults = circuit._faults(circ, 0.01, p_idle=0.01)
    recs = circuit._propagate(circ, faults)
    lz = gf2.logical_basis(hz, hx)
    det, obs = circuit.detectors_and_observables(circ, recs, hz, lz)
    d = circuit._unpack_rows(det, len(faults))
    o = circuit._unpack_rows(obs, len(faults))
    # noiseless: every detector and observable is 0, whatever the random outcomes
    for seed in range(3):
        d0, o0 = detectors_from_records(circ, simulate(circ, None, seed), hz, lz)
        assert not d0.any() and not o0.any()
    step = 1 if len(faults) < 400 else 3
    checked = 0
    for f in range(0, len(faults), step):
        df, of = detectors_from_records(circ, simulate(circ, faults[f][:3], seed=f), hz, lz)
        assert np.array_equal(df, d[f]), (name, f, faults[f])
        assert np.array_equal(of, o[f]), (name, f, faults[f])
        checked += 1
    assert checked > 50


def test_merge_probability_is_odd_count_probability():
    # three faults with one signature: brute force over the 8 outcomes
    ps = [0.01, 0.03, 0.2]
    odd = sum(np.prod([p if (m >> i) & 1 else 1 - p for i, p in enumerate(ps)])
              for m in range(8) if bin(m).count("1") % 2 == 1)
    assert abs((1 - np.prod([1 - 2 * p for p in ps])) / 2 - odd) < 1e-15


@pytest.fixture(scope="module")
def dem144():
    c = codes.get_code("bb144")
    return c, circuit.build_dem(c.hx, c.hz, 12, 0.003)


def test_bb144_dem_shape(dem144):
    """d = 12 rounds: 72 x 13 detectors; the mechanism count is near the
    paper's 'approximately 8,000' for this code (another circuit schedule
    than the paper's, so not equal)."""
    c, dem = dem144
    assert dem.h.shape[0] == 72 * 13
    assert 7000 <= dem.h.shape[1] <= 10000
    assert dem.obs.shape[0] == 12
    # columns are distinct (mechanisms merged), every column flips a detector
    cols = np.packbits(np.vstack([dem.h, dem.obs]), axis=0).T
    assert len(np.unique(cols, axis=0)) == dem.h.shape[1]
    assert dem.h.any(axis=0).all()
    assert (dem.priors > 0).all() and (dem.priors < 0.5).all()


def test_bb144_dem_single_data_errors(dem144):
    """An X error on data qubit q between the Z-check CNOTs of rounds r and
    r+1 flips every later result of the Z checks of q: it shows in detector
    round r+1 only (later rounds compare two flipped results). After the last
    round, the final detector layer (results against the data) shows it.
    Such a mechanism (the three checks of q in one detector round) is a
    column of the DEM."""
    c, dem = dem144
    m = c.hz.shape[0]
    cols = {tuple(np.nonzero(dem.h[:, j])[0]) for j in range(dem.h.shape[1])}
    for q in (0, 17, 100):
        zc = np.nonzero(c.hz[:, q])[0]
        assert len(zc) == 3
        for r in (0, 5, 10, 11):
            assert tuple((r + 1) * m + zc) in cols, (q, r)


def test_bb144_measurement_error_column(dem144):
    """A flipped Z-check result in round r (r < 11) flips that check's
    detectors in rounds r and r+1 only."""
    c, dem = dem144
    m = c.hz.shape[0]
    cols = {tuple(np.nonzero(dem.h[:, j])[0]) for j in range(dem.h.shape[1])}
    for ch in (0, 33, 71):
        for r in (0, 6, 10):
            assert (r * m + ch, (r + 1) * m + ch) in cols


def test_dem_sampling_is_consistent(dem144):
    c, dem = dem144
    e, s, o = circuit.sample(dem, 300, shots.stream_key(shots.MASTER_SEED, 1200))
    assert np.array_equal(s, ((e.astype(np.int64) @ dem.h.T.astype(np.int64)) & 1).astype(np.uint8))
    assert np.array_equal(o, ((e.astype(np.int64) @ dem.obs.T.astype(np.int64)) & 1).astype(np.uint8))
    # mean number of fired mechanisms is the sum of the priors
    assert abs(e.sum(axis=1).mean() - dem.priors.sum()) < 5 * np.sqrt(dem.priors.sum() / 300)
