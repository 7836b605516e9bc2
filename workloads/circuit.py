"""Circuit-level noise: a syndrome-extraction circuit for a CSS code, the
propagation of every single fault through it, and the detector error model
(DEM) they induce.

Section V decodes, under circuit-level noise, the matrix whose rows are
detectors and whose columns are error mechanisms of a noisy
syndrome-extraction circuit run for d rounds (about 8,000 mechanisms for the
[[144,12,12]] code). This module builds such a matrix without a circuit
simulator library. Input generation only: it holds none of the decoder's
arithmetic.

Circuit (a Z-basis memory experiment, one ancilla per check):
  * data qubits start in |0>;
  * every round prepares the X-check ancillas in |+> and the Z-check
    ancillas in |0>, applies the X-check CNOTs (ancilla controls data), then
    the Z-check CNOTs (data controls ancilla), in layers where every qubit
    takes part in at most one gate (an edge colouring of each check graph
    with as many colours as its largest weight: 6 + 6 layers for the BB
    codes), and measures the X-check ancillas in the X basis and the Z-check
    ancillas in the Z basis;
  * after the last round every data qubit is measured in the Z basis.
Measuring all X checks before all Z checks measures every stabilizer exactly
(the CNOTs of one block commute), whatever the order inside a block.

Noise (uniform circuit noise of strength p on gates and measurements, as
Section V states it): each CNOT is followed by one of the 15 two-qubit
Paulis, each with probability p/15; each preparation is followed by a flip
(X after |0>, Z after |+>) with probability p; each measurement result is
flipped with probability p. Optionally (``p_idle`` > 0), each data qubit idle
during a CNOT layer suffers X, Y or Z, each with probability p_idle/3; the
paper names no idle errors, so the default is 0.

Detectors (rows): the Z-check result of round r XOR that of round r-1 (round
0 alone: the data start in |0>), and the last round's result XOR the parity
of the final data measurements on the check's support. Observables: the
Z-type logical operators read from the final data measurements. Every fault
is a Pauli at a point of the circuit; its image under the remaining gates
flips a set of measurement results, hence a set of detectors and
observables. Faults with the same detectors and observables merge into one
mechanism whose probability is that of an odd number of them occurring,
(1 - prod(1 - 2 p_i)) / 2; faults that flip no detector are dropped (the
circuit's distance keeps them off the observables). Mechanisms are then
treated as independent, as the decoder assumes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from workloads import gf2, shots


# ---------------------------------------------------------------- circuit --

@dataclass
class Op:
    kind: str                  # "R0", "RX", "CX", "MZ", "MX"
    a: np.ndarray              # qubits (R*, M*) or controls (CX)
    b: np.ndarray | None = None  # targets (CX)
    rec: np.ndarray | None = None  # measurement record indices (M*)


def cnot_layers(h: np.ndarray):
    """Edges (check c, bit q) of ``h`` split into the fewest layers in which
    every check and every bit appears at most once: as many layers as the
    largest row or column weight (Koenig's edge-colouring theorem for
    bipartite graphs). Edges are coloured in row order; an edge whose two
    ends have no common free colour a = free at c, b = free at q first swaps
    a and b along the alternating path that starts at q."""
    m, n = h.shape
    ncol = int(max(h.sum(axis=1).max(), h.sum(axis=0).max()))
    # colour -> neighbour at each vertex (checks 0..m-1, bits m..m+n-1), -1 free
    at = np.full((m + n, ncol), -1, np.int64)
    for c in range(m):
        for q in np.nonzero(h[c])[0]:
            u, v = c, m + int(q)
            a = int(np.nonzero(at[u] < 0)[0][0])
            b = int(np.nonzero(at[v] < 0)[0][0])
            if at[v, a] >= 0:
                # path from v alternating colours a, b; swap them along it
                path = [v]
                col = a
                while at[path[-1], col] >= 0:
                    path.append(int(at[path[-1], col]))
                    col = b if col == a else a
                edges = []
                col = a
                for i in range(len(path) - 1):
                    edges.append((path[i], path[i + 1], col))
                    col = b if col == a else a
                for x, y, k in edges:
                    at[x, k] = -1
                    at[y, k] = -1
                for x, y, k in edges:
                    k2 = b if k == a else a
                    at[x, k2] = y
                    at[y, k2] = x
            at[u, a] = v
            at[v, a] = u
    layers = []
    for k in range(ncol):
        layers.append([(c, int(at[c, k]) - m) for c in range(m) if at[c, k] >= 0])
    return layers


@dataclass
class Circuit:
    n_data: int
    n_x: int
    n_z: int
    rounds: int
    ops: list
    n_rec: int
    zrec: np.ndarray     # [rounds, n_z] record index of each Z-check result
    xrec: np.ndarray     # [rounds, n_x]
    drec: np.ndarray     # [n_data] final data records


def memory_circuit(hx: np.ndarray, hz: np.ndarray, rounds: int) -> Circuit:
    """The Z-basis memory circuit described in the module docstring."""
    hx = np.asarray(hx, np.uint8)
    hz = np.asarray(hz, np.uint8)
    n = hx.shape[1]
    mx, mz = hx.shape[0], hz.shape[0]
    xa = n + np.arange(mx)            # X-check ancillas
    za = n + mx + np.arange(mz)       # Z-check ancillas
    xl = cnot_layers(hx)
    zl = cnot_layers(hz)
    ops = [Op("R0", np.arange(n))]
    rec = 0
    zrec = np.zeros((rounds, mz), np.int64)
    xrec = np.zeros((rounds, mx), np.int64)
    for r in range(rounds):
        ops.append(Op("RX", xa.copy()))
        ops.append(Op("R0", za.copy()))
        for layer in xl:
            cs = np.array([c for c, _ in layer])
            qs = np.array([q for _, q in layer])
            ops.append(Op("CX", xa[cs], qs))
        for layer in zl:
            cs = np.array([c for c, _ in layer])
            qs = np.array([q for _, q in layer])
            ops.append(Op("CX", qs, za[cs]))
        xrec[r] = rec + np.arange(mx)
        ops.append(Op("MX", xa.copy(), rec=xrec[r].copy()))
        rec += mx
        zrec[r] = rec + np.arange(mz)
        ops.append(Op("MZ", za.copy(), rec=zrec[r].copy()))
        rec += mz
    drec = rec + np.arange(n)
    ops.append(Op("MZ", np.arange(n), rec=drec.copy()))
    rec += n
    return Circuit(n, mx, mz, rounds, ops, rec, zrec, xrec, drec)


# ------------------------------------------------------------------ faults --

# Pauli as (x, z) bits: I, X, Y, Z
_P1 = [(1, 0), (1, 1), (0, 1)]
_P2 = [(a, b) for a in range(4) for b in range(4) if (a, b) != (0, 0)]
_XZ = [(0, 0), (1, 0), (1, 1), (0, 1)]


def _faults(circ: Circuit, p: float, p_idle: float = 0.0):
    """Every fault location: (op index, when, [(qubit, x, z), ...], prob),
    'when' being 0 for before the op and 1 for after it."""
    out = []
    n = circ.n_data
    data = set(range(n))
    for i, op in enumerate(circ.ops):
        if op.kind == "R0":
            for q in op.a:
                out.append((i, 1, [(int(q), 1, 0)], p))
        elif op.kind == "RX":
            for q in op.a:
                out.append((i, 1, [(int(q), 0, 1)], p))
        elif op.kind in ("MZ", "MX"):
            for q in op.a:
                out.append((i, 0, [(int(q), 1, 0) if op.kind == "MZ" else (int(q), 0, 1)], p))
        elif op.kind == "CX":
            for c, t in zip(op.a, op.b):
                for pa, pb in _P2:
                    xa, za = _XZ[pa]
                    xb, zb = _XZ[pb]
                    out.append((i, 1, [(int(c), xa, za), (int(t), xb, zb)], p / 15.0))
            if p_idle > 0.0:
                busy = set(int(q) for q in op.a) | set(int(q) for q in op.b)
                for q in sorted(data - busy):
                    for x, z in _P1:
                        out.append((i, 1, [(q, x, z)], p_idle / 3.0))
    return out


def _propagate(circ: Circuit, faults):
    """Measurement records flipped by each fault: a bit matrix
    [n_rec, ceil(n_faults / 64)] of uint64 words, bit f of a row set when
    fault f flips that record. All faults travel together as Pauli frames,
    one bit per fault: a CNOT copies the control's X part onto the target and
    the target's Z part onto the control; a preparation clears the qubit's
    frame; a Z (X) measurement reads the frame's X (Z) part."""
    nq = circ.n_data + circ.n_x + circ.n_z
    nf = len(faults)
    nw = (nf + 63) // 64
    fx = np.zeros((nq, nw), np.uint64)
    fz = np.zeros((nq, nw), np.uint64)
    recs = np.zeros((circ.n_rec, nw), np.uint64)
    # faults grouped by (op, when)
    by_loc: dict = {}
    for f, (i, when, paulis, _) in enumerate(faults):
        by_loc.setdefault((i, when), []).append((f, paulis))

    def insert(key):
        for f, paulis in by_loc.get(key, ()):
            w, b = f >> 6, np.uint64(1) << np.uint64(f & 63)
            for q, x, z in paulis:
                if x:
                    fx[q, w] ^= b
                if z:
                    fz[q, w] ^= b

    for i, op in enumerate(circ.ops):
        insert((i, 0))
        if op.kind in ("R0", "RX"):
            fx[op.a] = 0
            fz[op.a] = 0
        elif op.kind == "CX":
            fx[op.b] ^= fx[op.a]
            fz[op.a] ^= fz[op.b]
        elif op.kind == "MZ":
            recs[op.rec] = fx[op.a]
        elif op.kind == "MX":
            recs[op.rec] = fz[op.a]
        insert((i, 1))
    return recs


# --------------------------------------------------------------------- DEM --

@dataclass
class DEM:
    h: np.ndarray        # [n_det, n_mech] uint8
    obs: np.ndarray      # [n_obs, n_mech] uint8
    priors: np.ndarray   # [n_mech] float64
    rounds: int
    p: float


def detectors_and_observables(circ: Circuit, recs: np.ndarray, hz: np.ndarray, lz: np.ndarray):
    """Packed detector and observable rows from packed record rows."""
    rows = []
    for r in range(circ.rounds):
        cur = recs[circ.zrec[r]]
        rows.append(cur ^ recs[circ.zrec[r - 1]] if r > 0 else cur.copy())
    last = recs[circ.zrec[circ.rounds - 1]].copy()
    for c in range(hz.shape[0]):
        for q in np.nonzero(hz[c])[0]:
            last[c] ^= recs[circ.drec[q]]
    rows.append(last)
    det = np.concatenate(rows)
    obs = np.zeros((lz.shape[0], recs.shape[1]), np.uint64)
    for i in range(lz.shape[0]):
        for q in np.nonzero(lz[i])[0]:
            obs[i] ^= recs[circ.drec[q]]
    return det, obs


def _unpack_rows(packed: np.ndarray, nf: int) -> np.ndarray:
    """[rows, words] uint64 -> [nf, rows] uint8 (fault-major)."""
    b = np.unpackbits(packed.view(np.uint8), axis=1, bitorder="little")[:, :nf]
    return np.ascontiguousarray(b.T)


def build_dem(hx: np.ndarray, hz: np.ndarray, rounds: int, p: float, p_idle: float = 0.0) -> DEM:
    """The detector error model of ``memory_circuit(hx, hz, rounds)`` under
    depolarizing circuit noise of strength ``p`` (module docstring).
    Mechanisms are ordered by their lowest detector, then by their detector
    pattern."""
    hx = np.asarray(hx, np.uint8)
    hz = np.asarray(hz, np.uint8)
    circ = memory_circuit(hx, hz, rounds)
    faults = _faults(circ, p, p_idle)
    recs = _propagate(circ, faults)
    lz = gf2.logical_basis(hz, hx)
    det, obs = detectors_and_observables(circ, recs, hz, lz)
    nf = len(faults)
    d = _unpack_rows(det, nf)          # [nf, n_det]
    o = _unpack_rows(obs, nf)          # [nf, n_obs]
    pr = np.array([f[3] for f in faults])
    keep = d.any(axis=1)
    d, o, pr = d[keep], o[keep], pr[keep]
    sig = np.concatenate([np.packbits(d, axis=1), np.packbits(o, axis=1)], axis=1)
    uniq, inv = np.unique(sig, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nm = uniq.shape[0]
    # probability of an odd number of the merged faults
    prod = np.ones(nm)
    np.multiply.at(prod, inv, 1.0 - 2.0 * pr)
    prob = (1.0 - prod) / 2.0
    first = np.zeros(nm, np.int64)
    hd = np.zeros((nm, d.shape[1]), np.uint8)
    hd[inv] = d
    ho = np.zeros((nm, o.shape[1]), np.uint8)
    ho[inv] = o
    first = hd.argmax(axis=1)
    order = np.lexsort((np.arange(nm), first))
    return DEM(np.ascontiguousarray(hd[order].T), np.ascontiguousarray(ho[order].T), prob[order], rounds, p)


def sample(dem: DEM, n_shots: int, key: np.uint64, shot_start: int = 0, chunk: int = 4096):
    """Seeded shots of a DEM: every mechanism fires independently with its
    probability (the counter-based stream of ``workloads.shots``). Returns
    ``(errors [n, n_mech], syndromes [n, n_det], observable flips [n, n_obs])``."""
    nm = dem.h.shape[1]
    errs = np.empty((n_shots, nm), np.uint8)
    syns = np.empty((n_shots, dem.h.shape[0]), np.uint8)
    obs = np.empty((n_shots, dem.obs.shape[0]), np.uint8)
    hs = dem.h.astype(np.int32)
    ho = dem.obs.astype(np.int32)
    for a in range(0, n_shots, chunk):
        b = min(n_shots, a + chunk)
        e = shots.sample_errors(key, nm, dem.priors, shot_start + a, b - a)
        errs[a:b] = e
        ei = e.astype(np.int32)
        syns[a:b] = (ei @ hs.T) & 1
        obs[a:b] = (ei @ ho.T) & 1
    return errs, syns, obs
