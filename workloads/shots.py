"""Seeded synthetic shots: i.i.d. bit-flip errors and their syndromes.

Input generation only. Randomness comes from a counter-based generator so any
partition of a workload (by shot range, by process) reproduces the same data:
the value for (stream, index) is SplitMix64's output function applied to
``key + (index + 1) * 0x9E3779B97F4A7C15`` (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), where ``key`` is the
same function applied to the seed and the stream identifiers.

An error bit is set when the 53-bit uniform ``(u >> 11) * 2^-53`` is below its
probability; the syndrome is ``s = H e mod 2`` (the decoding problem of the
paper's Section II-B).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASTER_SEED = 2507_00254


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(*ids: int) -> np.uint64:
    """Fold integer identifiers (seed, config, code, p index, ...) into one key."""
    with np.errstate(over="ignore"):
        k = np.uint64(0)
        for i in ids:
            k = _mix(np.asarray(k + (np.uint64(i & 0xFFFFFFFFFFFFFFFF) + np.uint64(1)) * GAMMA, dtype=np.uint64))
        return np.uint64(k)


def uniforms(key: np.uint64, start: int, count: int) -> np.ndarray:
    """``count`` doubles in [0, 1) for counters ``start .. start+count-1``."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start, start + count, dtype=np.uint64) + np.uint64(1)
        z = _mix(np.uint64(key) + ctr * GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def sample_errors(key: np.uint64, n_bits: int, p, shot_start: int, n_shots: int) -> np.ndarray:
    """Errors ``e[shot, bit] = U(key, shot * n_bits + bit) < p[bit]`` as uint8."""
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), (n_bits,))
    u = uniforms(key, shot_start * n_bits, n_shots * n_bits).reshape(n_shots, n_bits)
    return (u < p[None, :]).astype(np.uint8)


def syndromes_of(h: np.ndarray, errors: np.ndarray) -> np.ndarray:
    """``s = H e mod 2`` for a batch of error rows (XOR over each row's support)."""
    h = np.asarray(h, dtype=np.uint8)
    out = np.zeros((errors.shape[0], h.shape[0]), dtype=np.uint8)
    for c in range(h.shape[0]):
        cols = np.nonzero(h[c])[0]
        if cols.size:
            out[:, c] = np.bitwise_xor.reduce(errors[:, cols], axis=1)
    return out


def make_shots(h: np.ndarray, p, n_shots: int, key: np.uint64, shot_start: int = 0,
               chunk: int = 1 << 16):
    """Seeded shots for check matrix ``h``: returns ``(errors, syndromes)`` uint8."""
    m, n = h.shape
    errs = np.empty((n_shots, n), dtype=np.uint8)
    syns = np.empty((n_shots, m), dtype=np.uint8)
    for a in range(0, n_shots, chunk):
        b = min(n_shots, a + chunk)
        e = sample_errors(key, n, p, shot_start + a, b - a)
        errs[a:b] = e
        syns[a:b] = syndromes_of(h, e)
    return errs, syns


def headline_shots(h: np.ndarray, p: float, n_shots: int):
    """The benchmark's shots for check matrix ``h`` at error rate ``p``: stream
    (master seed, 2, N, p * 10^5). Returns ``(errors, syndromes)``."""
    key = stream_key(MASTER_SEED, 2, h.shape[1], int(round(p * 100000)))
    return make_shots(h, p, n_shots, key)


def random_syndromes(m: int, n_shots: int, key: np.uint64, density: float = 0.5) -> np.ndarray:
    """Arbitrary (not necessarily feasible-by-low-weight) syndromes, for edge cases."""
    u = uniforms(key, 0, n_shots * m).reshape(n_shots, m)
    return (u < density).astype(np.uint8)


def interleave_order(key: np.uint64, n: int) -> np.ndarray:
    """A seeded permutation of ``range(n)`` (shots sorted by a counter-based
    hash of their position)."""
    return np.argsort(_mix(np.uint64(key) ^ np.arange(n, dtype=np.uint64)), kind="stable")


def mixed_batch(hs, p: float, per_code: int, key: np.uint64):
    """Shots of several check matrices mixed in one batch: ``per_code`` seeded
    shots of each ``hs[c]`` (stream ``stream_key(key, c)``) interleaved by a
    seeded permutation. Returns ``(shot_code int32 [n], syndromes uint8
    [n, max M] zero-padded, errors list per code, order)`` where ``order[i]``
    is the position in the code-major concatenation of shot ``i``."""
    n_codes = len(hs)
    mmax = max(h.shape[0] for h in hs)
    errs, syns = [], []
    for c, h in enumerate(hs):
        e, s = make_shots(h, p, per_code, stream_key(int(key), c))
        errs.append(e)
        pad = np.zeros((per_code, mmax), np.uint8)
        pad[:, :h.shape[0]] = s
        syns.append(pad)
    code_major = np.concatenate(syns)
    codes_major = np.repeat(np.arange(n_codes, dtype=np.int32), per_code)
    order = interleave_order(stream_key(int(key), 0x6d6978), n_codes * per_code)
    return codes_major[order], np.ascontiguousarray(code_major[order]), errs, order
