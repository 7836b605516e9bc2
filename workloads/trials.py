"""Sampled trial vectors (the sampling-based trial sets of Section IV's
circuit-level experiments): for every weight w in 1..w_max, n_s distinct
w-subsets of the k positions of Phi, or every w-subset when there are no
more than n_s. Masks use bit j <-> Phi[j]; weights come in ascending order,
subsets of one weight in draw order. Draws use the counter-based generator
of ``shots`` (SplitMix64 keyed by (key, list, weight, draw)), so a list is a
pure function of its key and index; nothing here decodes anything."""
from __future__ import annotations

from math import comb

import numpy as np

from .shots import stream_key, uniforms


def _subset(key: np.uint64, k: int, w: int, draw: int) -> int:
    """A uniform w-subset of range(k) by a partial Fisher-Yates shuffle."""
    u = uniforms(stream_key(int(key), draw), 0, w)
    pos = list(range(k))
    mask = 0
    for i in range(w):
        j = i + int(u[i] * (k - i))
        pos[i], pos[j] = pos[j], pos[i]
        mask |= 1 << pos[i]
    return mask


def sample_trial_list(k: int, w_max: int, n_s: int, key: np.uint64, index: int = 0) -> np.ndarray:
    """One list of trial masks: uint32 for |Phi| = k <= 32, uint64 up to 64."""
    if not (1 <= w_max <= k <= 64) or n_s < 1:
        raise ValueError("need 1 <= w_max <= k <= 64 and n_s >= 1")
    out = []
    for w in range(1, w_max + 1):
        lk = stream_key(int(key), index, w)
        if comb(k, w) <= n_s:
            # every subset, in combination order
            pos = list(range(w))
            while True:
                out.append(sum(1 << p for p in pos))
                j = w - 1
                while j >= 0 and pos[j] == k - w + j:
                    j -= 1
                if j < 0:
                    break
                pos[j] += 1
                for q in range(j + 1, w):
                    pos[q] = pos[q - 1] + 1
            continue
        seen, draw = [], 0
        while len(seen) < n_s:
            m = _subset(lk, k, w, draw)
            draw += 1
            if m not in seen:
                seen.append(m)
        out.extend(seen)
    return np.array(out, np.uint32 if k <= 32 else np.uint64)


def list_length(k: int, w_max: int, n_s: int) -> int:
    return sum(min(comb(k, w), n_s) for w in range(1, w_max + 1))


def sample_trial_table(k: int, w_max: int, n_s: int, key: np.uint64, shots: int) -> np.ndarray:
    """One list per shot: [shots, list_length(k, w_max, n_s)] (uint32, or
    uint64 for k > 32)."""
    return np.stack([sample_trial_list(k, w_max, n_s, key, i) for i in range(shots)]) if shots else \
        np.zeros((0, list_length(k, w_max, n_s)), np.uint32 if k <= 32 else np.uint64)
