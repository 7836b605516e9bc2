"""Linear algebra over GF(2) used to check codes and to score decoder outputs.

Evaluation helpers only (ranks, kernels, logical operators): the decoder
itself never calls these.
"""
from __future__ import annotations

import numpy as np


def _rref(m: np.ndarray):
    """Reduced row echelon form over GF(2). Returns (matrix, pivot columns)."""
    a = (np.asarray(m, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    pivots = []
    r = 0
    for c in range(cols):
        if r >= rows:
            break
        nz = np.nonzero(a[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        hit = np.nonzero(a[:, c])[0]
        hit = hit[hit != r]
        if hit.size:
            a[hit] ^= a[r]
        pivots.append(c)
        r += 1
    return a[:r], pivots


def rank(m: np.ndarray) -> int:
    return len(_rref(m)[1])


def nullspace(m: np.ndarray) -> np.ndarray:
    """Basis (rows) of ``{x : m x = 0}`` over GF(2)."""
    m = np.asarray(m, dtype=np.uint8)
    n = m.shape[1]
    red, piv = _rref(m)
    free = [c for c in range(n) if c not in set(piv)]
    basis = np.zeros((len(free), n), dtype=np.uint8)
    for i, f in enumerate(free):
        basis[i, f] = 1
        for row, pc in zip(red, piv):
            if row[f]:
                basis[i, pc] = 1
    return basis


def logical_basis(h_detect: np.ndarray, h_other: np.ndarray) -> np.ndarray:
    """Logical operators that read out errors detected by ``h_detect``.

    An error ``r`` with ``h_detect r = 0`` is harmless exactly when it lies in the
    row space of ``h_other`` (the stabilizers of the same type as ``r``). The
    returned rows span ``ker(h_other)`` modulo ``rowspace(h_detect)``, so
    ``L r != 0`` flags a logical error.
    """
    ker = nullspace(h_other)
    base = np.asarray(h_detect, dtype=np.uint8)
    cur = rank(base)
    picked = []
    for v in ker:
        trial = np.vstack([base] + picked + [v[None, :]])
        rk = rank(trial)
        if rk > cur:
            picked.append(v[None, :])
            cur = rk
    if not picked:
        return np.zeros((0, base.shape[1]), dtype=np.uint8)
    return np.vstack(picked).astype(np.uint8)


def code_dimension(hx: np.ndarray, hz: np.ndarray) -> int:
    """Number of logical qubits ``k = n - rank(H_X) - rank(H_Z)``."""
    return hx.shape[1] - rank(hx) - rank(hz)


def parity(mat: np.ndarray, vecs: np.ndarray) -> np.ndarray:
    """``vecs @ mat.T mod 2`` for a batch of 0/1 row vectors (exact via int32)."""
    return ((np.asarray(vecs, dtype=np.int32) @ np.asarray(mat, dtype=np.int32).T) & 1).astype(np.uint8)
