"""Parity-check matrices of the codes the decoder is exercised on.

Input generation only: these constructors produce H, which both the CPU
oracle and the GPU library take as an input. Nothing here decodes.

Constructions follow the paper's Appendix A ("Code Construction"):

* shift matrix ``S_l = I_l >> 1`` (each row of the identity cyclically shifted
  right by one, so ``S[i, (i+1) % l] = 1``; the paper prints ``S_3`` as a
  worked example);
* generalized-bicycle (GB) codes: ``x = S_l``, ``A = a(x)``, ``B = b(x)``;
* bivariate-bicycle (BB) codes: ``x = S_l (x) I_m``, ``y = I_l (x) S_m``,
  ``A = a(x, y)``, ``B = b(x, y)`` (table "BB Codes Used in Simulations");
* coprime-BB codes: ``pi = x y``, ``A = a(pi)``, ``B = b(pi)``
  (table "Coprime-BB Codes Used in Simulations");
* in all three, ``H_X = [A | B]`` and ``H_Z = [B^T | A^T]``.

The phenomenological space-time matrix (repeated noisy syndrome rounds) is not
in the paper; its reading is documented at :func:`phenomenological`.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def shift_matrix(l: int) -> np.ndarray:
    """``S_l = I_l >> 1``: row ``i`` has its single one in column ``(i+1) mod l``."""
    s = np.zeros((l, l), dtype=np.uint8)
    s[np.arange(l), (np.arange(l) + 1) % l] = 1
    return s


def _matpow_mod2(m: np.ndarray, e: int) -> np.ndarray:
    out = np.eye(m.shape[0], dtype=np.int64)
    base = m.astype(np.int64)
    while e:
        if e & 1:
            out = (out @ base) & 1
        base = (base @ base) & 1
        e >>= 1
    return out.astype(np.uint8)


def _poly2(terms, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Sum over GF(2) of monomials ``x^i y^j`` given as ``(i, j)`` pairs."""
    acc = np.zeros_like(x, dtype=np.uint8)
    for i, j in terms:
        acc ^= ((_matpow_mod2(x, i).astype(np.int64) @ _matpow_mod2(y, j).astype(np.int64)) & 1).astype(np.uint8)
    return acc


def _css(a: np.ndarray, b: np.ndarray):
    hx = np.concatenate([a, b], axis=1)
    hz = np.concatenate([b.T, a.T], axis=1)
    return np.ascontiguousarray(hx), np.ascontiguousarray(hz)


@dataclass
class Code:
    """A CSS code given by its two check matrices (uint8 0/1, dense)."""
    name: str
    hx: np.ndarray
    hz: np.ndarray
    n: int
    k: int | None = None      # logical qubits, when known
    d: int | None = None      # distance, when known
    meta: dict = field(default_factory=dict)


def bb_code(l: int, m: int, a_terms, b_terms, name: str = "") -> Code:
    """Bivariate-bicycle code: ``x = S_l (x) I_m``, ``y = I_l (x) S_m``."""
    x = np.kron(shift_matrix(l), np.eye(m, dtype=np.uint8)).astype(np.uint8)
    y = np.kron(np.eye(l, dtype=np.uint8), shift_matrix(m)).astype(np.uint8)
    a = _poly2(a_terms, x, y)
    b = _poly2(b_terms, x, y)
    hx, hz = _css(a, b)
    return Code(name or f"bb_{l}x{m}", hx, hz, hx.shape[1],
                meta={"family": "bb", "l": l, "m": m, "a": list(a_terms), "b": list(b_terms)})


def gb_code(l: int, a_pows, b_pows, name: str = "") -> Code:
    """Generalized-bicycle code: ``x = S_l``, ``A = a(x)``, ``B = b(x)``."""
    x = shift_matrix(l)
    one = np.eye(l, dtype=np.uint8)
    a = _poly2([(p, 0) for p in a_pows], x, one)
    b = _poly2([(p, 0) for p in b_pows], x, one)
    hx, hz = _css(a, b)
    return Code(name or f"gb_{l}", hx, hz, hx.shape[1],
                meta={"family": "gb", "l": l, "a": list(a_pows), "b": list(b_pows)})


def coprime_bb_code(l: int, m: int, a_pows, b_pows, name: str = "") -> Code:
    """Coprime-BB code: ``pi = x y`` with x, y as for BB codes."""
    x = np.kron(shift_matrix(l), np.eye(m, dtype=np.uint8)).astype(np.uint8)
    y = np.kron(np.eye(l, dtype=np.uint8), shift_matrix(m)).astype(np.uint8)
    pi = ((x.astype(np.int64) @ y.astype(np.int64)) & 1).astype(np.uint8)
    one = np.eye(l * m, dtype=np.uint8)
    a = _poly2([(p, 0) for p in a_pows], pi, one)
    b = _poly2([(p, 0) for p in b_pows], pi, one)
    hx, hz = _css(a, b)
    return Code(name or f"cbb_{l}x{m}", hx, hz, hx.shape[1],
                meta={"family": "coprime_bb", "l": l, "m": m, "a": list(a_pows), "b": list(b_pows)})


# Polynomials as (power of x, power of y) pairs.
_XY_A = [(3, 0), (0, 1), (0, 2)]          # x^3 + y + y^2
_XY_B = [(0, 3), (1, 0), (2, 0)]          # y^3 + x + x^2


def bb72() -> Code:
    """[[72,12,6]]: l = m = 6 (Appendix A, BB table)."""
    c = bb_code(6, 6, _XY_A, _XY_B, "bb72")
    c.k, c.d = 12, 6
    return c


def bb90() -> Code:
    """[[90,8,10]]: l = 15, m = 3, a = x^9 + y + y^2, b = 1 + x^2 + x^7."""
    c = bb_code(15, 3, [(9, 0), (0, 1), (0, 2)], [(0, 0), (2, 0), (7, 0)], "bb90")
    c.k, c.d = 8, 10
    return c


def bb108() -> Code:
    """[[108,8,10]]: l = 9, m = 6 with the [[72]]/[[144]] polynomials.

    The paper does not list this code; the polynomials are a reading (same
    family as the gross code), confirmed by the GF(2) rank giving k = 8.
    """
    c = bb_code(9, 6, _XY_A, _XY_B, "bb108")
    c.k, c.d = 8, 10
    return c


def bb144() -> Code:
    """[[144,12,12]] "gross" code: l = 12, m = 6 (Appendix A, BB table)."""
    c = bb_code(12, 6, _XY_A, _XY_B, "bb144")
    c.k, c.d = 12, 12
    return c


def bb288() -> Code:
    """[[288,12,18]]: l = m = 12, a = x^3 + y^2 + y^7, b = y^3 + x + x^2."""
    c = bb_code(12, 12, [(3, 0), (0, 2), (0, 7)], _XY_B, "bb288")
    c.k, c.d = 12, 18
    return c


def gb254() -> Code:
    """[[254,28]] GB code, l = 127 (Appendix A, GB codes)."""
    c = gb_code(127, [0, 15, 20, 28, 66], [0, 58, 59, 100, 121], "gb254")
    c.k = 28
    return c


def cbb126() -> Code:
    """[[126,12,10]] coprime-BB, l = 7, m = 9, a = 1 + pi + pi^58, b = 1 + pi^13 + pi^41."""
    c = coprime_bb_code(7, 9, [0, 1, 58], [0, 13, 41], "cbb126")
    c.k, c.d = 12, 10
    return c


def cbb154() -> Code:
    """[[154,6,16]] coprime-BB, l = 7, m = 11, a = 1 + pi + pi^31, b = 1 + pi^19 + pi^53."""
    c = coprime_bb_code(7, 11, [0, 1, 31], [0, 19, 53], "cbb154")
    c.k, c.d = 6, 16
    return c


def phenomenological(h: np.ndarray, rounds: int) -> np.ndarray:
    """Space-time check matrix for ``rounds`` noisy syndrome-extraction rounds.

    Reading (the paper uses Stim detector error models for circuit noise and
    does not describe a phenomenological model):
    ``H = [I_R (x) H | B_R (x) I_M]`` where ``B_R`` is lower bidiagonal. Rows are
    detectors (round-major: the difference of consecutive syndrome
    measurements); the first ``R*N`` columns are data errors occurring before
    round ``r``'s measurement (they flip only detectors of round ``r``); the last
    ``R*M`` columns are measurement errors of round ``r`` (they flip detectors
    ``r`` and ``r+1``; in the last round only ``r``, as there is no perfect final
    round).
    """
    m, n = h.shape
    r = rounds
    data = np.kron(np.eye(r, dtype=np.uint8), h)
    b = np.eye(r, dtype=np.uint8) + np.eye(r, k=-1, dtype=np.uint8)
    meas = np.kron(b, np.eye(m, dtype=np.uint8))
    return np.ascontiguousarray(np.concatenate([data, meas], axis=1).astype(np.uint8))


def csr(h: np.ndarray):
    """Row-major sparse form of a dense 0/1 matrix: ``(row_ptr, col_idx)`` int32,
    column indices ascending within each row."""
    h = np.asarray(h, dtype=np.uint8)
    rows, cols = np.nonzero(h)
    row_ptr = np.zeros(h.shape[0] + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr, dtype=np.int64).astype(np.int32)
    return row_ptr, cols.astype(np.int32)


CODES = {
    "bb72": bb72, "bb90": bb90, "bb108": bb108, "bb144": bb144, "bb288": bb288,
    "gb254": gb254, "cbb126": cbb126, "cbb154": cbb154,
}


def get_code(name: str) -> Code:
    return CODES[name]()
