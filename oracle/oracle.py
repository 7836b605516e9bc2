"""Python access to the CPU oracle for BP-SF (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module. It wraps ``bpsf_oracle.c`` (see that file for the method and the
readings of the paper it follows) and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build


class _Params(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("cand_max_iter", C.c_int32), ("k", C.c_int32),
                ("cand_mode", C.c_int32), ("w_max", C.c_int32), ("select_mode", C.c_int32),
                ("alpha", C.c_double), ("flags", C.c_int32), ("rule", C.c_int32)]


NO_EARLY_STOP = 1
FORCE_PP = 2
LAYERED = 8          # layered schedule: checks by greedy layer, then by index
ALL_SUBSETS, WEIGHT_LE = 0, 1
MIN_WEIGHT, FIRST = 0, 1
MIN_SUM, SUM_PRODUCT = 0, 1


@dataclass
class Params:
    max_iter: int = 100
    cand_max_iter: int = 20
    k: int = 6
    cand_mode: int = ALL_SUBSETS
    w_max: int = 1
    select_mode: int = MIN_WEIGHT
    alpha: float = 0.625
    flags: int = 0
    rule: int = MIN_SUM

    def c(self) -> _Params:
        return _Params(self.max_iter, self.cand_max_iter, self.k, self.cand_mode, self.w_max,
                       self.select_mode, float(self.alpha), self.flags, self.rule)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _csr(h):
    if isinstance(h, tuple):
        row_ptr, col_idx, m, n = h
        return (np.ascontiguousarray(row_ptr, dtype=np.int32), np.ascontiguousarray(col_idx, dtype=np.int32),
                int(m), int(n))
    h = np.asarray(h, dtype=np.uint8)
    rows, cols = np.nonzero(h)
    counts = np.bincount(rows, minlength=h.shape[0])
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return row_ptr, cols.astype(np.int32), h.shape[0], h.shape[1]


def _real(prec):
    return (np.float64, C.c_double) if prec == "f64" else (np.float32, C.c_float)


def _priors(p, n):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(p, dtype=np.float64), (n,)))


class OracleLib:
    """The oracle's two builds (double and float). ``paths`` overrides the
    in-tree libraries (used to run the pins against planted mistakes)."""

    def __init__(self, paths: dict | None = None):
        self._paths = paths
        self._libs = {}

    def lib(self, prec: str = "f64"):
        if prec not in self._libs:
            if self._paths is not None:
                path = self._paths[prec]
            else:
                path = _build.lib_path(prec)
                if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                    _build.build(force=True)
            self._libs[prec] = C.CDLL(path)
        return self._libs[prec]

    def bp(self, h, syndrome, priors, params: Params, max_iter: int | None = None, prec: str = "f64",
           trace: bool = False):
        """One BP run (no post-processing). Returns hard decision, marginals,
        flip counts, iterations, converged flag and, with ``trace``,
        per-iteration records (edges in row-major order of H)."""
        row_ptr, col_idx, m, n = _csr(h)
        e = int(row_ptr[-1])
        it_max = params.max_iter if max_iter is None else max_iter
        dt, ct = _real(prec)
        s = np.ascontiguousarray(syndrome, dtype=np.uint8)
        p = _priors(priors, n)
        hard = np.zeros(n, np.uint8)
        lout = np.zeros(n, dt)
        flips = np.zeros(n, np.int32)
        tc = np.zeros((it_max, e), dt) if trace else None
        tv = np.zeros((it_max, e), dt) if trace else None
        tl = np.zeros((it_max, n), dt) if trace else None
        th = np.zeros((it_max, n), np.uint8) if trace else None
        iters = C.c_int32(0)
        conv = C.c_uint8(0)
        prm = params.c()
        fn = getattr(self.lib(prec), f"oracle_bp_{prec}")
        rc = fn(C.c_int32(m), C.c_int32(n), _ptr(row_ptr, C.c_int32), _ptr(col_idx, C.c_int32),
                _ptr(s, C.c_uint8), _ptr(p, C.c_double), C.byref(prm), C.c_int32(it_max),
                _ptr(hard, C.c_uint8), _ptr(lout, ct), _ptr(flips, C.c_int32),
                _ptr(tc, ct), _ptr(tv, ct), _ptr(tl, ct), _ptr(th, C.c_uint8),
                C.byref(iters), C.byref(conv))
        if rc != 0:
            raise ValueError("oracle_bp rejected its arguments")
        out = {"hard": hard, "lout": lout, "flips": flips, "iterations": iters.value,
               "converged": conv.value}
        if trace:
            k = iters.value
            out.update(trace_c2v=tc[:k], trace_v2c=tv[:k], trace_lout=tl[:k], trace_hard=th[:k])
        return out

    def trial_masks(self, params: Params) -> np.ndarray:
        fn = self.lib("f64").oracle_num_trials_f64
        fn.restype = C.c_int64
        prm = params.c()
        n = fn(C.byref(prm), None)
        if n < 0:
            raise ValueError("invalid trial parameters")
        masks = np.zeros(max(n, 1), np.uint32)
        fn(C.byref(prm), _ptr(masks, C.c_uint32))
        return masks[:n]

    def bpsf_detail(self, h, syndrome, priors, params: Params, prec: str = "f64"):
        """BP-SF on one syndrome with every intermediate (Phi, flip counts,
        per-trial results)."""
        row_ptr, col_idx, m, n = _csr(h)
        nt = len(self.trial_masks(params))
        s = np.ascontiguousarray(syndrome, dtype=np.uint8)
        p = _priors(priors, n)
        corr = np.zeros(n, np.uint8)
        phi = np.full(max(params.k, 1), -1, np.int32)
        flips = np.zeros(n, np.int32)
        tconv = np.zeros(max(nt, 1), np.uint8)
        titer = np.zeros(max(nt, 1), np.int32)
        twt = np.zeros(max(nt, 1), np.int32)
        summ = np.zeros(5, np.int32)
        ttot = C.c_int64(0)
        prm = params.c()
        fn = getattr(self.lib(prec), f"oracle_bpsf_detail_{prec}")
        rc = fn(C.c_int32(m), C.c_int32(n), _ptr(row_ptr, C.c_int32), _ptr(col_idx, C.c_int32),
                _ptr(s, C.c_uint8), _ptr(p, C.c_double), C.byref(prm), _ptr(corr, C.c_uint8),
                _ptr(phi, C.c_int32), _ptr(flips, C.c_int32), _ptr(tconv, C.c_uint8),
                _ptr(titer, C.c_int32), _ptr(twt, C.c_int32), _ptr(summ, C.c_int32), C.byref(ttot))
        if rc != 0:
            raise ValueError("oracle_bpsf_detail rejected its arguments")
        return {"correction": corr, "phi": phi[:params.k], "flips": flips,
                "trial_converged": tconv[:nt], "trial_iterations": titer[:nt], "trial_weight": twt[:nt],
                "converged": int(summ[0]), "iterations": int(summ[1]), "main_iterations": int(summ[2]),
                "main_converged": int(summ[3]), "winner": int(summ[4]),
                "trial_iteration_total": ttot.value}

    def bpsf_batch(self, h, syndromes, priors, params: Params, prec: str = "f64", threads: int = 1,
                   masks=None):
        """BP-SF over a batch of syndromes ``[shots, M]``; shots split over threads.
        ``masks``: trial vectors given by the caller instead of
        ``params.cand_mode``, either ``[n_trials]`` (every shot) or
        ``[shots, n_trials]`` (one list per shot)."""
        row_ptr, col_idx, m, n = _csr(h)
        syn = np.ascontiguousarray(syndromes, dtype=np.uint8)
        if syn.ndim != 2 or syn.shape[1] != m:
            raise ValueError("syndromes must be [shots, M]")
        shots = syn.shape[0]
        p = _priors(priors, n)
        k = max(params.k, 1)
        corr = np.zeros((shots, n), np.uint8)
        conv = np.zeros(shots, np.uint8)
        iters = np.zeros(shots, np.int32)
        winner = np.zeros(shots, np.int32)
        phi = np.zeros((shots, k), np.int32)
        main_it = np.zeros(shots, np.int32)
        trial_it = np.zeros(shots, np.int64)
        prm = params.c()
        outs = (_ptr(corr, C.c_uint8), _ptr(conv, C.c_uint8), _ptr(iters, C.c_int32),
                _ptr(winner, C.c_int32), _ptr(phi, C.c_int32), _ptr(main_it, C.c_int32),
                _ptr(trial_it, C.c_int64), C.c_int32(threads))
        if masks is None:
            fn = getattr(self.lib(prec), f"oracle_bpsf_batch_{prec}")
            rc = fn(C.c_int32(m), C.c_int32(n), _ptr(row_ptr, C.c_int32), _ptr(col_idx, C.c_int32),
                    _ptr(syn, C.c_uint8), C.c_int64(shots), _ptr(p, C.c_double), C.byref(prm), *outs)
        else:
            # 64-bit masks when the list is 64-bit (|Phi| up to 64), else 32-bit
            wide = np.asarray(masks).dtype in (np.uint64, np.int64)
            tab = np.ascontiguousarray(masks, dtype=np.uint64 if wide else np.uint32)
            if tab.ndim == 1:
                nt, stride = tab.shape[0], 0
            elif tab.ndim == 2 and tab.shape[0] == shots:
                nt, stride = tab.shape[1], tab.shape[1]
            else:
                raise ValueError("masks must be [n_trials] or [shots, n_trials]")
            fn = getattr(self.lib(prec), f"oracle_bpsf_batch_table{'64' if wide else ''}_{prec}")
            rc = fn(C.c_int32(m), C.c_int32(n), _ptr(row_ptr, C.c_int32), _ptr(col_idx, C.c_int32),
                    _ptr(syn, C.c_uint8), C.c_int64(shots), _ptr(p, C.c_double), C.byref(prm),
                    _ptr(tab, C.c_uint64 if wide else C.c_uint32), C.c_int64(nt), C.c_int64(stride), *outs)
        if rc != 0:
            raise ValueError("oracle_bpsf_batch rejected its arguments")
        return {"correction": corr, "converged": conv, "iterations": iters, "winner": winner,
                "phi": phi[:, :params.k], "main_iterations": main_it, "trial_iterations": trial_it}


_DEFAULT = OracleLib()
bp = _DEFAULT.bp
trial_masks = _DEFAULT.trial_masks
bpsf_detail = _DEFAULT.bpsf_detail
bpsf_batch = _DEFAULT.bpsf_batch
