"""Python binding of ``libbpsf.so`` (argument marshalling only).

Every decoding step runs in the library's HIP kernels; PyTorch provides device
memory and streams. The functions keep the C ABI's names (``include/bpsf.h``);
:class:`Decoder` is a convenience wrapper around them. Importing this module
loads the library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpsf.so")

BPSF_OK, BPSF_EINVAL, BPSF_ENOMEM, BPSF_ENOTSUP, BPSF_EDEVICE = 0, -1, -2, -3, -4
TRIALS_ALL_SUBSETS, TRIALS_WEIGHT_LE, TRIALS_TABLE = 0, 1, 2
SELECT_MIN_WEIGHT, SELECT_FIRST = 0, 1
FLAG_NO_EARLY_STOP, FLAG_FORCE_PP, FLAG_PRUNE, FLAG_LAYERED = 1, 2, 4, 8
PREC_FP32, PREC_FP64 = 0, 1


class bpsf_params(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("cand_max_iter", C.c_int32), ("k", C.c_int32),
                ("cand_mode", C.c_int32), ("w_max", C.c_int32), ("select_mode", C.c_int32),
                ("alpha", C.c_double), ("flags", C.c_int32), ("precision", C.c_int32)]


class bpsf_stats(C.Structure):
    _fields_ = [("main_iterations", C.c_int64), ("trial_iterations", C.c_int64),
                ("rerun_iterations", C.c_int64), ("failed_shots", C.c_int64),
                ("converged_trials", C.c_int64), ("errors", C.c_int64)]


class bpsf_tuning(C.Structure):
    _fields_ = [("decodes_per_wave", C.c_int32), ("waves_per_cu", C.c_int32), ("ms", C.c_float),
                ("candidates", C.c_int32)]


class BpsfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbpsf error {code}: {msg}")
        self.code = code


class BpsfArgumentError(BpsfError, ValueError):
    """An argument the binding rejects before calling the library (a tensor of
    the wrong shape, element type or device, or a priors array of the wrong
    length): the library would read or write out of bounds with it."""

    def __init__(self, msg):
        super().__init__(BPSF_EINVAL, msg)


def _load():
    # torch brings its own HIP runtime; it has to be in the process before
    # this library resolves libamdhip64, or torch later finds no GPU
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2507_00254_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    lib.bpsf_load_code.argtypes = [P(i32), P(i32), i32, i32, P(vp)]
    lib.bpsf_free_code.argtypes = [vp]
    lib.bpsf_free_code.restype = None
    lib.bpsf_decode.argtypes = [vp, vp, P(C.c_double), i64, P(bpsf_params), vp, vp, vp, vp]
    lib.bpsf_decode_noalloc.argtypes = [vp, vp, P(C.c_double), i64, P(bpsf_params), vp, vp, vp, vp]
    lib.bpsf_last_stats.argtypes = [vp, vp, P(bpsf_stats)]
    lib.bpsf_bp_trace.argtypes = [vp, P(C.c_uint8), P(C.c_double), P(bpsf_params), vp, vp, P(C.c_uint8),
                                  P(i32), P(C.c_uint8)]
    lib.bpsf_num_trials.argtypes = [P(bpsf_params), P(C.c_uint32), i64]
    lib.bpsf_num_trials.restype = i64
    lib.bpsf_set_timing.argtypes = [vp, C.c_int]
    lib.bpsf_last_timing.argtypes = [vp, P(C.c_float)]
    lib.bpsf_code_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(i32)]
    lib.bpsf_sparse_layout.argtypes = [P(i32), P(i32), i32, i32, P(i32), vp, vp, vp, vp, vp]
    lib.bpsf_tile_options.argtypes = [vp, P(i32), i32]
    lib.bpsf_reserve.argtypes = [vp, i64, P(bpsf_params)]
    lib.bpsf_set_trial_table.argtypes = [vp, vp, i64, i64]
    lib.bpsf_set_trial_table64.argtypes = [vp, vp, i64, i64]
    lib.bpsf_mix_reserve.argtypes = [vp, i64, P(bpsf_params)]
    lib.bpsf_set_tile.argtypes = [vp, i32, i32]
    lib.bpsf_autotune.argtypes = [vp, vp, P(C.c_double), i64, P(bpsf_params), i32, vp, P(bpsf_tuning)]
    lib.bpsf_mix_create.argtypes = [P(vp), i32, P(vp)]
    lib.bpsf_server_create.argtypes = [P(vp), i32, P(P(C.c_double)), P(bpsf_params), i32, i64, i32, i64, P(vp)]
    lib.bpsf_server_memory.argtypes = [vp, P(i64), P(i64), P(i64), P(i64), P(i64)]
    lib.bpsf_server_submit.argtypes = [vp, i32, vp, i32, vp, vp, vp, P(i64)]
    lib.bpsf_server_wait.argtypes = [vp, i64, P(C.c_double)]
    lib.bpsf_server_poll.argtypes = [vp, P(i64), i64]
    lib.bpsf_server_poll.restype = i64
    lib.bpsf_server_replay.argtypes = [vp, i64, P(C.c_double), P(i32), P(i32), P(vp), P(vp), P(vp), P(vp),
                                       P(C.c_double), P(C.c_double)]
    lib.bpsf_server_counters.argtypes = [vp, P(i64), P(i64), P(i64)]
    lib.bpsf_server_destroy.argtypes = [vp]
    lib.bpsf_mix_free.argtypes = [vp]
    lib.bpsf_mix_free.restype = None
    lib.bpsf_mix_decode.argtypes = [vp, vp, vp, i64, P(P(C.c_double)), i64, P(bpsf_params), vp, i64, vp, vp, vp]
    lib.bpsf_mix_last_stats.argtypes = [vp, vp, P(bpsf_stats), P(i64)]
    lib.bpsf_mix_decode_grouped.argtypes = [vp, P(i64), vp, i64, P(P(C.c_double)), P(bpsf_params), vp, i64, vp, vp,
                                            vp]
    lib.bpsf_last_error.argtypes = []
    lib.bpsf_last_error.restype = C.c_char_p
    return lib


LIB = _load()


def _check(rc):
    if rc != 0:
        raise BpsfError(rc, LIB.bpsf_last_error().decode())
    return rc


def make_params(max_iter=100, cand_max_iter=20, k=6, cand_mode=TRIALS_ALL_SUBSETS, w_max=1,
                select_mode=SELECT_MIN_WEIGHT, alpha=0.625, flags=0, precision=PREC_FP32) -> bpsf_params:
    return bpsf_params(max_iter, cand_max_iter, k, cand_mode, w_max, select_mode, float(alpha), flags, precision)


def _csr(h):
    if isinstance(h, tuple):
        row_ptr, col_idx, m, n = h
    else:
        h = np.asarray(h, dtype=np.uint8)
        rows, cols = np.nonzero(h)
        m, n = h.shape
        row_ptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))])
        col_idx = cols
    return (np.ascontiguousarray(row_ptr, dtype=np.int32), np.ascontiguousarray(col_idx, dtype=np.int32),
            int(m), int(n))


def bpsf_load_code(h) -> int:
    """H as a dense 0/1 array or ``(row_ptr, col_idx, M, N)``; returns the handle."""
    row_ptr, col_idx, m, n = _csr(h)
    out = C.c_void_p()
    _check(LIB.bpsf_load_code(row_ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                              col_idx.ctypes.data_as(C.POINTER(C.c_int32)), m, n, C.byref(out)))
    return out.value


def bpsf_free_code(handle) -> None:
    LIB.bpsf_free_code(handle)


def bpsf_num_trials(params: bpsf_params) -> np.ndarray:
    n = LIB.bpsf_num_trials(C.byref(params), None, 0)
    _check(n if n < 0 else 0)
    masks = np.zeros(max(n, 1), np.uint32)
    LIB.bpsf_num_trials(C.byref(params), masks.ctypes.data_as(C.POINTER(C.c_uint32)), n)
    return masks[:n]


def _stream_ptr(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _tensor(t, name, dtype, ndim):
    """A contiguous device tensor of the given element type and rank."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise BpsfArgumentError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise BpsfArgumentError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise BpsfArgumentError(f"{name} must have {ndim} dimension(s), got shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise BpsfArgumentError(f"{name} must be contiguous")
    return t


def _outputs(corrections, converged, iterations, shots, n_min, exact_n=None):
    """Output tensors able to hold `shots` results: corrections uint8 [>= shots,
    N] (N == exact_n, or >= n_min), converged uint8 [>= shots], iterations
    int32 [>= shots]."""
    import torch
    _tensor(corrections, "corrections", torch.uint8, 2)
    _tensor(converged, "converged", torch.uint8, 1)
    _tensor(iterations, "iterations", torch.int32, 1)
    if corrections.shape[0] < shots:
        raise BpsfArgumentError(f"corrections has {corrections.shape[0]} rows for {shots} shots")
    if exact_n is not None and corrections.shape[1] != exact_n:
        raise BpsfArgumentError(f"corrections rows must hold N = {exact_n} bits, got {corrections.shape[1]}")
    if corrections.shape[1] < n_min:
        raise BpsfArgumentError(f"corrections rows must hold at least {n_min} bits, got {corrections.shape[1]}")
    if converged.shape[0] < shots or iterations.shape[0] < shots:
        raise BpsfArgumentError(f"converged and iterations need at least {shots} entries")


def _priors_of(priors, n, what="priors"):
    pri = np.ascontiguousarray(priors, dtype=np.float64)
    if pri.ndim != 1 or pri.shape[0] != n:
        raise BpsfArgumentError(f"{what} must be a 1-D array of N = {n} probabilities, got shape {pri.shape}")
    return pri


def _on_device(*ts):
    for t in ts:
        if not t.is_cuda:
            raise BpsfArgumentError("device tensors must be CUDA (HIP) tensors")


def bpsf_decode(handle, syndromes, priors, params: bpsf_params, corrections, converged, iterations,
                stream=None, noalloc: bool = False) -> None:
    """Enqueue a decode. ``syndromes`` uint8 [shots, M], ``corrections`` uint8
    [shots, N], ``converged`` uint8 [shots], ``iterations`` int32 [shots] are
    torch tensors on the GPU; ``priors`` is a host array of N probabilities.
    Shapes and element types are checked here (the library takes rows of M
    and N bytes). ``noalloc`` calls bpsf_decode_noalloc (scratch in the
    library's fixed device array, no allocation)."""
    import torch
    info = bpsf_code_info(handle)
    m, n = info["M"], info["N"]
    _tensor(syndromes, "syndromes", torch.uint8, 2)
    if syndromes.shape[1] != m:
        raise BpsfArgumentError(f"syndromes rows must hold M = {m} checks, got {syndromes.shape[1]}")
    shots = int(syndromes.shape[0])
    _outputs(corrections, converged, iterations, shots, n, exact_n=n)
    pri = _priors_of(priors, n)
    _on_device(syndromes, corrections, converged, iterations)
    fn = LIB.bpsf_decode_noalloc if noalloc else LIB.bpsf_decode
    _check(fn(C.c_void_p(handle), C.c_void_p(syndromes.data_ptr()),
                           pri.ctypes.data_as(C.POINTER(C.c_double)), shots, C.byref(params),
                           C.c_void_p(corrections.data_ptr()), C.c_void_p(converged.data_ptr()),
                           C.c_void_p(iterations.data_ptr()), _stream_ptr(stream)))


def bpsf_last_stats(handle, stream=None) -> dict:
    st = bpsf_stats()
    _check(LIB.bpsf_last_stats(C.c_void_p(handle), _stream_ptr(stream), C.byref(st)))
    return {f: getattr(st, f) for f, _ in bpsf_stats._fields_}


def bpsf_set_timing(handle, enable: bool) -> None:
    _check(LIB.bpsf_set_timing(C.c_void_p(handle), int(bool(enable))))


def bpsf_last_timing(handle) -> dict:
    """Durations (ms) of the last timed decode: whole call and each phase."""
    ms = (C.c_float * 4)()
    _check(LIB.bpsf_last_timing(C.c_void_p(handle), ms))
    return {"total": ms[0], "main": ms[1], "trials": ms[2], "rerun": ms[3]}


def bpsf_set_trial_table(handle, masks=None) -> None:
    """Trial list for TRIALS_TABLE: a device tensor [n_trials] (every shot) or
    [shots, n_trials] (one list per shot) of 32-bit masks (int32 / uint32
    bits), or of 64-bit masks (int64, |Phi| up to 64: bpsf_set_trial_table64),
    kept alive by the caller; None clears it."""
    if masks is None:
        _check(LIB.bpsf_set_trial_table(C.c_void_p(handle), None, 0, 0))
        return
    if not masks.is_cuda or not masks.is_contiguous():
        raise ValueError("masks must be a contiguous device tensor")
    n = int(masks.shape[-1])
    stride = n if masks.dim() == 2 else 0
    if masks.element_size() == 8:
        _check(LIB.bpsf_set_trial_table64(C.c_void_p(handle), C.c_void_p(masks.data_ptr()), n, stride))
    elif masks.element_size() == 4:
        _check(LIB.bpsf_set_trial_table(C.c_void_p(handle), C.c_void_p(masks.data_ptr()), n, stride))
    else:
        raise ValueError("masks must hold 32-bit or 64-bit elements")


def bpsf_reserve(handle, shots: int, params: bpsf_params) -> None:
    _check(LIB.bpsf_reserve(C.c_void_p(handle), int(shots), C.byref(params)))


def bpsf_mix_reserve(mix, shots: int, params: bpsf_params) -> None:
    _check(LIB.bpsf_mix_reserve(C.c_void_p(mix), int(shots), C.byref(params)))


def bpsf_tile_options(handle) -> list:
    """Decodes per wave the code fits, most first."""
    buf = (C.c_int32 * 8)()
    n = LIB.bpsf_tile_options(C.c_void_p(handle), buf, 8)
    _check(n if n < 0 else 0)
    return [buf[i] for i in range(min(n, 8))]


def bpsf_set_tile(handle, decodes_per_wave: int = 0, waves_per_cu: int = 0) -> None:
    _check(LIB.bpsf_set_tile(C.c_void_p(handle), int(decodes_per_wave), int(waves_per_cu)))


def bpsf_autotune(handle, syndromes, priors, params: bpsf_params, reps: int = 3, stream=None) -> dict:
    """Time every launch shape on a device sample of syndromes; keep the fastest."""
    import torch
    info = bpsf_code_info(handle)
    _tensor(syndromes, "syndromes", torch.uint8, 2)
    if syndromes.shape[1] != info["M"]:
        raise BpsfArgumentError(f"syndromes rows must hold M = {info['M']} checks, got {syndromes.shape[1]}")
    pri = _priors_of(priors, info["N"])
    _on_device(syndromes)
    out = bpsf_tuning()
    _check(LIB.bpsf_autotune(C.c_void_p(handle), C.c_void_p(syndromes.data_ptr()),
                             pri.ctypes.data_as(C.POINTER(C.c_double)), int(syndromes.shape[0]), C.byref(params),
                             int(reps), _stream_ptr(stream), C.byref(out)))
    return {f: getattr(out, f) for f, _ in bpsf_tuning._fields_}


def bpsf_mix_create(handles) -> int:
    """A mix handle over loaded codes (see bpsf_mix_decode)."""
    arr = (C.c_void_p * len(handles))(*handles)
    out = C.c_void_p()
    _check(LIB.bpsf_mix_create(arr, len(handles), C.byref(out)))
    _MIX_SHAPES[out.value] = [(i["M"], i["N"]) for i in (bpsf_code_info(h) for h in handles)]
    return out.value


# (M, N) of every code of a mix handle, for argument checks
_MIX_SHAPES: dict = {}


def bpsf_mix_free(mix) -> None:
    _MIX_SHAPES.pop(mix, None)
    LIB.bpsf_mix_free(mix)


def _mix_args(mix, syndromes, priors, corrections, converged, iterations, shots):
    import torch
    shapes = _MIX_SHAPES.get(mix)
    if shapes is None:
        raise BpsfArgumentError("unknown mix handle (create it with bpsf_mix_create)")
    _tensor(syndromes, "syndromes", torch.uint8, 2)
    mmax = max(m for m, _ in shapes)
    nmax = max(n for _, n in shapes)
    if syndromes.shape[0] < shots:
        raise BpsfArgumentError(f"syndromes has {syndromes.shape[0]} rows for {shots} shots")
    if syndromes.shape[1] < mmax:
        raise BpsfArgumentError(f"syndromes rows must hold the largest M = {mmax}, got {syndromes.shape[1]}")
    _outputs(corrections, converged, iterations, shots, nmax)
    if len(priors) != len(shapes):
        raise BpsfArgumentError(f"need one priors array per code ({len(shapes)}), got {len(priors)}")
    return [_priors_of(x, n, f"priors[{c}]") for c, (x, (_, n)) in enumerate(zip(priors, shapes))]


def bpsf_mix_decode(mix, shot_code, syndromes, priors, params: bpsf_params, corrections, converged, iterations,
                    stream=None) -> None:
    """Enqueue a decode of shots of several codes. ``shot_code`` int32
    [shots], ``syndromes`` uint8 [shots, syn_stride], ``corrections`` uint8
    [shots, corr_stride], ``converged`` uint8 [shots], ``iterations`` int32
    [shots] are device tensors; ``priors`` is a list of host arrays, one per
    code of the mix."""
    import torch
    _tensor(shot_code, "shot_code", torch.int32, 1)
    shots = int(shot_code.shape[0])
    pri = _mix_args(mix, syndromes, priors, corrections, converged, iterations, shots)
    _on_device(shot_code, syndromes, corrections, converged, iterations)
    parr = (C.POINTER(C.c_double) * len(pri))(*[x.ctypes.data_as(C.POINTER(C.c_double)) for x in pri])
    _check(LIB.bpsf_mix_decode(C.c_void_p(mix), C.c_void_p(shot_code.data_ptr()), C.c_void_p(syndromes.data_ptr()),
                               int(syndromes.shape[1]), parr, shots, C.byref(params),
                               C.c_void_p(corrections.data_ptr()), int(corrections.shape[1]),
                               C.c_void_p(converged.data_ptr()), C.c_void_p(iterations.data_ptr()),
                               _stream_ptr(stream)))


def bpsf_mix_decode_grouped(mix, counts, syndromes, priors, params: bpsf_params, corrections, converged, iterations,
                            stream=None) -> None:
    """As bpsf_mix_decode with code c's shots the counts[c] rows after those
    of the codes before it."""
    cnt = np.ascontiguousarray(counts, dtype=np.int64)
    shapes = _MIX_SHAPES.get(mix)
    if shapes is not None and (cnt.ndim != 1 or cnt.shape[0] != len(shapes)):
        raise BpsfArgumentError(f"counts must hold one entry per code ({len(shapes)})")
    if (cnt < 0).any():
        raise BpsfArgumentError("counts must be >= 0")
    pri = _mix_args(mix, syndromes, priors, corrections, converged, iterations, int(cnt.sum()))
    _on_device(syndromes, corrections, converged, iterations)
    parr = (C.POINTER(C.c_double) * len(pri))(*[x.ctypes.data_as(C.POINTER(C.c_double)) for x in pri])
    _check(LIB.bpsf_mix_decode_grouped(C.c_void_p(mix), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                       C.c_void_p(syndromes.data_ptr()), int(syndromes.shape[1]), parr,
                                       C.byref(params), C.c_void_p(corrections.data_ptr()), int(corrections.shape[1]),
                                       C.c_void_p(converged.data_ptr()), C.c_void_p(iterations.data_ptr()),
                                       _stream_ptr(stream)))


def bpsf_mix_last_stats(mix, n_codes: int, stream=None):
    """Per-code work counters of the last mixed decode and the number of
    shots skipped for an out-of-range code index."""
    st = (bpsf_stats * n_codes)()
    bad = C.c_int64()
    _check(LIB.bpsf_mix_last_stats(C.c_void_p(mix), _stream_ptr(stream), st, C.byref(bad)))
    return [{f: getattr(x, f) for f, _ in bpsf_stats._fields_} for x in st], bad.value


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


class Server:
    """A request loop over loaded codes (see bpsf_server_create). Request
    buffers are numpy arrays; they are kept alive until collected."""

    def __init__(self, handles, priors, params: bpsf_params, lanes: int = 2, max_batch_shots: int = 65536,
                 batching: bool = True, device_budget_bytes: int = 0):
        self._pri = [np.ascontiguousarray(x, dtype=np.float64) for x in priors]
        parr = (C.POINTER(C.c_double) * len(self._pri))(*[x.ctypes.data_as(C.POINTER(C.c_double))
                                                          for x in self._pri])
        arr = (C.c_void_p * len(handles))(*handles)
        out = C.c_void_p()
        self._shapes = [(i["M"], i["N"]) for i in (bpsf_code_info(h) for h in handles)]
        if len(self._pri) != len(handles):
            raise BpsfArgumentError(f"need one priors array per code ({len(handles)}), got {len(self._pri)}")
        for c, (x, (_, n)) in enumerate(zip(self._pri, self._shapes)):
            _priors_of(x, n, f"priors[{c}]")
        _check(LIB.bpsf_server_create(arr, len(handles), parr, C.byref(params), int(lanes), int(max_batch_shots),
                                      int(bool(batching)), int(device_budget_bytes), C.byref(out)))
        self.h = out.value
        self._live = {}

    def submit(self, code: int, syndromes: np.ndarray):
        """Enqueue host syndromes uint8 [n, M]; returns (id, corrections,
        converged, iterations) whose arrays fill in once the request is done."""
        syn = self._syndromes(code, syndromes)
        n = syn.shape[0]
        nbits = self._n_of(code)
        corr = np.empty((n, nbits), np.uint8)
        conv = np.empty(n, np.uint8)
        it = np.empty(n, np.int32)
        rid = C.c_int64()
        _check(LIB.bpsf_server_submit(C.c_void_p(self.h), int(code), _ptr(syn), n, _ptr(corr), _ptr(conv), _ptr(it),
                                      C.byref(rid)))
        self._live[rid.value] = (syn, corr, conv, it)
        return rid.value, corr, conv, it

    def wait(self, rid: int) -> float:
        lat = C.c_double()
        try:
            _check(LIB.bpsf_server_wait(C.c_void_p(self.h), int(rid), C.byref(lat)))
        finally:
            self._live.pop(rid, None)
        return lat.value

    def poll(self, cap: int = 4096):
        ids = np.zeros(cap, np.int64)
        n = LIB.bpsf_server_poll(C.c_void_p(self.h), ids.ctypes.data_as(C.POINTER(C.c_int64)), cap)
        _check(n if n < 0 else 0)
        return ids[:n].tolist()

    def replay(self, arrival_s, codes, syndromes):
        """Open-loop replay: request i (host syndromes[i] of codes[i]) submitted
        arrival_s[i] s after the start. Returns (latencies_s, wall_s, outputs)."""
        n = len(codes)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        cd = np.ascontiguousarray(codes, dtype=np.int32)
        if len(syndromes) != n or arr.shape != (n,):
            raise BpsfArgumentError("arrival_s, codes and syndromes must have one entry per request")
        syns = [self._syndromes(int(c), x) for c, x in zip(cd, syndromes)]
        sh = np.array([x.shape[0] for x in syns], np.int32)
        outs = [(np.empty((x.shape[0], self._n_of(int(c))), np.uint8), np.empty(x.shape[0], np.uint8),
                 np.empty(x.shape[0], np.int32)) for x, c in zip(syns, cd)]
        vp = C.c_void_p
        psyn = (vp * n)(*[x.ctypes.data for x in syns])
        pcor = (vp * n)(*[o[0].ctypes.data for o in outs])
        pcon = (vp * n)(*[o[1].ctypes.data for o in outs])
        pit = (vp * n)(*[o[2].ctypes.data for o in outs])
        lat = np.zeros(n, np.float64)
        wall = C.c_double()
        dp = C.POINTER(C.c_double)
        _check(LIB.bpsf_server_replay(C.c_void_p(self.h), n, arr.ctypes.data_as(dp),
                                      cd.ctypes.data_as(C.POINTER(C.c_int32)), sh.ctypes.data_as(C.POINTER(C.c_int32)),
                                      psyn, pcor, pcon, pit, lat.ctypes.data_as(dp), C.byref(wall)))
        return lat, wall.value, outs

    def counters(self) -> dict:
        v = [C.c_int64() for _ in range(3)]
        _check(LIB.bpsf_server_counters(C.c_void_p(self.h), *[C.byref(x) for x in v]))
        return dict(zip(("batches", "batch_shots", "requests_done"), (x.value for x in v)))

    def memory(self) -> dict:
        """Device pool: size, bytes in use now and at most, the largest
        request it holds, and the requests that waited for memory."""
        v = [C.c_int64() for _ in range(5)]
        _check(LIB.bpsf_server_memory(C.c_void_p(self.h), *[C.byref(x) for x in v]))
        return dict(zip(("budget", "in_use", "peak", "max_request", "waited_for_memory"), (x.value for x in v)))

    def close(self):
        if self.h:
            rc = LIB.bpsf_server_destroy(C.c_void_p(self.h))
            self.h = None
            self._live.clear()
            _check(rc)

    def _n_of(self, code: int) -> int:
        # an out-of-range code is left for the library to reject
        return self._shapes[code][1] if 0 <= code < len(self._shapes) else 1

    def _syndromes(self, code: int, syndromes) -> np.ndarray:
        """Host syndromes uint8 [n, M of the code] (the library copies n x M bytes)."""
        syn = np.ascontiguousarray(syndromes, dtype=np.uint8)
        if 0 <= code < len(self._shapes) and (syn.ndim != 2 or syn.shape[1] != self._shapes[code][0]):
            raise BpsfArgumentError(f"syndromes of code {code} must be [n, {self._shapes[code][0]}], got {syn.shape}")
        return syn


def bpsf_code_info(handle) -> dict:
    vals = [C.c_int32() for _ in range(5)]
    _check(LIB.bpsf_code_info(C.c_void_p(handle), *[C.byref(v) for v in vals]))
    return dict(zip(("M", "N", "edges", "row_weight", "col_weight"), (v.value for v in vals)))


SPARSE_INFO_WORDS = 9


def bpsf_sparse_layout(h):
    """The sparse family's LDS layout of a matrix (host only, no device):
    None when the matrix takes another kernel family, else a dict with the
    family, cells, WMAX, T, CPT, DVMAX, the layout's quality counts and the tables
    roff [M, WMAX], rw [M], bits [N], cperm [N], rperm [M]."""
    row_ptr, col_idx, m, n = _csr(h)
    info = np.zeros(SPARSE_INFO_WORDS, np.int32)
    ip = info.ctypes.data_as(C.POINTER(C.c_int32))
    rp, ci = row_ptr.ctypes.data_as(C.POINTER(C.c_int32)), col_idx.ctypes.data_as(C.POINTER(C.c_int32))
    _check(LIB.bpsf_sparse_layout(rp, ci, m, n, ip, None, None, None, None, None))
    if info[0] < 0:
        return None
    wmax = int(info[2])
    roff = np.zeros((m, wmax), np.uint16)
    rw = np.zeros(m, np.uint8)
    bits = np.zeros(n, np.uint32)
    cperm = np.zeros(n, np.uint16)
    rperm = np.zeros(m, np.uint16)
    _check(LIB.bpsf_sparse_layout(rp, ci, m, n, ip, *(C.c_void_p(a.ctypes.data) for a in (roff, rw, bits, cperm, rperm))))
    return {"family": int(info[0]), "cells": int(info[1]), "WMAX": wmax, "T": int(info[3]), "CPT": int(info[4]),
            "DVMAX": int(info[5]), "overflow": int(info[6]), "extra_positions": int(info[7]), "folded": int(info[8]),
            "roff": roff, "rw": rw, "bits": bits, "cperm": cperm, "rperm": rperm}


def bpsf_bp_trace(handle, syndrome, priors, params: bpsf_params):
    """Plain BP on one syndrome with every iteration's marginals and c2v messages."""
    info = bpsf_code_info(handle)
    m, n, w = info["M"], info["N"], info["row_weight"]
    dt = np.float64 if params.precision == PREC_FP64 else np.float32
    lout = np.zeros((params.max_iter, n), dt)
    c2v = np.zeros((params.max_iter, m * w), dt)
    hard = np.zeros(n, np.uint8)
    it = C.c_int32()
    conv = C.c_uint8()
    s = np.ascontiguousarray(syndrome, dtype=np.uint8)
    pri = np.ascontiguousarray(np.broadcast_to(np.asarray(priors, np.float64), (n,)))
    _check(LIB.bpsf_bp_trace(C.c_void_p(handle), s.ctypes.data_as(C.POINTER(C.c_uint8)),
                             pri.ctypes.data_as(C.POINTER(C.c_double)), C.byref(params),
                             lout.ctypes.data_as(C.c_void_p), c2v.ctypes.data_as(C.c_void_p),
                             hard.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(it), C.byref(conv)))
    k = it.value
    return {"hard": hard, "iterations": k, "converged": conv.value, "trace_lout": lout[:k], "trace_c2v": c2v[:k]}


class Decoder:
    """A loaded code plus output buffers; ``decode`` returns torch tensors."""

    def __init__(self, h, device="cuda"):
        import torch
        self.torch = torch
        self.device = device
        self.handle = bpsf_load_code(h)
        info = bpsf_code_info(self.handle)
        self.M, self.N = info["M"], info["N"]

    def decode(self, syndromes, priors, params: bpsf_params, stream=None, out=None):
        torch = self.torch
        shots = int(syndromes.shape[0])
        if out is None:
            out = (torch.empty((shots, self.N), dtype=torch.uint8, device=syndromes.device),
                   torch.empty((shots,), dtype=torch.uint8, device=syndromes.device),
                   torch.empty((shots,), dtype=torch.int32, device=syndromes.device))
        pri = np.broadcast_to(np.asarray(priors, np.float64), (self.N,))
        bpsf_decode(self.handle, syndromes, pri, params, out[0], out[1], out[2], stream)
        return out

    def stats(self, stream=None):
        return bpsf_last_stats(self.handle, stream)

    def close(self):
        if self.handle:
            bpsf_free_code(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
