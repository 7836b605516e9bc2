#!/usr/bin/env python3
"""Throughput benchmark of the BP-SF decoder on one MI355X.

Workload: the [[144,12,12]] bivariate-bicycle code (H_X, 72 x 144, 432 edges),
code-capacity i.i.d. bit flips with p = 0.03, 10^6 seeded shots resident in
HBM; min-sum with alpha = 0.625, 100 first-BP iterations, |Phi| = 6 giving 64
trial vectors of 20-iteration BP, lightest successful trial kept, float
messages. One step decodes all 10^6 shots (first BP, trial BPs, winner
re-runs). Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

EDGE_BYTES = 16          # one float v2c and one float c2v per edge, each written once and read once
LDS_SPEC_GBS = 256 * 128 * 2.4   # data-sheet figure: 256 CUs x 128 B/clk x 2.4 GHz = 78,643 GB/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4 / 1000   # 32-bit VALU lane-ops: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz

_LDS = {}


def lds_peak() -> dict:
    """The device's LDS bandwidth, measured now by the streaming probe
    (include/lds_probe.h): every read and write width at a few occupancies;
    the peak is the largest rate (ds_read_b128 on gfx950)."""
    if not _LDS:
        from paper_2507_00254_amd import lds_probe
        m = lds_probe.measure()
        rate = {(r["kind"], r["width"]): max(x["GBps"] for x in m["rows"]
                                             if (x["kind"], x["width"]) == (r["kind"], r["width"]))
                for r in m["rows"]}
        # the roof of the decoder's own access mix: one 4-byte read and one
        # 4-byte write per message, reads and writes sharing the LDS
        mix = 2.0 / (1.0 / rate[("read", 4)] + 1.0 / rate[("write", 4)])
        _LDS.update({"peak": m["peak_GBps"], "peak_at": m["peak_at"], "b32_read_write_mix": mix,
                     "rates_GBps": {f"{k}_b{8 * w}": round(v, 1) for (k, w), v in sorted(rate.items())}})
    return _LDS


def lds_roofline(kernel: str, achieved: float, per_unit: str, traffic=None) -> dict:
    """The roofline object of an LDS-bound kernel against the measured peak."""
    L = lds_peak()
    return {"bound": "lds", "kernel": kernel, "achieved": achieved, "peak": L["peak"], "unit": "GB/s",
            "frac": achieved / L["peak"], "traffic": traffic, "per_unit": per_unit,
            "peak_source": f"measured this run: {L['peak_at']['kind']} b{8 * L['peak_at']['width']} streaming "
                           f"probe (liblds_probe.so)",
            "spec_peak": LDS_SPEC_GBS, "frac_of_spec": achieved / LDS_SPEC_GBS,
            "b32_read_write_mix_peak": L["b32_read_write_mix"],
            "frac_of_b32_mix": achieved / L["b32_read_write_mix"], "probe_GBps": L["rates_GBps"]}


def valu_from_profile(phase: str, ms: float):
    """VALU lane-op rate of a phase: SQ_INSTS_VALU per dispatch from the
    committed counter summary (when it was taken on the current kernel
    source, else None) x 64 lanes over the phase's live mean duration."""
    path = os.path.join(ROOT, "profiles", "counters_bb144_p003.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_src_sha") != kernel_hash():
        return None
    insts = rec.get("phases", {}).get(phase, {}).get("SQ_INSTS_VALU")
    if not insts:
        return None
    tops = 64.0 * insts / (ms * 1e-3) / 1e12
    return {"lane_ops_per_dispatch": 64.0 * insts, "achieved_Tops": tops, "peak_Tops": VALU_PEAK_TOPS,
            "frac": tops / VALU_PEAK_TOPS, "source": "SQ_INSTS_VALU, profiles/counters_bb144_p003.json"}
KERNEL_SOURCES = ("paper_2507_00254_amd/csrc/bpsf_kernels.hip", "paper_2507_00254_amd/csrc/bpsf_tiles.h",
                  "paper_2507_00254_amd/csrc/bpsf_internal.h")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(phase: str, launches_bytes_key: str = "hbm_bytes_per_dispatch"):
    """HBM bytes per launch from a committed counter summary, when it was taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_bb144_p003.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_src_sha") != kernel_hash():
        return None
    return rec.get("phases", {}).get(phase, {}).get(launches_bytes_key)


COPY_BYTES = 1 << 30


def copy_calibration(reps: int = 3):
    """A plain device copy of known size, profiled beside the decoder to scale
    FETCH_SIZE / WRITE_SIZE into bytes."""
    import torch
    src = torch.ones(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "reps": reps}), flush=True)


def _pmc_per_dispatch(csv_path: str, counter: str):
    """Mean counter value per dispatch, by decode phase (and for the copy kernel)."""
    import csv
    acc, seen = {}, {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            kn = r["Kernel_Name"]
            if "bpsf_kernel<" in kn:
                # template arguments: Real, IC, IV, W, DV, UL, MODE, TRACE, LAY
                targs = [x.strip() for x in kn.split("bpsf_kernel<", 1)[1].split(">", 1)[0].split(",")]
                if len(targs) > 8 and targs[8] == "true":
                    continue
                ph = {"0": "main", "1": "trials", "2": "rerun"}[targs[6]]
            elif "copy" in kn.lower():
                ph = "copy"
            else:
                continue
            acc[ph] = acc.get(ph, 0.0) + float(r["Counter_Value"])
            seen.setdefault(ph, set()).add(r["Dispatch_Id"])
    return {ph: acc[ph] / len(seen[ph]) for ph in acc}


def counter_summary(csv_paths, out_path):
    """Per-dispatch mean of every counter in rocprofv3 --pmc CSVs, by decode
    phase, stamped with the kernel source hash (bench.py reads
    SQ_INSTS_VALU from it for the VALU fraction)."""
    import csv
    names = set()
    for path in csv_paths:
        with open(path) as f:
            names.update(r["Counter_Name"] for r in csv.DictReader(f))
    rec = {"kernel_src_sha": kernel_hash(), "phases": {}}
    for name in sorted(names):
        for path in csv_paths:
            per = _pmc_per_dispatch(path, name)
            for ph, v in per.items():
                if ph != "copy":
                    rec["phases"].setdefault(ph, {})[name] = v
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


def traffic_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, out_path):
    """Per-dispatch HBM bytes of every phase from two counter runs, scaled by
    what the same counters read for a plain copy of COPY_BYTES."""
    fe = _pmc_per_dispatch(fetch_csv, "FETCH_SIZE")
    wr = _pmc_per_dispatch(write_csv, "WRITE_SIZE")
    cf = _pmc_per_dispatch(copy_fetch_csv, "FETCH_SIZE")["copy"]
    cw = _pmc_per_dispatch(copy_write_csv, "WRITE_SIZE")["copy"]
    kib = COPY_BYTES / 1024.0
    f_scale, w_scale = kib / cf, kib / cw
    rec = {"kernel_src_sha": kernel_hash(), "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_scale, "write_scale": w_scale, "phases": {}}
    for ph in fe:
        if ph == "copy":
            continue
        b = (fe[ph] * f_scale + wr.get(ph, 0.0) * w_scale) * 1024.0
        rec["phases"][ph] = {"fetch_kib_per_dispatch": fe[ph], "write_kib_per_dispatch": wr.get(ph, 0.0),
                             "hbm_bytes_per_dispatch": b}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_share() -> int:
    """Threads the oracle may use: the host's CPU share for this job (the
    OMP_NUM_THREADS it sets), else the cores this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), aff)
    return aff


def cpu_baseline(h, syn, p, prm, seconds: float):
    """The double-precision oracle on the host over the first shots of the
    same workload: one thread for about a third of `seconds`, then the
    host's CPU share for the rest (static shot partition)."""
    from oracle.oracle import OracleLib
    O = OracleLib()
    share = _cpu_share()

    def leg(threads, budget):
        done, t0 = 0, time.perf_counter()
        chunk = 4000 * threads
        while time.perf_counter() - t0 < budget and done < len(syn):
            O.bpsf_batch(h, syn[done:done + chunk], p, prm, prec="f64", threads=threads)
            done += min(chunk, len(syn) - done)
        return done, time.perf_counter() - t0

    n1, t1 = leg(1, seconds / 3.0)
    n, t = leg(share, seconds * 2.0 / 3.0)
    return {"value": n / t, "unit": "shots/s", "cores": share, "kind": "oracle",
            "sample": f"first {n} shots of the same workload, double-precision oracle, {share} threads, {t:.1f} s",
            "single_thread": {"value": n1 / t1, "shots": n1, "seconds": t1},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


MIXED_NAMES = ("bb72", "bb90", "bb108", "bb144", "bb288")


def small_mixed_latency(B, hs, handles, mix, syn, sc, pri, prm, stream, calls):
    """Latency of small calls on an idle GPU (GPU events, scratch reserved up
    front, after one untimed call of each kind): a request of U{1..256} shots
    of one code alone, and two such requests of two codes in one grouped
    mixed call."""
    import torch
    if calls <= 0:
        return None
    rng = np.random.default_rng(17)
    mmax = max(h.shape[0] for h in hs)
    nmax = max(h.shape[1] for h in hs)
    rows = [np.nonzero(sc == c)[0] for c in range(len(hs))]
    g_syn = torch.zeros((512, mmax), dtype=torch.uint8, device="cuda")
    g_corr = torch.empty((512, nmax), dtype=torch.uint8, device="cuda")
    g_conv = torch.empty((512,), dtype=torch.uint8, device="cuda")
    g_it = torch.empty((512,), dtype=torch.int32, device="cuda")
    # scratch sized up front for the largest such calls: no call grows it
    for h in handles:
        B.bpsf_reserve(h, 256, prm)
    B.bpsf_mix_reserve(mix, 512, prm)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    alone, pair = [], []
    for i in range(calls + 1):
        c1, c2 = sorted(int(x) for x in rng.choice(len(hs), 2, replace=False))
        n1, n2 = (int(x) for x in rng.integers(1, 257, 2))
        s1 = torch.from_numpy(np.ascontiguousarray(syn[rows[c1][:n1], :hs[c1].shape[0]])).cuda()
        s2 = torch.from_numpy(np.ascontiguousarray(syn[rows[c2][:n2], :hs[c2].shape[0]])).cuda()
        g_syn.zero_()
        g_syn[:n1, :hs[c1].shape[0]] = s1
        g_syn[n1:n1 + n2, :hs[c2].shape[0]] = s2
        counts = np.zeros(len(hs), np.int64)
        counts[c1], counts[c2] = n1, n2
        o1 = torch.empty((n1, hs[c1].shape[1]), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        ev0.record(stream)
        B.bpsf_decode(handles[c1], s1, pri[c1], prm, o1, g_conv[:n1], g_it[:n1], stream)
        ev1.record(stream)
        ev1.synchronize()
        t_alone = ev0.elapsed_time(ev1) * 1e3
        ev0.record(stream)
        B.bpsf_mix_decode_grouped(mix, counts, g_syn[:n1 + n2], pri, prm, g_corr[:n1 + n2], g_conv[:n1 + n2],
                                  g_it[:n1 + n2], stream)
        ev1.record(stream)
        ev1.synchronize()
        if i > 0:   # the first of each kind loads its kernels
            alone.append(t_alone)
            pair.append(ev0.elapsed_time(ev1) * 1e3)
    q = lambda v, x: float(np.percentile(np.array(v), x))
    return {"calls": calls, "request_shots": "U{1..256}",
            "one_request_us": {"p50": q(alone, 50), "p99": q(alone, 99), "max": float(max(alone))},
            "two_codes_grouped_us": {"p50": q(pair, 50), "p99": q(pair, 99), "max": float(max(pair))}}


def run_mixed(args):
    """Five bivariate-bicycle codes, args.per_code shots each at p, interleaved
    by a seeded permutation, decoded by one bpsf_mix_decode per step; the same
    shots decoded by five single-code calls per step are timed beside it."""
    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import codes, shots

    p = args.p
    hs = [codes.get_code(nm).hx for nm in MIXED_NAMES]
    sc, syn, _, _ = shots.mixed_batch(hs, p, args.per_code, shots.stream_key(shots.MASTER_SEED, 3))
    n = len(sc)
    prm = B.make_params(max_iter=100, cand_max_iter=20, k=6, alpha=0.625, precision=B.PREC_FP32)
    torch.cuda.set_device(0)
    handles = [B.bpsf_load_code(h) for h in hs]
    mix = B.bpsf_mix_create(handles)
    pri = [np.full(h.shape[1], p) for h in hs]
    d_sc = torch.from_numpy(sc).cuda()
    d_syn = torch.from_numpy(syn).cuda()
    nmax = max(h.shape[1] for h in hs)
    corr = torch.empty((n, nmax), dtype=torch.uint8, device="cuda")
    conv = torch.empty((n,), dtype=torch.uint8, device="cuda")
    it = torch.empty((n,), dtype=torch.int32, device="cuda")
    # the same shots per code, contiguous, for the one-call-per-code baseline
    per = []
    for c, h in enumerate(hs):
        sel = np.nonzero(sc == c)[0]
        per.append((torch.from_numpy(np.ascontiguousarray(syn[sel, :h.shape[0]])).cuda(),
                    torch.empty((len(sel), h.shape[1]), dtype=torch.uint8, device="cuda"),
                    torch.empty((len(sel),), dtype=torch.uint8, device="cuda"),
                    torch.empty((len(sel),), dtype=torch.int32, device="cuda")))
    stream = torch.cuda.current_stream()

    def mixed_step():
        B.bpsf_mix_decode(mix, d_sc, d_syn, pri, prm, corr, conv, it, stream)

    def separate_step():
        for c in range(len(hs)):
            s_c, o1, o2, o3 = per[c]
            B.bpsf_decode(handles[c], s_c, pri[c], prm, o1, o2, o3, stream)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_sep = timed(separate_step)
    ms_mix = timed(mixed_step)
    st, bad = B.bpsf_mix_last_stats(mix, len(hs), stream)
    small = small_mixed_latency(B, hs, handles, mix, syn, sc, pri, prm, stream, args.latency_calls)
    edge_iters = 0
    for c, h in enumerate(hs):
        e = int(h.sum())
        edge_iters += e * (st[c]["main_iterations"] + st[c]["trial_iterations"] + st[c]["rerun_iterations"])
    lds_gbs = EDGE_BYTES * edge_iters / (ms_mix * 1e-3) / 1e9
    out = {
        "metric": "decoded shots/s, uneven batch of five BB codes in one persistent launch per phase",
        "value": n / (ms_mix * 1e-3), "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_mix, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded i.i.d. bit flips, s = H_X e, codes interleaved by a seeded permutation)",
        "config": {"workload": f"mixed5_p{p}_{args.per_code}x5", "codes": list(MIXED_NAMES), "shots": n, "p": p,
                   "max_iter": 100, "k": 6, "trials": 64, "trial_iter": 20, "alpha": 0.625},
        "separate_calls": {"ms_per_step": ms_sep, "value": n / (ms_sep * 1e-3)},
        "speedup_vs_separate": ms_sep / ms_mix,
        "whole_call_lds_equiv": {"achieved": lds_gbs, "peak": lds_peak()["peak"], "unit": "GB/s",
                                 "frac": lds_gbs / lds_peak()["peak"]},
        "per_code": [{"code": MIXED_NAMES[c], **st[c]} for c in range(len(hs))],
        "invalid_shots": bad,
        "small_calls": small,
    }
    B.bpsf_mix_free(mix)
    for h in handles:
        B.bpsf_free_code(h)
    print(json.dumps(out), flush=True)


def run_phen(args):
    """Phenomenological noise on [[144,12,12]] over 12 rounds (864 x 2592, one
    decode per workgroup of three waves): 10^5 shots at each of p = q = 0.002
    and 0.005, 200 first-BP iterations, k = 8 (256 trials of 30 iterations),
    float messages."""
    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import codes, shots

    torch.cuda.set_device(0)
    h = codes.phenomenological(codes.bb144().hx, 12)
    n = 100_000
    prm = B.make_params(max_iter=200, cand_max_iter=30, k=8, alpha=0.625, precision=B.PREC_FP32)
    handle = B.bpsf_load_code(h)
    edges = B.bpsf_code_info(handle)["edges"]
    stream = torch.cuda.current_stream()
    rows = []
    for p in (0.002, 0.005):
        _, syn = shots.make_shots(h, p, n, shots.stream_key(shots.MASTER_SEED, 4, h.shape[1], int(round(p * 1e5))))
        s = torch.from_numpy(syn).cuda()
        corr = torch.empty((n, h.shape[1]), dtype=torch.uint8, device="cuda")
        conv = torch.empty((n,), dtype=torch.uint8, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        pri = np.full(h.shape[1], p)
        for _ in range(args.warmup):
            B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
        torch.cuda.synchronize()
        B.bpsf_set_timing(handle, True)
        phase = {"main": 0.0, "trials": 0.0, "rerun": 0.0}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
            tm = B.bpsf_last_timing(handle)
            for k2 in phase:
                phase[k2] += tm[k2]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        B.bpsf_set_timing(handle, False)
        st = B.bpsf_last_stats(handle, stream)
        iters = {"main": st["main_iterations"], "trials": st["trial_iterations"], "rerun": st["rerun_iterations"]}
        avg = {k2: v / args.steps for k2, v in phase.items()}
        dom = max(avg, key=avg.get)
        ach = EDGE_BYTES * edges * iters[dom] / (avg[dom] * 1e-3) / 1e9
        rows.append({"p": p, "shots": n, "ms_per_step": ms, "value": n / (ms * 1e-3), "phases_ms": avg,
                     "work": {**iters, "failed_shots": st["failed_shots"], "errors": st["errors"],
                              "converged_rate": float(conv.float().mean().item())},
                     "roofline": lds_roofline(dom, ach, f"{EDGE_BYTES} B per edge-iteration x {edges} edges x "
                                                        f"{iters[dom]} iterations")})
        print(json.dumps(rows[-1]), flush=True)
    B.bpsf_free_code(handle)
    print(json.dumps({"metric": "decoded shots/s, phenomenological [[144,12,12]] over 12 rounds (864 x 2592)",
                      "unit": "shots/s", "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic (seeded i.i.d. data and measurement flips, p = q)",
                      "config": {"workload": "phen144_r12_1e5", "max_iter": 200, "k": 8, "trials": 256,
                                 "trial_iter": 30, "alpha": 0.625}, "points": rows}), flush=True)


def _timed_decodes(B, handle, s, pri, prm, corr, conv, it, stream, steps, warmup, table=None):
    """Warmup, then `steps` timed decodes with per-phase events; returns
    (ms per step, mean phase ms, stats of the last call)."""
    import torch
    for _ in range(warmup):
        B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
    torch.cuda.synchronize()
    B.bpsf_set_timing(handle, True)
    phase = {"main": 0.0, "trials": 0.0, "rerun": 0.0}
    t0 = time.perf_counter()
    for _ in range(steps):
        B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
        tm = B.bpsf_last_timing(handle)
        for k2 in phase:
            phase[k2] += tm.get(k2, 0.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    B.bpsf_set_timing(handle, False)
    st = B.bpsf_last_stats(handle, stream)
    return ms, {k2: v / steps for k2, v in phase.items()}, st


def run_dem(args):
    """Circuit-level noise on [[144,12,12]] over d = 12 rounds: the detector
    error model of the memory circuit of workloads.circuit (936 detectors x
    8,784 mechanisms), 2x10^4 shots sampled from it at each of p = 0.001,
    0.002, 0.003; adaptive alpha, 100 first-BP iterations, |Phi| = 16 with
    n_s = 5 sampled trials per weight 1..6 (30 trials of 100 iterations),
    first success kept with pruning; float messages (sparse kernel family).
    A fourth point runs p = 0.003 with |Phi| = 50 and n_s = 10 per weight
    1..10 (100 trials), a fifth [[288,12,18]] over 6 rounds at p = 0.003
    (1008 x 8928, about the size of the [[144]] model). Each point also
    times single-syndrome calls."""
    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import circuit, codes, shots, trials

    torch.cuda.set_device(0)
    c = codes.bb144()
    n = args.dem_shots
    stream = torch.cuda.current_stream()
    masks = trials.sample_trial_list(16, 6, 5, shots.stream_key(shots.MASTER_SEED, 1500))
    d_masks = torch.from_numpy(masks.view(np.int32)).cuda()
    prm = B.make_params(max_iter=100, cand_max_iter=100, k=16, cand_mode=B.TRIALS_TABLE, select_mode=1, alpha=0.0,
                        flags=B.FLAG_PRUNE, precision=B.PREC_FP32)
    # the paper's complexity-study setting as a fourth point: |Phi| = 50,
    # n_s = 10 per weight 1..10 (100 trials), p = 0.003
    masks50 = trials.sample_trial_list(50, 10, 10, shots.stream_key(shots.MASTER_SEED, 1502))
    d_masks50 = torch.from_numpy(masks50.view(np.int64)).cuda()
    prm50 = B.make_params(max_iter=100, cand_max_iter=100, k=50, cand_mode=B.TRIALS_TABLE, select_mode=1,
                          alpha=0.0, flags=B.FLAG_PRUNE, precision=B.PREC_FP32)
    rows = []
    c288 = codes.bb288()
    points = [(c, 12, 0.001, 16), (c, 12, 0.002, 16), (c, 12, 0.003, 16), (c, 12, 0.003, 50),
              (c288, 6, 0.003, 16)]
    for code, rounds, p, phi in points:
        dem = circuit.build_dem(code.hx, code.hz, rounds, p)
        salt = int(round(p * 1e5)) if code is c else 1_000_000 + int(round(p * 1e5))
        err, syn, obs = circuit.sample(dem, n, shots.stream_key(shots.MASTER_SEED, 1501, salt))
        handle = B.bpsf_load_code(dem.h)
        edges = B.bpsf_code_info(handle)["edges"]
        B.bpsf_set_trial_table(handle, d_masks if phi == 16 else d_masks50)
        s = torch.from_numpy(syn).cuda()
        corr = torch.empty((n, dem.h.shape[1]), dtype=torch.uint8, device="cuda")
        conv = torch.empty((n,), dtype=torch.uint8, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        ms, avg, st = _timed_decodes(B, handle, s, dem.priors, prm if phi == 16 else prm50, corr, conv, it, stream,
                                     args.steps, args.warmup)
        iters = {"main": st["main_iterations"], "trials": st["trial_iterations"], "rerun": st["rerun_iterations"]}
        dom = max(avg, key=avg.get)
        ach = EDGE_BYTES * edges * iters[dom] / (avg[dom] * 1e-3) / 1e9
        res = (corr.cpu().numpy() ^ err).astype(np.int64)
        fail = ((res @ dem.obs.T.astype(np.int64)) & 1).any(axis=1) | (conv.cpu().numpy() == 0)
        ler = float(fail.mean())
        # per-syndrome latency: one syndrome per call on an idle GPU (GPU
        # events around the call), the first args.dem_latency_calls shots
        lat = []
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if args.dem_latency_calls > 0:
            # one untimed call: a call this small keeps its trials' corrections,
            # and the first one sizes that buffer
            B.bpsf_decode(handle, s[:1], dem.priors, prm if phi == 16 else prm50, corr[:1], conv[:1], it[:1], stream)
            torch.cuda.synchronize()
        for i in range(min(args.dem_latency_calls, n)):
            ev0.record(stream)
            B.bpsf_decode(handle, s[i:i + 1], dem.priors, prm if phi == 16 else prm50, corr[i:i + 1], conv[i:i + 1],
                          it[i:i + 1], stream)
            ev1.record(stream)
            ev1.synchronize()
            lat.append(ev0.elapsed_time(ev1) * 1e3)
        lat = np.array(lat) if lat else np.array([np.nan])
        rows.append({"code": code.name, "rounds": rounds, "p": p, "phi": phi,
                     "trials": int(len(masks) if phi == 16 else len(masks50)),
                     "shots": n, "mechanisms": int(dem.h.shape[1]), "edges": edges,
                     "ms_per_step": ms, "value": n / (ms * 1e-3), "phases_ms": avg,
                     "mean_latency_iterations": float(it.float().mean().item()),
                     "work": {**iters, "failed_shots": st["failed_shots"], "errors": st["errors"]},
                     "ler": ler, "ler_per_round": 1.0 - (1.0 - ler) ** (1.0 / rounds),
                     "syndrome_latency_us": {"calls": int(len(lat)), "mean": float(lat.mean()),
                                             "p50": float(np.percentile(lat, 50)),
                                             "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
                     "roofline": lds_roofline(dom, ach, f"{EDGE_BYTES} B per edge-iteration x {edges} edges x "
                                                        f"{iters[dom]} iterations")})
        print(json.dumps(rows[-1]), flush=True)
        B.bpsf_free_code(handle)
    print(json.dumps({"metric": "decoded shots/s, circuit-level detector error models of [[144,12,12]] (d = 12 "
                                "rounds) and [[288,12,18]] (6 rounds)",
                      "unit": "shots/s", "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic (mechanisms sampled from a self-built detector error model)",
                      "config": {"workload": "dem144_d12_2e4", "max_iter": 100, "k": [16, 50],
                                 "trials": [int(len(masks)), int(len(masks50))], "trial_iter": 100,
                                 "alpha": "adaptive", "select": "first", "prune": True},
                      "points": rows}), flush=True)


def run_layered(args):
    """Flooding against layered BP on [[288,12,18]] (the code the paper runs
    with the layered schedule) and [[144,12,12]], code-capacity p = 0.03,
    2x10^5 shots, the headline's decoder parameters."""
    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import codes, shots

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = 200_000
    rows = []
    for name in ("bb288", "bb144"):
        code = codes.get_code(name)
        p = 0.03
        _, syn = shots.make_shots(code.hx, p, n, shots.stream_key(shots.MASTER_SEED, 7, code.n, 3000))
        handle = B.bpsf_load_code(code.hx)
        s = torch.from_numpy(syn).cuda()
        corr = torch.empty((n, code.n), dtype=torch.uint8, device="cuda")
        conv = torch.empty((n,), dtype=torch.uint8, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        for sched, flags in (("flooding", 0), ("layered", B.FLAG_LAYERED)):
            prm = B.make_params(max_iter=100, cand_max_iter=20, k=6, alpha=0.625, flags=flags,
                                precision=B.PREC_FP32)
            ms, avg, st = _timed_decodes(B, handle, s, np.full(code.n, p), prm, corr, conv, it, stream,
                                         args.steps, args.warmup)
            rows.append({"code": name, "schedule": sched, "shots": n, "ms_per_step": ms, "value": n / (ms * 1e-3),
                         "phases_ms": avg, "main_iterations_per_shot": st["main_iterations"] / n,
                         "failed_shots": st["failed_shots"], "converged_rate": float(conv.float().mean().item())})
            print(json.dumps(rows[-1]), flush=True)
        B.bpsf_free_code(handle)
    print(json.dumps({"metric": "decoded shots/s, flooding vs layered BP-SF, p = 0.03", "unit": "shots/s",
                      "n_gpus": 1, "dtype": "f32", "data": "synthetic (seeded i.i.d. bit flips)",
                      "config": {"workload": "layered_bb288_bb144_2e5"}, "points": rows}), flush=True)


def run_serve(args):
    """Open-loop serving of the five-code mix: Poisson arrivals of requests of
    U{1..256} shots of a uniformly drawn code, at each offered load, through
    the batched server and through the per-request server on the same
    requests. Latency = completion - scheduled arrival."""
    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import codes, shots

    torch.cuda.set_device(0)
    p = args.p
    hs = [codes.get_code(nm).hx for nm in MIXED_NAMES]
    pools = [shots.make_shots(h, p, 60000, shots.stream_key(shots.MASTER_SEED, 5, c))[1] for c, h in enumerate(hs)]
    handles = [B.bpsf_load_code(h) for h in hs]
    prm = B.make_params(max_iter=100, cand_max_iter=20, k=6, alpha=0.625, precision=B.PREC_FP32)
    pri = [np.full(h.shape[1], p) for h in hs]
    points = []
    for li, load in enumerate(float(x) for x in args.loads.split(",")):
        rng = np.random.default_rng(1000 + li)
        n_req = int(min(max(3000, args.min_requests), max(args.min_requests, load * 0.4 / 128.5)))
        code = rng.integers(0, len(hs), n_req).astype(np.int32)
        size = rng.integers(1, 257, n_req)
        gaps = rng.exponential(128.5 / load, n_req)
        arrival = np.cumsum(gaps) - gaps[0]
        offs = rng.integers(0, 60000 - 256, n_req)
        syns = [pools[c][o:o + n] for c, o, n in zip(code, offs, size)]
        total = int(size.sum())
        row = {"offered_shots_per_s": load, "requests": n_req, "shots": total}
        outs = {}
        for mode, batching, lanes in (("batched", True, args.lanes), ("per_request", False, 1)):
            srv = B.Server(handles, pri, prm, lanes=lanes, max_batch_shots=65536, batching=batching)
            try:
                srv.replay(arrival[:20], code[:20], syns[:20])          # warm: tables, scratch, streams
                lat, wall, out = srv.replay(arrival, code, syns)
                cnt = srv.counters()
            finally:
                srv.close()
            outs[mode] = out
            row[mode] = {"shots_per_s": total / wall, "wall_s": wall,
                         "p50_us": float(np.percentile(lat, 50) * 1e6), "p99_us": float(np.percentile(lat, 99) * 1e6),
                         "max_us": float(lat.max() * 1e6), "batches": cnt["batches"] - (20 if not batching else 0)}
        diff = sum(int((a[0] != b[0]).any(axis=1).sum() + (a[1] != b[1]).sum())
                   for a, b in zip(outs["batched"], outs["per_request"]))
        row["shots_differing_between_modes"] = diff
        row["converged_rate"] = float(np.mean(np.concatenate([o[1] for o in outs["batched"]])))
        print(json.dumps(row), flush=True)
        points.append(row)
    for h in handles:
        B.bpsf_free_code(h)
    out = {"metric": "open-loop serving of the five-code mix: throughput and latency vs offered load",
           "unit": "shots/s", "n_gpus": 1, "dtype": "f32", "lanes": args.lanes,
           "data": "synthetic (seeded i.i.d. bit flips p=%g, Poisson arrivals, request sizes U{1..256})" % p,
           "config": {"workload": "serve_mixed5", "codes": list(MIXED_NAMES), "max_batch_shots": 65536},
           "points": points}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--p", type=float, default=0.03)
    ap.add_argument("--cpu-seconds", type=float, default=18.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--workload", choices=("bb144", "mixed5", "serve", "phen", "dem", "layered"), default="bb144",
                    help="bb144: the headline workload; mixed5: five BB codes' shots interleaved in one call; "
                         "serve: open-loop request serving, batched vs per-request, over a load sweep; "
                         "phen: phenomenological [[144]] over 12 rounds; dem: circuit-level detector error "
                         "model of [[144]] over 12 rounds; layered: flooding vs layered BP")
    ap.add_argument("--dem-shots", type=int, default=20_000, help="dem: shots per error rate")
    ap.add_argument("--dem-latency-calls", type=int, default=300,
                    help="dem: single-syndrome calls timed per error rate")
    ap.add_argument("--loads", type=str, default="1e4,3e4,1e5,3e5,1e6,3e6,1e7",
                    help="serve: offered loads in shots/s")
    ap.add_argument("--lanes", type=int, default=2, help="serve: streams of the batched server")
    ap.add_argument("--min-requests", type=int, default=400, help="serve: requests per load point at least")
    ap.add_argument("--per-code", type=int, default=200_000, help="mixed5: shots of each code")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the plain copy used to scale counters")
    ap.add_argument("--traffic-summary", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                           "COPY_WRITE_CSV", "OUT_JSON"),
                    help="write the per-phase HBM traffic summary from rocprofv3 counter CSVs")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV_THEN_OUT_JSON",
                    help="write the per-phase counter summary from rocprofv3 --pmc CSVs (last argument: output)")
    args = ap.parse_args()
    if args.counter_summary:
        counter_summary(args.counter_summary[:-1], args.counter_summary[-1])
        return
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(shots shard independently across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "mixed5":
        run_mixed(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "phen":
        run_phen(args)
        return
    if args.workload == "dem":
        run_dem(args)
        return
    if args.workload == "layered":
        run_layered(args)
        return

    import torch

    from paper_2507_00254_amd import bpsf as B
    from workloads import codes, shots

    code = codes.bb144()
    p = args.p
    n = args.shots
    _, syn = shots.headline_shots(code.hx, p, n)
    pri = np.full(code.n, p)
    prm = B.make_params(max_iter=100, cand_max_iter=20, k=6, alpha=0.625, precision=B.PREC_FP32)

    torch.cuda.set_device(0)
    handle = B.bpsf_load_code(code.hx)
    edges = B.bpsf_code_info(handle)["edges"]
    s = torch.from_numpy(syn).cuda()
    corr = torch.empty((n, code.n), dtype=torch.uint8, device="cuda")
    conv = torch.empty((n,), dtype=torch.uint8, device="cuda")
    it = torch.empty((n,), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
    torch.cuda.synchronize()

    B.bpsf_set_timing(handle, True)
    phase_ms = {"main": 0.0, "trials": 0.0, "rerun": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.bpsf_decode(handle, s, pri, prm, corr, conv, it, stream)
        tm = B.bpsf_last_timing(handle)          # waits for this step's events
        for k2 in phase_ms:
            phase_ms[k2] += tm[k2]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.bpsf_set_timing(handle, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    st = B.bpsf_last_stats(handle, stream)
    conv_rate = float(conv.float().mean().item())

    # dominant kernel: the phase with the largest mean duration
    iters = {"main": st["main_iterations"], "trials": st["trial_iterations"], "rerun": st["rerun_iterations"]}
    avg_ms = {k2: v / args.steps for k2, v in phase_ms.items()}
    dom = max(avg_ms, key=avg_ms.get)
    alg_bytes = EDGE_BYTES * edges * iters[dom]
    achieved = alg_bytes / (avg_ms[dom] * 1e-3) / 1e9
    traffic = traffic_from_profile(dom)

    # request latency: 256-shot batches decoded one at a time on an idle GPU
    lat = []
    if args.latency_calls > 0:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sub = s[:256]
        o1, o2, o3 = corr[:256], conv[:256], it[:256]
        B.bpsf_decode(handle, sub, pri, prm, o1, o2, o3, stream)   # untimed: the first call of this tile
        torch.cuda.synchronize()
        for i in range(args.latency_calls):
            off = (i * 256) % (n - 256)
            sub = s[off:off + 256]
            ev0.record(stream)
            B.bpsf_decode(handle, sub, pri, prm, o1, o2, o3, stream)
            ev1.record(stream)
            ev1.synchronize()
            lat.append(ev0.elapsed_time(ev1) * 1e3)
    lat = np.array(lat) if lat else np.array([np.nan])

    out = {
        "metric": f"decoded shots/s at [[144,12,12]] p={p:g} (BP-SF); p99 decode latency (us)",
        "value": n / (ms_per_step * 1e-3),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded i.i.d. bit flips, s = H_X e)",
        "config": {"workload": "bb144_codecap_p0.03_1e6", "code": "[[144,12,12]] H_X 72x144", "shots": n, "p": p,
                   "max_iter": 100, "k": 6, "trials": 64, "trial_iter": 20, "alpha": 0.625},
        "p99_latency_us": float(np.percentile(lat, 99)),
        "latency": {"request_shots": 256, "calls": int(len(lat)), "p50_us": float(np.percentile(lat, 50)),
                    "p99_us": float(np.percentile(lat, 99)), "max_us": float(np.max(lat))},
        "phases_ms": avg_ms,
        "work": {"edges": edges, **iters, "failed_shots": st["failed_shots"], "converged_rate": conv_rate},
        "roofline": lds_roofline(dom, achieved, f"{EDGE_BYTES} B per edge-iteration x {edges} edges x "
                                                f"{iters[dom]} iterations", traffic),
        "valu": valu_from_profile(dom, avg_ms[dom]),
        "kernel_src_sha": kernel_hash(),
    }
    total_edge_iters = edges * sum(iters.values())
    out["whole_call"] = {"edge_iterations_per_s": total_edge_iters / (ms_per_step * 1e-3),
                         "lds_equiv_GBps": EDGE_BYTES * total_edge_iters / (ms_per_step * 1e-3) / 1e9}
    if not args.no_cpu_baseline:
        from oracle.oracle import Params
        oprm = Params(max_iter=100, cand_max_iter=20, k=6, alpha=0.625)
        out["cpu_baseline"] = cpu_baseline(code.hx, syn, p, oprm, args.cpu_seconds)
    B.bpsf_free_code(handle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
