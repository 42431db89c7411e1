#!/usr/bin/env python
"""Benchmark of the delayed Slater-determinant update on one MI355X.

Headline (`value`): electron moves per second of the FP32-batched delayed
update on 32 walkers of N = 4096 (plane-wave orbitals, periodic box L = 10,
acceptance ~0.99, K from the autotuner, FP64 recompute every 20 sweeps; a step
is one sweep of every walker: N proposals each, their look-ahead ratios,
Metropolis decisions and en-bloc Woodbury updates).  Beside it: moves/s vs K
at N = 4096, the FP32 batch at N = 1024 and 2048, the plain FP64 single
walker (host-driven through the C ABI, and device-driven), a short serving
run (p50/p99 sweep latency), the flush kernel against the matrix-core
roofline, and the CPU oracle timed on a bounded sample.

All inputs are seeded and synthetic.  Usage:
    python bench.py [--steps K] [--warmup W] [--quick] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BOX_L = 10.0
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6    # TFLOP/s
PEAK_HBM = 8000.0        # GB/s


# HBM bytes per launch of the flush kernel at this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE), each scaled by what the
# counter reads for a plain 1 GiB device copy (fetch x 2.000, write x 1.000).
# Valid only for the kernel sources it was taken on; null once they change.
FLUSH_TRAFFIC = {
    "kernel": "k_flush_stream32<128>",
    "bytes_per_launch": 4760582301.0,
    "sources_sha256": {
        "k_stream.hip": "1b0e820d4c5aae2cdad738b251de8c0150faec9aa187d7ba68dd5b7f12d535cc",
        "tiles.hpp": "f3151b7fba3593f0981f140fb1a6c41aaed2bd10a123f31234b57d39231b13cd",
        "dsu_internal.hpp": "4df692350565731d670465881db8c52c7c4d6713742be52dd9b383652db36350",
    },
}


def measured_traffic(kernel):
    import hashlib
    if kernel != FLUSH_TRAFFIC["kernel"]:
        return None
    csrc = os.path.join(ROOT, "paper_1708_00744_amd", "csrc")
    for f, h in FLUSH_TRAFFIC["sources_sha256"].items():
        with open(os.path.join(csrc, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    return FLUSH_TRAFFIC["bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_positions(n, walkers, spins=1, seed0=1000):
    from paper_1708_00744_amd import inputs
    return np.stack([inputs.positions(seed0 + w, w, spins * n, BOX_L).reshape(spins, n, 3) for w in range(walkers)])


def sigma_or_default(n, target, cache):
    from paper_1708_00744_amd import tune
    s = tune.sigma_for(n, target, cache)
    if s is None:
        log(f"no tuned sigma for n={n} acc={target}: tuning now (not timed)")
        s, _ = tune.tune_sigma(n, target)
    return s


def time_sweeps(b, steps, warmup, force=False):
    import torch
    b.sweep(warmup, force)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(steps, force)
    b.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


# Starts: seeded uniform positions equilibrated by FP64 sweeps with a large
# step (set-up, not timed).  Uniform-random placement puts electrons close
# together (cond(A) ~1e5 at N = 4096) where |Psi|^2 sampling keeps them
# apart; from such starts FP32 inverses drift past 1e-2 in a sweep.
BURN_SWEEPS, BURN_SIGMA = 10, 0.4
RECOMPUTE_EVERY = 20
# residual watchdog of the timed run: rows per side and determinant per sweep
RESID_SAMPLES, RESID_THRESHOLD = 16, 1e-3
DIAG_WALKERS = 16


def burn_in(n, pos, seeds, wids, sweeps=BURN_SWEEPS, sigma=BURN_SIGMA, K=128):
    """FP64 batched sweeps at step sigma from `pos`; returns the positions
    (walkers, 1, n, 3) and the acceptance."""
    from paper_1708_00744_amd import dsu
    with dsu.Batch(n, pos, seeds, wids, sigma, K, precision=dsu.FP64, box_l=BOX_L) as b:
        b.sweep(sweeps)
        acc = float(b.stats()["accepted"].sum()) / (len(seeds) * n * sweeps)
        out = np.stack([b.positions(d).reshape(1, n, 3) for d in range(len(seeds))])
    return out, acc


def headline(args, cache):
    from paper_1708_00744_amd import dsu, tune
    n, walkers = 4096, 32
    sigma = sigma_or_default(n, 0.99, cache)
    dkey = tune.delay_key(n, walkers, dsu.FP32_MIXED)
    K = int(cache["delay"].get(dkey, {}).get("best", 64))
    seeds, wids = [1000 + w for w in range(walkers)], list(range(walkers))
    t0 = time.perf_counter()
    pos, acc_burn = burn_in(n, batch_positions(n, walkers), seeds, wids)
    burn_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = dsu.Batch(n, pos, seeds, wids, sigma, 256, precision=dsu.FP32_MIXED, box_l=BOX_L,
                  recompute_every=RECOMPUTE_EVERY)
    setup_s = time.perf_counter() - t0
    b.set_sweep(BURN_SWEEPS)  # the random stream continues after the burn-in sweeps
    b.set_delay(K)
    tiles = tune.recompute_tiles_for(n, walkers, cache)
    if tiles:
        b.set_recompute_tiles(*tiles)
    b.set_residual_watchdog(RESID_SAMPLES, RESID_THRESHOLD)
    b.sweep(args.warmup)
    b.sync()
    # timed region: the K sweeps, each followed by a wait so that its own
    # duration is known (median and spread across the K sweeps); HIP events
    # bracket the flush launches only, the kernel the roofline is quoted for.
    # Every sweep includes the residual watchdog (sampled residuals of every
    # inverse, FP64 recompute of any above the threshold) and every 20th the
    # periodic FP64 recompute of all inverses.
    b.set_timing(dsu.TIMING_FLUSH)
    import torch
    b.sync()
    torch.cuda.synchronize()
    acc_before = float(b.stats()["accepted"].sum())
    wd_before = b.accuracy()["recomputes"]
    per, right, drift = [], [], []
    last_drift = b.accuracy()["drift"]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        b.sweep(1)
        b.sync()
        per.append(time.perf_counter() - t1)
        a = b.accuracy()
        right.append(float(a["residual"].max()))
        changed = a["drift"] != last_drift
        if changed.any():  # the determinants recomputed during this step
            drift.append(float(np.abs(a["drift"][changed]).max()))
            last_drift = a["drift"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = b.stats()
    cnt, ms = b.kernel_time(dsu.PHASE_FLUSH)
    moves = walkers * n * args.steps
    acc = (float(st["accepted"].sum()) - acc_before) / moves
    accuracy = {
        "residual_right_max": max(right), "residual_right_per_sweep": right,
        "residual_rows_per_sweep": RESID_SAMPLES, "watchdog_threshold": RESID_THRESHOLD,
        "watchdog_recomputes": int(b.accuracy()["recomputes"] - wd_before),
        "logdet_drift_at_recompute": max(drift) if drift else None,
        "measured": "right residual max |A A^-1 - I| after every timed sweep (residual watchdog, %d rotating rows of "
                    "every determinant, A rebuilt in FP64 from the positions, before any recompute it triggers; it "
                    "bounds the relative ratio error of a small move); log|det| drift = max over determinants of "
                    "running minus fresh at the FP64 recompute(s) in the timed region" % RESID_SAMPLES,
    }
    # per-phase split from one more sweep after the timed region, with events
    # around every launch
    b.set_timing(dsu.TIMING_ALL)
    b.sweep(1)
    b.sync()
    phases = {name: b.kernel_time(p) for name, p in (("rows", dsu.PHASE_ROWS), ("lookahead_G", dsu.PHASE_G),
                                                      ("decide", dsu.PHASE_DECIDE), ("flush", dsu.PHASE_FLUSH),
                                                      ("recompute", dsu.PHASE_RECOMPUTE))}
    b.set_timing(False)
    # flush roofline: algorithmic work of one launch = every walker's rank-K update
    avg_s = ms / cnt / 1e3
    flops = walkers * (4.0 * n * n * K + 2.0 * n * K * K)
    bytes_ = walkers * 2.0 * n * n * 4
    intensity = flops / bytes_
    if intensity > PEAK_FP32_MFMA * 1e12 / (PEAK_HBM * 1e9):
        roof = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": PEAK_HBM, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    kp = 16 if K <= 16 else 1 << math.ceil(math.log2(K))
    roof["kernel"] = ("k_flush_stream32<%d>" if kp in (32, 64, 128) else "k_flush_stream<float,%d>") % kp
    roof["traffic"] = measured_traffic(roof["kernel"])
    roof["mfma_frac"] = flops / avg_s / 1e12 / PEAK_FP32_MFMA
    roof["avg_launch_ms"] = ms / cnt
    roof["launches"] = cnt
    roof["flops_per_launch"] = flops
    roof["bytes_per_launch"] = bytes_
    per_ms = sorted(1e3 * x for x in per)
    # repeated runs of the same length (each with its share of periodic
    # recomputes and the watchdog), after the timed region: run-to-run spread
    runs = [moves / dt]
    for _ in range(args.repeats - 1):
        b.sync()
        t1 = time.perf_counter()
        b.sweep(args.steps)
        b.sync()
        runs.append(moves / (time.perf_counter() - t1))
    # ratio accuracy against the FP64 oracle at the end of a recompute interval:
    # run to the last sweep before the next periodic recompute and record that
    # sweep's ratios and decisions for the first walkers (the oracle replays
    # them from the same positions with a fresh FP64 inverse, cpu_baseline)
    done = int(b.stats()["sweeps"][0]) - BURN_SWEEPS
    to_last = (RECOMPUTE_EVERY - 1 - done % RECOMPUTE_EVERY) % RECOMPUTE_EVERY
    b.sweep(to_last)
    b.sync()
    diag = {"sweep": int(b.stats()["sweeps"][0]), "seeds": seeds[:DIAG_WALKERS], "wids": wids[:DIAG_WALKERS],
            "pos": np.stack([b.positions(d) for d in range(DIAG_WALKERS)]),
            "sweeps_since_recompute": RECOMPUTE_EVERY - 1}
    b.set_trace(1)
    b.sweep(1)
    tr = [b.trace(d) for d in range(DIAG_WALKERS)]
    b.set_trace(0)
    # both residuals of every determinant at that point (the end of the
    # interval, the largest they get before the recompute), 64 rows each
    rr, rl = b.residual(64)
    accuracy["end_of_interval"] = {"residual_right_max": float(rr.max()), "residual_left_max": float(rl.max()),
                                   "residual_left_median": float(np.median(rl)),
                                   "walkers_left_above_1e-3": int((rl > 1e-3).sum()), "rows_per_side": 64,
                                   "sweeps_since_recompute": RECOMPUTE_EVERY}
    diag["ratio"] = np.stack([x[0] for x in tr])
    diag["accepted"] = np.stack([x[1] for x in tr])
    out = {
        "moves_per_s": moves / dt, "ms_per_step": 1e3 * dt / args.steps, "K": K, "sigma": sigma,
        "sweep_ms": {"median": per_ms[len(per_ms) // 2], "min": per_ms[0], "max": per_ms[-1]},
        "runs_moves_per_s": {"runs": len(runs), "median": float(np.median(runs)), "min": float(min(runs)),
                             "max": float(max(runs)),
                             "protocol": "the timed run (value) and %d more runs of the same length after it"
                                         % (len(runs) - 1)},
        "accepted_moves_per_s": None,
        "acceptance": acc, "setup_s": setup_s,
        "burn_in": {"sweeps": BURN_SWEEPS, "sigma": BURN_SIGMA, "precision": "fp64", "acceptance": acc_burn,
                    "seconds": burn_s},
        "phase_ms_per_sweep": {k: v[1] for k, v in phases.items()},
        "phase_split_from": "one sweep after the timed region, events around every launch",
        "recompute_tiles": dict(b.recompute_tiles(), source="autotuner" if tiles else "built-in"),
        "roofline": roof, "accuracy": accuracy, "diag": diag, "batch": b,
    }
    out["accepted_moves_per_s"] = out["moves_per_s"] * acc
    return out


def k_curve(b, steps=1):
    from paper_1708_00744_amd import dsu
    res = {}
    for k in (32, 64, 128, 256):
        b.set_delay(k)
        dt = time_sweeps(b, steps, 1)
        res[str(k)] = b.walkers * b.n * steps / dt
    return res


def batched_at(n, walkers, cache, steps=2, precision=None, k_curve_ks=()):
    """Batched form at size n: moves/s at the tuned K, and optionally at other K."""
    from paper_1708_00744_amd import dsu, tune
    precision = dsu.FP32_MIXED if precision is None else precision
    sigma = sigma_or_default(n, 0.99, cache)
    K = int(cache["delay"].get(tune.delay_key(n, walkers, dsu.FP32_MIXED), {}).get("best", 64))
    pos = batch_positions(n, walkers)
    kmax = max((K,) + tuple(k_curve_ks))
    out = {"walkers": walkers, "K": K, "precision": "fp64" if precision == dsu.FP64 else "fp32_mixed"}
    with dsu.Batch(n, pos, [1000 + w for w in range(walkers)], list(range(walkers)), sigma, kmax,
                   precision=precision, box_l=BOX_L) as b:
        b.set_delay(K)
        tiles = tune.recompute_tiles_for(n, walkers, cache)
        if tiles:
            b.set_recompute_tiles(*tiles)
        dt = time_sweeps(b, steps, 1)
        out["moves_per_s"] = walkers * n * steps / dt
        if k_curve_ks:
            curve = {}
            for k in k_curve_ks:
                b.set_delay(k)
                curve[str(k)] = walkers * n / time_sweeps(b, 1, 1)
            out["k_curve_moves_per_s"] = curve
    return out


def c3_batched(cache, burn, n=512, walkers=512, K=32, sweeps=100, recompute_every=50, diag_walkers=16):
    """512 walkers x N = 512 in one batch, K = 32, FP32 with FP64 recompute
    every 50 sweeps, acceptance ~0.99, 100 sweeps, from the seeded uniform
    starts or after 2 FP64 burn-in sweeps (set-up).  Per sweep: the residual
    watchdog's sampled right residual (16 rows of every determinant); at each
    recompute the log|det| drift; at the end of each interval both residuals
    on 64 rows; and the FP32 ratios of the last sweep before the first
    recompute against the oracle's FP64 ones on the first 16 walkers."""
    import oracle
    from paper_1708_00744_amd import dsu, tune
    sigma = sigma_or_default(n, 0.99, cache)
    seeds, wids = [1000 + w for w in range(walkers)], list(range(walkers))
    pos = batch_positions(n, walkers)
    if burn:
        pos, _ = burn_in(n, pos, seeds, wids, sweeps=2)
    out = {"walkers": walkers, "n": n, "K": K, "sweeps": sweeps, "recompute_every": recompute_every,
           "burn_in_sweeps": 2 if burn else 0, "sigma": sigma}
    with dsu.Batch(n, pos, seeds, wids, sigma, K, precision=dsu.FP32_MIXED, box_l=BOX_L,
                   recompute_every=recompute_every) as b:
        if burn:
            b.set_sweep(2)
        tiles = tune.recompute_tiles_for(n, walkers, cache)
        if tiles:
            b.set_recompute_tiles(*tiles)
        b.set_residual_watchdog(16, 1e-3)
        per, right, drift, left_end = [], [], [], []
        last = b.accuracy()["drift"]
        ratio_acc = None
        for sw in range(sweeps):
            trace = sw == recompute_every - 1
            if trace:
                p_diag = np.stack([b.positions(d) for d in range(diag_walkers)])
                sweep_idx = int(b.stats()["sweeps"][0])
                b.set_trace(1)
            t1 = time.perf_counter()
            b.sweep(1)
            b.sync()
            per.append(time.perf_counter() - t1)
            a = b.accuracy()
            right.append(float(a["residual"].max()))
            changed = a["drift"] != last
            if changed.any():  # the determinants recomputed before or after this sweep
                drift.append(float(np.abs(a["drift"][changed]).max()))
                last = a["drift"]
            if sw % recompute_every == recompute_every - 1:
                rr, rl = b.residual(64)
                left_end.append({"after_sweep": sw + 1, "right_max": float(rr.max()), "left_max": float(rl.max()),
                                 "left_median": float(np.median(rl))})
            if trace:
                tr = [b.trace(d) for d in range(diag_walkers)]
                b.set_trace(0)
                kv = oracle.pw_kvectors(n)
                a_or = np.stack([oracle.pw_matrix(kv, BOX_L, p_diag[w]) for w in range(diag_walkers)])
                i_or = np.ascontiguousarray(np.stack([np.linalg.inv(x) for x in a_or]))
                r_or = np.zeros((diag_walkers, n))
                oracle.walkers_moves(n, BOX_L, seeds[:diag_walkers], wids[:diag_walkers], sigma, sweep_idx, 0, n,
                                     np.ascontiguousarray(p_diag), a_or, i_or, ratios=r_or)
                diag = {"seeds": seeds[:diag_walkers], "wids": wids[:diag_walkers], "sweep": sweep_idx,
                        "ratio": np.stack([x[0] for x in tr]), "accepted": np.stack([x[1] for x in tr]),
                        "sweeps_since_recompute": recompute_every - 1}
                ratio_acc = ratio_accuracy(diag, r_or, n, sigma)
                ratio_acc.pop("measured")
        st = b.stats()
        wd = b.accuracy()["recomputes"]
    t = sum(per)
    out.update({"moves_per_s": walkers * n * sweeps / t,
                "acceptance": float(st["accepted"].sum()) / (walkers * n * sweeps),
                "sweep_ms_median": 1e3 * sorted(per)[len(per) // 2],
                "residual_right_max_per_sweep": right, "logdet_drift_at_recompute": drift,
                "end_of_interval": left_end, "watchdog_recomputes": int(wd),
                "ratio_vs_fp64_oracle_last_sweep_before_recompute": ratio_acc})
    return out


def walker_propose(n=4096, K=128, moves=256):
    """The host-driven walker's look-ahead ratio (eq. (3)) as its own launch:
    k_walker_propose reads the stale column BT[e, :] and the k pending rows of
    U and Vg, (2k + 1) n s bytes at k pending moves (s = 4 in FP32).  An FP32
    walker of N = 4096 with K = 128, rows already on the device, every move
    accepted (so k runs 0..127 in each window).  HIP events on the walker's
    stream bracket each dsu_propose_ratio_dev (the row's conversion and the
    look-ahead kernel; the host's wait is outside them): achieved algorithmic
    bytes per second over all proposals, against HBM."""
    import torch
    from paper_1708_00744_amd import dsu, inputs
    pos = inputs.positions(2, 0, n, BOX_L)
    a0 = dsu.plane_wave_rows(n, BOX_L, pos)
    rows = dsu.plane_wave_rows(n, BOX_L, pos + 0.001 * inputs.normals(3, (n, 3)))
    dev_rows = torch.tensor(rows[:moves], dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()  # default priority; handed to the walker, events recorded on it
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(moves)]
    nbytes = 0.0
    with dsu.Walker(a0, K, precision=dsu.FP32_MIXED, policy=dsu.FLUSH_K_ACCEPTED, stream=st) as w:
        for e in range(8):  # warm-up
            w.propose_dev(e, dev_rows[e].data_ptr())
            w.reject()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(moves):
            k = w.pending()
            ev[e][0].record(st)
            w.propose_dev(e, dev_rows[e].data_ptr())
            ev[e][1].record(st)
            w.accept()
            nbytes += (2 * k + 1) * n * 4.0
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    gpu_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    return {"kernel": "k_walker_propose<float>", "n": n, "K": K, "proposals": moves,
            "algorithmic_bytes": nbytes, "gpu_ms_per_proposal": 1e3 * gpu_s / moves,
            "achieved_GBps": nbytes / gpu_s / 1e9, "frac_of_hbm_peak": nbytes / gpu_s / 1e9 / PEAK_HBM,
            "wall_moves_per_s": moves / wall,
            "note": "one walker's look-ahead reads at most (2K - 1) n s = 4.2 MB: a few microseconds of launch and "
                    "reduction latency, not bandwidth, bound it; the batched form forms the same products inside "
                    "the flush pass (no separate read of BT)"}


def c2_k_study(cache, n=1024, ks=(1, 4, 16, 32, 64, 128), device_sweeps=10, host_sweeps=1):
    """One FP64 walker of N = 1024: moves/s against the delay K at acceptance
    0.99 and 0.5 (sigma from the tuner) and with every move accepted (the
    paper's test regime), driven on the device (a batch of one walker: K
    proposals per window, decisions on the device, 10 sweeps) and from the
    host through the C ABI (one propose/accept call per move, K accepted moves
    per flush, one sweep), the latter with the flush on the vector ALUs and on
    the matrix cores (the crossover of the two flush kernels)."""
    from paper_1708_00744_amd import dsu, inputs
    pos0 = inputs.positions(2, 0, n, BOX_L)
    a0 = dsu.plane_wave_rows(n, BOX_L, pos0)
    out = {"n": n, "K": list(ks), "device_sweeps": device_sweeps, "host_sweeps": host_sweeps}
    for label, target in (("acc0.99", 0.99), ("acc0.5", 0.5), ("force_accept", None)):
        sigma = sigma_or_default(n, target, cache) if target else sigma_or_default(n, 0.99, cache)
        force = target is None
        dev, acc = {}, {}
        for K in ks:
            with dsu.Batch(n, pos0[None], [2], [0], sigma, K, precision=dsu.FP64, box_l=BOX_L) as b:
                dt = time_sweeps(b, device_sweeps, 1, force)
                acc[str(K)] = float(b.stats()["accepted"][0]) / (n * (device_sweeps + 1))
            dev[str(K)] = n * device_sweeps / dt
        host = {}
        g = inputs.normals(3, (host_sweeps, n, 3))
        us = inputs.uniforms(4, host_sweeps * n)
        for mode, mname in ((dsu.FLUSH_VALU, "valu"), (dsu.FLUSH_MFMA, "mfma")):
            curve = {}
            for K in ks:
                if mode == dsu.FLUSH_VALU and K > 64:
                    continue
                pos = pos0.copy()
                with dsu.Walker(a0, K, precision=dsu.FP64, policy=dsu.FLUSH_K_ACCEPTED) as w:
                    w.set_flush_kernel(mode)
                    t0 = time.perf_counter()
                    for sw in range(host_sweeps):
                        prop = pos + sigma * g[sw]
                        rows = dsu.plane_wave_rows(n, BOX_L, prop)
                        for e in range(n):
                            r = w.propose(e, rows[e])
                            if force or us[sw * n + e] < r * r:
                                w.accept()
                                pos[e] = prop[e]
                            else:
                                w.reject()
                    w.flush()
                    curve[str(K)] = n * host_sweeps / (time.perf_counter() - t0)
            host[mname] = curve
        out[label] = {"sigma": sigma, "device_driven_moves_per_s": dev, "device_acceptance": acc,
                      "host_driven_moves_per_s": host}
    return out


def drift_single_walker(n=1024, moves=1024, tau=0.002):
    """Host-driven drift-diffusion (DMC-style) moves in FP64: per move the
    drift at the present position (dsu_eval_grad), R and grad R at the
    proposed one (dsu_propose_ratio_grad), accept with the Green's-function
    ratio.  The caller evaluates the plane-wave rows and their gradients with
    numpy; `library_us_per_move` counts only the library calls."""
    from paper_1708_00744_amd import dsu, inputs
    kv = dsu.plane_wave_table(n).astype(np.float64)
    kind = kv[:, 3]
    g2 = 2 * np.pi / BOX_L

    def rows(r):
        ph = g2 * (kv[:, :3] @ r)
        c, s = np.cos(ph), np.sin(ph)
        row = np.where(kind == 0, 1.0, np.where(kind == 1, c, s))
        d = np.where(kind == 1, -s, np.where(kind == 2, c, 0.0))
        return row, (g2 * kv[:, :3].T) * d

    pos = inputs.positions(2, 0, n, BOX_L)
    a0 = dsu.plane_wave_rows(n, BOX_L, pos)
    chi = inputs.normals(5, (moves, 3))
    us = inputs.uniforms(6, moves)
    res = {"n": n, "tau": tau, "moves": moves}
    for K in (1, 64):
        p = pos.copy()
        acc, t_lib = 0, 0.0
        with dsu.Walker(a0, K, precision=dsu.FP64, policy=dsu.FLUSH_K_ACCEPTED) as w:
            t0 = time.perf_counter()
            for m in range(moves):
                e = m % n
                _, d_old = rows(p[e])
                t1 = time.perf_counter()
                v_old = w.grad(e, d_old)
                t_lib += time.perf_counter() - t1
                rp = p[e] + tau * v_old + np.sqrt(tau) * chi[m]
                row, drow = rows(rp)
                t1 = time.perf_counter()
                r, g = w.propose_grad(e, row, drow)
                t_lib += time.perf_counter() - t1
                v_new = g / r
                log_g = (np.sum((rp - p[e] - tau * v_old) ** 2) - np.sum((p[e] - rp - tau * v_new) ** 2)) / (2 * tau)
                t1 = time.perf_counter()
                if us[m] < r * r * np.exp(log_g):
                    w.accept()
                    p[e] = rp
                    acc += 1
                else:
                    w.reject()
                t_lib += time.perf_counter() - t1
            w.flush()
            dt = time.perf_counter() - t0
        res[f"K{K}_moves_per_s"] = moves / dt
        res[f"K{K}_library_us_per_move"] = 1e6 * t_lib / moves
        res[f"K{K}_acceptance"] = acc / moves
    return res


def complex_single_walker(n=1024, sigma=0.02, sweeps=1):
    """Complex orbitals (twisted plane waves, FP64 complex), host-driven through
    the C ABI: one propose/accept call per move.  The caller evaluates the
    orbital rows with numpy (a sweep's proposals do not depend on its
    decisions, so they are evaluated before the timed loop).  Also the time of
    one fresh inverse (Gauss-Jordan, log|det| and phase)."""
    from paper_1708_00744_amd import dsu, inputs
    theta = np.array([0.31, -0.17, 0.42])
    g = np.arange(-12, 13)
    cube = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    k2 = ((cube + theta) ** 2).sum(1)
    kv = cube[np.lexsort((cube[:, 2], cube[:, 1], cube[:, 0], k2))[:n]] + theta

    def rows(p):
        return np.exp(2j * np.pi / BOX_L * (p @ kv.T))

    pos0 = inputs.positions(2, 0, n, BOX_L)
    a0 = rows(pos0)
    res = {"n": n, "sigma": sigma}
    for K in (1, 16, 64):
        pos = pos0.copy()
        gs = inputs.normals(3, (sweeps, n, 3))
        us = inputs.uniforms(4, sweeps * n)
        with dsu.ZWalker(a0, K, policy=dsu.FLUSH_K_ACCEPTED) as w:
            t_rec = time.perf_counter()
            w.recompute()
            t_rec = time.perf_counter() - t_rec
            t0 = time.perf_counter()
            acc = 0
            for s in range(sweeps):
                prop = pos + sigma * gs[s]
                rws = rows(prop)
                for e in range(n):
                    r = w.propose(e, rws[e])
                    if us[s * n + e] < abs(r) ** 2:
                        w.accept()
                        pos[e] = prop[e]
                        acc += 1
                    else:
                        w.reject()
            w.flush()
            dt = time.perf_counter() - t0
        res[f"host_driven_K{K}_moves_per_s"] = n * sweeps / dt
        res[f"K{K}_acceptance"] = acc / (n * sweeps)
        res["recompute_s"] = t_rec
    return res


def md_expansion(n, m, nocc=8):
    """Reference, all singles from the top `nocc` occupied orbitals into the m
    virtual ones, and doubles from pairs of them into pairs of virtual ones."""
    top = list(range(n - nocc, n))
    dets = [(1.0, [])]
    for a, j in enumerate(top):
        for v in range(m):
            dets.append((0.1 / (1 + a + v), [(j, v)]))
    for a in range(0, nocc - 1, 2):
        for v in range(0, m - 1, 2):
            dets.append((0.02 / (1 + a + v), [(top[a], v), (top[a + 1], v + 1)]))
    return dets


def multidet_single_walker(n=1024, m=16, sigma=0.002):
    """Multideterminant expansion on a single reference (FP64, host-driven):
    one dsu_propose_ratio_md / accept per move over one sweep, plane waves (the
    n lowest occupied, the next m virtual), caller-side rows (numpy)."""
    from paper_1708_00744_amd import dsu, inputs
    kv = dsu.plane_wave_table(n + m).astype(np.float64)
    kind, g2 = kv[:, 3], 2 * np.pi / BOX_L

    def rows(p):
        ph = g2 * (p @ kv[:, :3].T)
        return np.where(kind == 0, 1.0, np.where(kind == 1, np.cos(ph), np.sin(ph)))

    dets = md_expansion(n, m)
    pos0 = inputs.positions(2, 0, n, BOX_L)
    full = rows(pos0)
    res = {"n": n, "m": m, "determinants": len(dets), "sigma": sigma}
    for K in (1, 64):
        pos = pos0.copy()
        gs, us = inputs.normals(3, (n, 3)), inputs.uniforms(4, n)
        with dsu.Walker(np.ascontiguousarray(full[:, :n]), K, precision=dsu.FP64) as w:
            w.set_multidet(np.ascontiguousarray(full[:, n:]), dets)
            prop = pos + sigma * gs
            rp = rows(prop)
            acc = 0
            t0 = time.perf_counter()
            for e in range(n):
                r, _ = w.propose_md(e, rp[e, :n], rp[e, n:])
                if us[e] < r * r:
                    w.accept()
                    pos[e] = prop[e]
                    acc += 1
                else:
                    w.reject()
            w.flush()
            dt = time.perf_counter() - t0
        res[f"host_driven_K{K}_moves_per_s"] = n / dt
        res[f"K{K}_acceptance"] = acc / n
    return res


def serving_requests(cache, count, seed, arrival_rate=None):
    from paper_1708_00744_amd import inputs
    sizes, accs, seeds = inputs.serving_mix(seed, count)
    arr = inputs.poisson_arrivals(seed, count, rate_per_s=arrival_rate) if arrival_rate else np.zeros(count)
    reqs = []
    for i in range(count):
        n = int(sizes[i])
        reqs.append({"request_id": i, "n": n, "spins": 2, "seed": int(seeds[i]),
                     "sigma": sigma_or_default(n, float(accs[i]), cache), "sweeps": 20, "arrival_s": float(arr[i]),
                     "positions": inputs.positions(int(seeds[i]), i, 2 * n, BOX_L)})
    return reqs


def serve(reqs, budget, K=64):
    from paper_1708_00744_amd import dsu
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=BOX_L, budget_bytes=budget, recompute_every=10) as srv:
        t0 = time.perf_counter()
        results, lat = srv.run(reqs)
        wall = time.perf_counter() - t0
    return results, lat, wall


def serving(cache, count=200, seed=7, budget=8 << 30, load=0.8):
    """Poisson stream of walker requests (N from {128, ..., 2048}, two spins,
    target acceptance 0.5-0.99, 20 sweeps each, FP32 with an FP64 recompute
    every 10 sweeps) into a pool with an 8 GiB budget.  The arrival rate is
    `load` times the capacity measured first: the completion rate of the same
    kind of requests all waiting at time zero (a closed, saturated pool)."""
    cal = serving_requests(cache, 60, seed + 1000)
    results, _, wall = serve(cal, budget)
    capacity = sum(r["status"] == 0 for r in results) / wall
    rate = load * capacity
    reqs = serving_requests(cache, count, seed, arrival_rate=rate)
    results, lat, wall = serve(reqs, budget)
    ok = [(q, r) for q, r in zip(reqs, results) if r["status"] == 0]
    moves = sum(2 * q["n"] * q["sweeps"] for q, _ in ok)
    e2e = [r["finish_s"] - q["arrival_s"] for q, r in ok]
    wait = [r["admit_s"] - q["arrival_s"] for q, r in ok]
    return {"requests": count, "completed": len(ok), "budget_bytes": budget,
            "capacity_requests_per_s": capacity, "arrival_rate_per_s": rate, "load": load, "wall_s": wall,
            "moves_per_s": moves / wall,
            "sweep_latency_ms_p50": float(np.percentile(lat, 50)), "sweep_latency_ms_p99": float(np.percentile(lat, 99)),
            "queue_wait_s_p50": float(np.percentile(wait, 50)), "queue_wait_s_p99": float(np.percentile(wait, 99)),
            "end_to_end_s_p50": float(np.percentile(e2e, 50)), "end_to_end_s_p99": float(np.percentile(e2e, 99))}


def ratio_accuracy(diag, r_or, upto, sigma):
    """FP32 device ratios against the oracle's FP64 ones for the first `upto`
    moves of each walker's traced sweep, up to and including the first move
    whose decision differs (after it the two trajectories part)."""
    import oracle
    errs, flips, compared = [], 0, 0
    for w in range(r_or.shape[0]):
        rg, ag = diag["ratio"][w][:upto], diag["accepted"][w][:upto].astype(bool)
        stop = upto
        for e in range(upto):
            _, u = oracle.move_randoms(diag["seeds"][w], diag["wids"][w], diag["sweep"], e)
            if (u < r_or[w, e] ** 2) != ag[e]:
                stop = e + 1
                flips += 1
                break
        ro = r_or[w, :stop]
        errs.append(np.abs(rg[:stop] - ro) / np.maximum(np.abs(ro), 1e-3))
        compared += stop
    e = np.concatenate(errs)
    return {"moves_compared": int(compared), "median": float(np.median(e)), "p99": float(np.percentile(e, 99)),
            "max": float(e.max()), "decision_flips": flips,
            "measured": "relative error |R - R_fp64| / max(|R_fp64|, 1e-3) of the device's FP32 ratios against the "
                        "oracle's (FP64 Sherman-Morrison from a fresh inverse at the same positions) on the last sweep "
                        "before a periodic recompute (%d sweeps since the last), each walker compared up to its first "
                        "differing decision" % diag["sweeps_since_recompute"]}


def cpu_baseline(diag, sigma, n=4096, target_s=15.0):
    """The oracle (plain FP64 Sherman-Morrison in C) on the host cores: a
    bounded sample of the headline workload -- one thread per walker, each
    running the first moves of the sweep the headline traced, from the same
    positions with a fresh inverse (set-up by LAPACK, not timed).  Its ratios
    double as the FP64 reference of the device's FP32 ones."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, len(diag["seeds"])))
    walkers = threads
    seeds, wids, sweep = diag["seeds"][:walkers], diag["wids"][:walkers], diag["sweep"]
    kv = oracle.pw_kvectors(n)
    pos = np.ascontiguousarray(diag["pos"][:walkers])
    a = np.stack([oracle.pw_matrix(kv, BOX_L, pos[w]) for w in range(walkers)])
    ainv = np.ascontiguousarray(np.stack([np.linalg.inv(a[w]) for w in range(walkers)]))
    # calibrate the sample size with 4 moves
    r0 = np.zeros((walkers, 4))
    t0 = time.perf_counter()
    oracle.walkers_moves(n, BOX_L, seeds, wids, sigma, sweep, 0, 4, pos, a, ainv, ratios=r0)
    per = (time.perf_counter() - t0) / 4
    m = min(max(8, int(target_s / max(per, 1e-6))), n - 4 - 24)
    r1 = np.zeros((walkers, m))
    t0 = time.perf_counter()
    _, used = oracle.walkers_moves(n, BOX_L, seeds, wids, sigma, sweep, 4, m, pos, a, ainv, ratios=r1)
    dt = time.perf_counter() - t0
    ratio_acc = ratio_accuracy(diag, np.concatenate([r0, r1], axis=1), 4 + m, sigma)
    # one thread, one walker: the next 24 moves of walker 0
    t1 = time.perf_counter()
    e1 = 4 + m
    oracle.walkers_moves(n, BOX_L, seeds[:1], wids[:1], sigma, sweep, e1, 24, pos[:1].copy(), a[:1].copy(),
                         ainv[:1].copy())
    single = 24 / (time.perf_counter() - t1)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": walkers * m / dt, "unit": "moves/s", "cores": int(used), "kind": "oracle",
            "sample": f"{walkers} walkers x {m} moves of one sweep at N={n} from the headline's positions (FP64 "
                      f"Sherman-Morrison, one OpenMP thread per walker, set-up by LAPACK inverse not timed)",
            "single_thread_moves_per_s": single,
            "host": {"nproc": os.cpu_count(), "cpu": model},
            "walker_forms": cpu_baseline_walkers()}, ratio_acc


def cpu_baseline_walkers(n=1024, moves=100):
    """The oracle on the two host-driven walker workloads of the extras (one
    thread, first `moves` moves from a fresh inverse, set-up not timed)."""
    import oracle
    from paper_1708_00744_amd import inputs
    out = {}
    # drift-diffusion: drift at the present position, ratio and gradient at the proposal, Sherman-Morrison
    kv = oracle.pw_kvectors(n)
    pos = inputs.positions(2, 0, n, BOX_L)
    a = oracle.pw_matrix(kv, BOX_L, pos)
    ainv, _, _ = oracle.inverse(a)
    chi, us, tau = inputs.normals(5, (moves, 3)), inputs.uniforms(6, moves), 0.002
    t0 = time.perf_counter()
    for m in range(moves):
        e = m % n
        _, v_old = oracle.sm_ratio_grad(ainv, e, a[e], oracle.pw_row_grad(kv, BOX_L, pos[e]))
        rp = pos[e] + tau * v_old + np.sqrt(tau) * chi[m]
        row = oracle.pw_row(kv, BOX_L, rp)
        r, g = oracle.sm_ratio_grad(ainv, e, row, oracle.pw_row_grad(kv, BOX_L, rp))
        log_g = (np.sum((rp - pos[e] - tau * v_old) ** 2) - np.sum((pos[e] - rp - tau * g / r) ** 2)) / (2 * tau)
        if us[m] < r * r * np.exp(log_g):
            oracle.sm_accept(ainv, a, e, row, r)
            pos[e] = rp
    out["fp64_drift_walker_n1024"] = {"moves_per_s": moves / (time.perf_counter() - t0), "cores": 1,
                                      "sample": f"{moves} drift-diffusion moves at N={n}"}
    # complex orbitals: twisted plane waves, complex Sherman-Morrison
    theta = np.array([0.31, -0.17, 0.42])
    kz = oracle.zpw_kvectors(n, theta)
    pos = inputs.positions(2, 0, n, BOX_L)
    az = oracle.zpw_matrix(kz, theta, BOX_L, pos)
    azinv, _, _ = oracle.zinverse(az)
    gs, us = inputs.normals(3, (1, n, 3))[0], inputs.uniforms(4, n)
    t0 = time.perf_counter()
    for e in range(moves):
        rt = pos[e] + 0.02 * gs[e]
        row = oracle.zpw_row(kz, theta, BOX_L, rt)
        r = oracle.zsm_ratio(azinv, e, row)
        if us[e] < abs(r) ** 2:
            oracle.zsm_accept(azinv, az, e, row, r)
            pos[e] = rt
    out["complex_single_walker_n1024"] = {"moves_per_s": moves / (time.perf_counter() - t0), "cores": 1,
                                          "sample": f"{moves} moves of the first sweep at N={n}"}
    # multideterminant: Psi by definition (one LU per determinant) before and after each move
    m, nmd, md_moves = 16, 256, 4
    kv = oracle.pw_kvectors(nmd + m)
    pos = inputs.positions(2, 0, nmd, BOX_L)
    full = np.stack([oracle.pw_row(kv, BOX_L, p) for p in pos])
    a, v = np.ascontiguousarray(full[:, :nmd]), np.ascontiguousarray(full[:, nmd:])
    dets = md_expansion(nmd, m)
    t0 = time.perf_counter()
    for e in range(md_moves):
        row = oracle.pw_row(kv, BOX_L, pos[e] + 0.002 * np.ones(3))
        oracle.md_ratio(a, v, dets, e, row[:nmd], row[nmd:])
    out["multidet_single_walker"] = {"moves_per_s": md_moves / (time.perf_counter() - t0), "cores": 1,
                                     "sample": f"{md_moves} ratios at N={nmd}, m={m}, {len(dets)} determinants "
                                               f"(the extras leg runs N=1024)"}
    return out


def _cache():
    from paper_1708_00744_amd import tune
    return tune.load_cache()


EXTRA_LEGS = {
    "walker_propose_n4096": lambda: walker_propose(),
    "serving": lambda: serving(_cache()),
    "c2_k_study_n1024": lambda: c2_k_study(_cache()),
    "c3_n512_w512": lambda: c3_batched(_cache(), burn=False),
    "c3_n512_w512_burn_in": lambda: c3_batched(_cache(), burn=True),
    "complex_single_walker_n1024": lambda: complex_single_walker(),
    "multidet_single_walker_n1024": lambda: multidet_single_walker(),
    "fp64_drift_walker_n1024": lambda: drift_single_walker(),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--repeats", type=int, default=5,
                    help="runs of --steps sweeps for the run-to-run spread (the first is the timed one)")
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", default=None, choices=sorted(EXTRA_LEGS),
                    help="run one single-walker leg of the extras alone and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 3}))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: walkers shard across GPUs with no communication, "
                                   "so only --gpus 1 is supported"}))
        return 2
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        return 1
    torch.cuda.set_device(0)
    if args.extra:
        print(json.dumps({args.extra: EXTRA_LEGS[args.extra]()}))
        return 0
    from paper_1708_00744_amd import dsu, tune
    dsu.lib()
    cache = tune.load_cache()
    log("headline: 32 walkers, N=4096, FP32 batched")
    h = headline(args, cache)
    b = h.pop("batch")
    extras = {}
    if not args.quick:
        log("K curve")
        extras["k_curve_n4096_moves_per_s"] = k_curve(b)
        log("host-driven look-ahead ratio kernel, N=4096 FP32")
        extras["walker_propose_n4096"] = walker_propose()
    b.close()
    if not args.quick:
        log("512 walkers x N=512, 100 sweeps, with and without FP64 burn-in")
        extras["c3_n512_w512"] = c3_batched(cache, burn=False)
        extras["c3_n512_w512_burn_in"] = c3_batched(cache, burn=True)
        log("batched N=1024 / 2048, FP32 and FP64")
        extras["fp32_batched_n1024"] = batched_at(1024, 256, cache, k_curve_ks=(16, 32, 128))
        extras["fp32_batched_n2048"] = batched_at(2048, 64, cache, k_curve_ks=(16, 32, 128))
        extras["fp64_batched_n1024"] = batched_at(1024, 256, cache, precision=dsu.FP64)
        extras["fp64_batched_n2048"] = batched_at(2048, 64, cache, precision=dsu.FP64)
        extras["fp64_batched_n4096"] = batched_at(4096, 32, cache, precision=dsu.FP64)
        log("FP64 single walker N=1024: K study at acceptance 0.99, 0.5 and 1, VALU/MFMA flush")
        extras["c2_k_study_n1024"] = c2_k_study(cache)
        log("complex-orbital walker N=1024")
        extras["complex_single_walker_n1024"] = complex_single_walker()
        log("multideterminant walker N=1024")
        extras["multidet_single_walker_n1024"] = multidet_single_walker()
        log("FP64 drift-diffusion walker N=1024")
        extras["fp64_drift_walker_n1024"] = drift_single_walker()
        log("serving")
        extras["serving"] = serving(cache)
    cpu = None
    diag = h.pop("diag")
    accuracy = h.pop("accuracy")
    if not args.no_cpu:
        log("cpu baseline (oracle), ratio accuracy against it")
        cpu, accuracy["ratio_vs_fp64_oracle"] = cpu_baseline(diag, h["sigma"])
    roof = h.pop("roofline")
    line = {
        "metric": "electron moves/sec/GPU (FP32-batched delayed update, N=4096)",
        "value": h["moves_per_s"],
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 recompute and log-det)",
        "data": "synthetic: seeded uniform positions equilibrated by %d FP64 sweeps at sigma %.1f (set-up, not "
                "timed), plane-wave orbitals, device Philox4x64-10 moves" % (BURN_SWEEPS, BURN_SIGMA),
        "config": {"workload": "32 walkers x N=4096 Slater matrices, K=%d, acceptance %.3f, FP64 recompute every %d "
                               "sweeps, residual watchdog every sweep; step = one sweep of every walker"
                               % (h["K"], h["acceptance"], RECOMPUTE_EVERY),
                   "walkers": 32, "n": 4096, "K": h["K"], "sigma": h["sigma"], "precision": "fp32_mixed",
                   "recompute_every": RECOMPUTE_EVERY},
        "roofline": roof,
        "accuracy": accuracy,
        "cpu_baseline": cpu,
        "detail": {k: v for k, v in h.items() if k not in ("moves_per_s", "ms_per_step")},
        "extras": extras,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
