"""Autotuning of the batched form through the C ABI.

* tune_sigma: Gaussian step sigma that gives a target acceptance for a matrix
  size (bisection on log sigma; acceptance falls monotonically with sigma).
* tune_delay: the delay K with the highest moves/s for a workload (Sec. III:
  the best K depends on the architecture and the matrix size, and the paper
  suggests leaving its choice to an autotuner).
* tune_recompute: the blocking of the FP64 recompute (panel width, update
  chunk, apply columns per workgroup) with the shortest recompute.

Results are cached in tuning.json next to this file, keyed by workload.
Run `python -m paper_1708_00744_amd.tune` on the GPU to fill the cache.
"""
import json
import math
import os
import sys
import time

import numpy as np

from . import dsu, inputs

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
BOX_L = 10.0


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {"sigma": {}, "delay": {}}


def save_cache(c, path=CACHE):
    with open(path, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)


def sigma_key(n, target):
    return f"n={n}/acc={target:.3f}"


def delay_key(n, walkers, precision):
    return f"n={n}/w={walkers}/prec={'fp64' if precision == dsu.FP64 else 'fp32'}"


def measure_acceptance(n, sigma, walkers=2, sweeps=1, k_delay=32, precision=dsu.FP32_MIXED, seed=9):
    pos = np.stack([inputs.positions(seed, w, n, BOX_L) for w in range(walkers)])
    with dsu.Batch(n, pos, [seed] * walkers, list(range(walkers)), sigma, min(k_delay, n), precision=precision,
                   box_l=BOX_L) as b:
        b.sweep(sweeps)
        st = b.stats()
    return float(st["accepted"].sum()) / (walkers * n * sweeps)


def tune_sigma(n, target, walkers=2, iters=12, tol=0.004):
    lo, hi = math.log(1e-5 * BOX_L), math.log(0.5 * BOX_L)
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        acc = measure_acceptance(n, math.exp(mid), walkers=walkers)
        best = (math.exp(mid), acc)
        if abs(acc - target) <= tol:
            break
        if acc > target:
            lo = mid
        else:
            hi = mid
    return best


def sigma_for(n, target, cache=None):
    """Cached sigma for (n, target); otherwise interpolate the cached points
    of the same n in (acceptance, log sigma); None if nothing is cached."""
    c = cache or load_cache()
    key = sigma_key(n, target)
    if key in c["sigma"]:
        return c["sigma"][key]["sigma"]
    pts = sorted((v["acc"], math.log(v["sigma"])) for k, v in c["sigma"].items() if k.startswith(f"n={n}/"))
    if len(pts) < 2:
        return None
    accs = [p[0] for p in pts]
    logs = [p[1] for p in pts]
    return float(math.exp(np.interp(target, accs, logs)))


def tune_delay(n, walkers, sigma, candidates=(32, 64, 128, 256), precision=dsu.FP32_MIXED, sweeps=1, seed=1000):
    pos = np.stack([inputs.positions(seed + w, w, n, BOX_L) for w in range(walkers)])
    out = {}
    with dsu.Batch(n, pos, [seed + w for w in range(walkers)], list(range(walkers)), sigma, max(candidates),
                   precision=precision, box_l=BOX_L) as b:
        for k in candidates:
            b.set_delay(k)
            b.sweep(1)
            b.sync()
            t0 = time.perf_counter()
            b.sweep(sweeps)
            b.sync()
            dt = time.perf_counter() - t0
            out[k] = walkers * n * sweeps / dt
    best = max(out, key=out.get)
    return best, out


def recompute_key(n, walkers, precision):
    return f"n={n},walkers={walkers},prec={precision}"


def recompute_candidates(n):
    """Blockings of the FP64 recompute worth timing at this n: panel width
    (128 = pairs of 64-column panels sharing one trailing update, from n = 256
    while the padded size is at most 4096), update chunk (64 only where the
    padded size is a multiple of 128) and apply columns per workgroup."""
    np_ = -(-n // 64) * 64
    if n < 64:
        panels = (16, 32)
    elif n >= 256 and np_ <= 4096:
        panels = (32, 64, 128)
    else:
        panels = (32, 64)
    chunks = (32, 64) if np_ % 128 == 0 else (32,)
    return [(p, c, a) for p in panels for c in chunks for a in (1, 4)]


def tune_recompute(n, walkers, precision=dsu.FP32_MIXED, reps=2, seed=1000):
    """Time the batch's FP64 recompute for every candidate blocking; returns the
    fastest and the seconds per recompute of each."""
    pos = np.stack([inputs.positions(seed + w, w, n, BOX_L) for w in range(walkers)])
    out = {}
    with dsu.Batch(n, pos, [seed + w for w in range(walkers)], list(range(walkers)), 0.001, 32,
                   precision=precision, box_l=BOX_L) as b:
        for cand in recompute_candidates(n):
            b.set_recompute_tiles(*cand)
            b.recompute()
            t0 = time.perf_counter()
            for _ in range(reps):
                b.recompute()
            out[cand] = (time.perf_counter() - t0) / reps
    best = min(out, key=out.get)
    return best, out


def recompute_tiles_for(n, walkers, cache=None, precision=dsu.FP32_MIXED):
    c = cache if cache is not None else load_cache()
    e = c.get("recompute", {}).get(recompute_key(n, walkers, precision))
    return tuple(e["best"]) if e else None


def main(argv):
    import torch
    torch.cuda.set_device(0)
    c = load_cache()
    out_path = CACHE
    recompute_only = "--recompute-only" in argv
    delay_only = "--delay-only" in argv or recompute_only
    for a in argv:
        if a.startswith("--out="):
            out_path = a.split("=", 1)[1]
    for n in () if delay_only else (64, 128, 256, 512, 1024, 2048, 4096):
        targets = (0.5, 0.75, 0.9, 0.99) if n <= 2048 else (0.99,)
        for t in targets:
            s, acc = tune_sigma(n, t, walkers=2 if n >= 2048 else 4)
            c["sigma"][sigma_key(n, t)] = {"sigma": s, "acc": acc}
            print(f"sigma n={n} target={t}: sigma={s:.5g} acc={acc:.4f}", flush=True)
        save_cache(c, out_path)
    for n, w in ((4096, 32), (2048, 64), (1024, 256), (512, 512)):
        if not recompute_only:
            s = sigma_for(n, 0.99, c)
            best, rates = tune_delay(n, w, s)
            c["delay"][delay_key(n, w, dsu.FP32_MIXED)] = {"best": best,
                                                           "moves_per_s": {str(k): v for k, v in rates.items()}}
            print(f"delay n={n} walkers={w}: best K={best} {rates}", flush=True)
        best, secs = tune_recompute(n, w)
        c.setdefault("recompute", {})[recompute_key(n, w, dsu.FP32_MIXED)] = {
            "best": list(best), "seconds": {",".join(map(str, k)): v for k, v in secs.items()}}
        print(f"recompute n={n} walkers={w}: best (panel, chunk, apply)={best} "
              f"{ {k: round(v * 1e3, 2) for k, v in secs.items()} } ms", flush=True)
        save_cache(c, out_path)


if __name__ == "__main__":
    main(sys.argv[1:])
