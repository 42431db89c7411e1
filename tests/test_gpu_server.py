"""The serving pool (dsu_server_*): continuous batching of mixed-size walkers.

A walker's result must not depend on what else is resident (its random
stream is keyed by its own seed and request id and every kernel's arithmetic
is per determinant), and admission must respect the device-memory budget.
"""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from paper_1708_00744_amd import dsu, inputs

pytestmark = pytest.mark.gpu

L = 10.0


def positions(seed, rid, n, spins):
    return inputs.positions(seed, rid, spins * n, L).reshape(spins, n, 3)


def run_alone(prec, K, req, sweeps):
    with dsu.Server(K, precision=prec, box_l=L, budget_bytes=1 << 30) as s:
        slot = s.add(req["request_id"], req["n"], req["spins"], req["seed"], req["sigma"], sweeps, req["positions"])
        for _ in range(sweeps):
            s.step()
        return s.result(slot, remove=True)


def test_alone_equals_mix():
    require_gpu()
    K, sweeps = 16, 3
    mk = lambda rid, n, spins, sig: {"request_id": rid, "n": n, "spins": spins, "seed": 77, "sigma": sig,
                                     "positions": positions(77, rid, n, spins)}
    a = mk(1, 128, 2, 0.2)
    others = [mk(2, 256, 1, 0.15), mk(3, 128, 1, 0.3), mk(4, 64, 2, 0.4)]
    for prec in (dsu.FP64, dsu.FP32_MIXED):
        alone = run_alone(prec, K, a, sweeps)
        with dsu.Server(K, precision=prec, box_l=L, budget_bytes=1 << 30) as s:
            slots = [s.add(r["request_id"], r["n"], r["spins"], r["seed"], r["sigma"], sweeps, r["positions"])
                     for r in [others[0], a] + others[1:]]
            for _ in range(sweeps):
                s.step()
            mixed = s.result(slots[1], remove=True)
            used, res = s.usage()
            assert res == 3
        assert mixed["logdet"] == alone["logdet"] and mixed["sign"] == alone["sign"]
        assert mixed["accepted"] == alone["accepted"] and mixed["sweeps_done"] == sweeps


def test_server_matches_batch_and_oracle():
    require_gpu()
    n, K, sweeps, seed, rid, sigma = 96, 16, 2, 5, 9, 0.3
    pos = positions(seed, rid, n, 1)
    res = run_alone(dsu.FP64, K, {"request_id": rid, "n": n, "spins": 1, "seed": seed, "sigma": sigma,
                                  "positions": pos}, sweeps)
    with dsu.Batch(n, pos[None], [seed], [rid], sigma, K, precision=dsu.FP64, box_l=L) as b:
        b.sweep(sweeps)
        st = b.stats()
    assert res["logdet"][0] == st["logdet"][0] and res["accepted"] == st["accepted"][0]
    t = oracle.walker_run(n, L, seed, rid, 0, sigma, pos[0], sweeps, residual=False, fresh=False)
    assert res["accepted"] == t.n_accepted[0]
    assert abs(res["logdet"][0] - t.logdet_run[-1]) < 1e-9 and res["sign"][0] == t.sign_run[-1]


def test_budget_admission_and_run():
    require_gpu()
    K, n, sweeps = 16, 256, 4
    per = dsu.footprint_bytes(n, K, dsu.FP32_MIXED)
    budget = dsu.server_workspace_bytes(n) + int(2.5 * per)  # the size's workspace and two walkers at a time
    reqs = [{"request_id": 100 + i, "n": n, "spins": 1, "seed": 3, "sigma": 0.1, "sweeps": sweeps,
             "arrival_s": 0.0, "positions": positions(3, 100 + i, n, 1)} for i in range(5)]
    # one request that can never fit
    reqs.append({"request_id": 200, "n": 2048, "spins": 2, "seed": 3, "sigma": 0.1, "sweeps": 1, "arrival_s": 0.0,
                 "positions": positions(3, 200, 2048, 2)})
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=budget) as s:
        results, lat = s.run(reqs)
        assert s.usage() == (0, 0)
    ok = [r for r in results if r["status"] == dsu.OK]
    assert len(ok) == 5 and results[-1]["status"] == dsu.EBUDGET
    assert all(r["sweeps_done"] == sweeps for r in ok)
    # at most two resident at once: every admission after the second waits for a retirement
    admits = sorted(r["admit_s"] for r in ok)
    finishes = sorted(r["finish_s"] for r in ok)
    for i in range(2, 5):
        assert admits[i] >= finishes[i - 2] - 1e-6
    assert len(lat) == 5 * sweeps and np.all(lat > 0)
    # each result equals the same request alone
    for r, q in zip(results[:2], reqs[:2]):
        alone = run_alone(dsu.FP32_MIXED, K, q, sweeps)
        assert r["logdet"] == alone["logdet"] and r["accepted"] == alone["accepted"]


def test_continuous_batching_overlaps_arrivals():
    """Requests arriving while others run join at the next sweep boundary."""
    require_gpu()
    K = 16
    reqs = []
    for i, (n, t) in enumerate([(512, 0.0), (128, 0.01), (256, 0.02), (128, 0.03)]):
        reqs.append({"request_id": 300 + i, "n": n, "spins": 2, "seed": 11, "sigma": 0.05, "sweeps": 6,
                     "arrival_s": t, "positions": positions(11, 300 + i, n, 2)})
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=1 << 30, recompute_every=3) as s:
        results, lat = s.run(reqs)
    assert all(r["status"] == dsu.OK and r["sweeps_done"] == 6 for r in results)
    # the first request was still running when the later ones were admitted
    assert min(r["admit_s"] for r in results[1:]) < results[0]["finish_s"]
    assert np.all(np.isfinite([r["logdet"][0] for r in results]))


def test_singular_walker_is_reported_not_fatal():
    """A walker whose Slater matrix is singular (two electrons at one point)
    is refused by dsu_server_add and ends with DSU_ESINGULAR in a run, while
    the other requests of the run complete unchanged."""
    require_gpu()
    K, n, sweeps = 16, 128, 2
    bad = positions(5, 1, n, 1).copy()
    bad[0, 7] = bad[0, 3]
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=1 << 30) as s:
        with pytest.raises(dsu.DsuError) as ex:
            s.add(1, n, 1, 5, 0.1, sweeps, bad)
        assert ex.value.code == dsu.ESINGULAR
        assert s.usage() == (0, 0)
    good = {"request_id": 2, "n": n, "spins": 1, "seed": 5, "sigma": 0.1, "sweeps": sweeps, "arrival_s": 0.0,
            "positions": positions(5, 2, n, 1)}
    reqs = [dict(good), {"request_id": 1, "n": n, "spins": 1, "seed": 5, "sigma": 0.1, "sweeps": sweeps,
                         "arrival_s": 0.0, "positions": bad}]
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=1 << 30) as s:
        results, lat = s.run(reqs)
        assert s.usage() == (0, 0)
    assert results[0]["status"] == dsu.OK and results[0]["sweeps_done"] == sweeps
    assert results[1]["status"] == dsu.ESINGULAR
    alone = run_alone(dsu.FP32_MIXED, K, good, sweeps)
    assert results[0]["logdet"] == alone["logdet"] and results[0]["accepted"] == alone["accepted"]


def test_recompute_groups_beyond_four_determinants():
    """Three walkers x two spins of one size (six determinants: the serving
    recompute runs four per pass, so the periodic recompute takes two passes):
    each walker's result over five sweeps with a recompute every two equals
    the same request alone (two determinants, one pass), bit for bit."""
    require_gpu()
    K, n, sweeps = 16, 96, 5
    reqs = [{"request_id": 40 + i, "n": n, "spins": 2, "seed": 9, "sigma": 0.2,
             "positions": positions(9, 40 + i, n, 2)} for i in range(3)]
    for prec in (dsu.FP64, dsu.FP32_MIXED):
        with dsu.Server(K, precision=prec, box_l=L, budget_bytes=1 << 30, recompute_every=2) as s:
            slots = [s.add(r["request_id"], n, 2, r["seed"], r["sigma"], sweeps, r["positions"]) for r in reqs]
            for _ in range(sweeps):
                s.step()
            mixed = [s.result(slot, remove=True) for slot in slots]
        for r, m in zip(reqs, mixed):
            with dsu.Server(K, precision=prec, box_l=L, budget_bytes=1 << 30, recompute_every=2) as s:
                slot = s.add(r["request_id"], n, 2, r["seed"], r["sigma"], sweeps, r["positions"])
                for _ in range(sweeps):
                    s.step()
                alone = s.result(slot, remove=True)
            assert m["logdet"] == alone["logdet"] and m["sign"] == alone["sign"]
            assert m["accepted"] == alone["accepted"] and m["sweeps_done"] == sweeps


def test_device_memory_within_budget():
    """Everything a pool holds on the device beyond its budget is its
    descriptors, orbital tables and streams: walkers of three sizes resident at
    once (their recompute workspaces included, 268 MB at n = 2048) raise the
    device memory in use by the budget and at most 16 MiB more (measured: 4
    MiB; the workspaces alone would be 357 MiB); dropping the last walker of a size releases that size's
    workspace to the budget."""
    torch = require_gpu()
    K, budget = 64, 1 << 30
    sizes = (512, 1024, 2048)
    reqs = [(100 + i, n, positions(13, 100 + i, n, 2)) for i, n in enumerate(sizes)]

    def fill(s):
        return [s.add(rid, n, 2, 13, 0.01, 2, p) for rid, n, p in reqs]

    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=budget) as s:  # load the kernels once
        fill(s)
        s.step()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with dsu.Server(K, precision=dsu.FP32_MIXED, box_l=L, budget_bytes=budget) as s:
        slots = fill(s)
        s.step()
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        used, resident = s.usage()
        ws = sum(dsu.server_workspace_bytes(n) for n in sizes)
        walkers = sum(2 * dsu.footprint_bytes(n, K, dsu.FP32_MIXED) for n in sizes)
        print(f"device memory raised by {(free0 - free1) / 2**20:.1f} MiB for a {budget / 2**20:.0f} MiB budget; "
              f"arena in use {used / 2**20:.1f} MiB (workspaces {ws / 2**20:.1f}, walkers {walkers / 2**20:.1f})",
              flush=True)
        assert resident == 3 and used >= ws + walkers
        assert free0 - free1 <= budget + (16 << 20)
        s.result(slots[2], remove=True)
        used2, _ = s.usage()
        assert used - used2 >= dsu.server_workspace_bytes(2048) + 2 * dsu.footprint_bytes(2048, K, dsu.FP32_MIXED)
