"""The streaming flush with split-bf16 products (flush path 2) of the FP32
batched form: each FP32 operand is split into three bf16 parts and six cross
products are kept, which bounds a product's error by that of FP32 products.
So every FP32 bound of the other paths applies unchanged: the same ratios
against the oracle, the same inverse residual, the same agreement with the
FP32-product paths, bit-identical graph replays.
"""
import numpy as np
import pytest

import oracle
from gpu_util import FP32_RESIDUAL, assert_fp32_ratio_stats, marginal, rel_err, require_gpu
from paper_1708_00744_amd import dsu
from test_gpu_batch import L, burned_in, make_batch, oracle_det

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,K,walkers", [(256, 32, 4), (192, 64, 3), (256, 128, 2), (320, 128, 2), (160, 100, 2)])
def test_x6_force_accept_against_oracle(n, K, walkers):
    """100% acceptance: every ratio compared with the oracle's Sherman-Morrison
    chain; n = 192 and 320 leave a 64-row last block, K = 100 pads to 128.
    The inverse residual is held to the FP32 bound where that bound's premise
    holds (cond(A) <= 3e3 at the end) and, everywhere, to within a factor 3
    of the FP32-product path on the same inputs."""
    require_gpu()
    sigma = 0.02
    p0 = burned_in(n, walkers, 1, 21)
    kv = oracle.pw_kvectors(n)
    res = {}
    for path in (dsu.PATH_STREAM_X6, dsu.PATH_STREAM):
        b, pos = make_batch(n, walkers, 1, K, dsu.FP32_MIXED, sigma, seed=21, pos=p0)
        b.set_flush_path(path)
        b.set_trace(2)
        b.sweep(2, force_accept=True)
        st = b.stats()
        errs = []
        for w in range(walkers):
            t = oracle_det(n, pos, w, 0, sigma, 2, seed=21, force=True)
            r, a = b.trace(w)
            assert a.all()
            errs.append(rel_err(r, t.ratio))
            assert abs(st["logdet"][w] - t.logdet_run[-1]) < 2e-2
            a_end = oracle.pw_matrix(kv, L, t.pos)
            res[path, w] = (np.abs(b.inverse(w) @ a_end - np.eye(n)).max(), np.linalg.cond(a_end))
        print(f"path {path}: ratio error median/p99/max", assert_fp32_ratio_stats(np.concatenate(errs)), flush=True)
        b.close()
    for w in range(walkers):
        (r6, cond), (r1, _) = res[dsu.PATH_STREAM_X6, w], res[dsu.PATH_STREAM, w]
        print(f"walker {w}: cond {cond:.1e} residual x6 {r6:.2e} fp32 {r1:.2e}", flush=True)
        assert r6 <= 3 * r1 + 1e-5
        if cond <= 3e3:
            assert r6 < FP32_RESIDUAL


@pytest.mark.parametrize("n,K", [(128, 32), (256, 64), (256, 128)])
def test_x6_decisions_match_oracle_until_marginal(n, K):
    require_gpu()
    walkers, sigma = 4, 0.2
    b, pos = make_batch(n, walkers, 1, K, dsu.FP32_MIXED, sigma, seed=31, pos=burned_in(n, walkers, 1, 31))
    b.set_flush_path(dsu.PATH_STREAM_X6)
    b.set_trace(2)
    b.sweep(2)
    compared = 0
    for w in range(walkers):
        t = oracle_det(n, pos, w, 0, sigma, 2, seed=31)
        r, a = b.trace(w)
        diff = np.nonzero(a != t.accepted)[0]
        upto = diff[0] if len(diff) else len(a)
        if len(diff):
            m = diff[0]
            assert marginal(t.u[m], t.ratio[m], 1e-2), (w, m, r[m], t.ratio[m], t.u[m])
        assert_fp32_ratio_stats(rel_err(r[:upto], t.ratio[:upto]))
        compared += upto
    assert compared > walkers * n
    b.close()


@pytest.mark.parametrize("n,K", [(256, 64), (192, 128)])
def test_x6_agrees_with_fp32_product_paths(n, K):
    require_gpu()
    p0 = burned_in(n, 2, 1, 51)
    out = []
    for path in (dsu.PATH_STREAM_X6, dsu.PATH_STREAM, dsu.PATH_WINDOWS):
        b, _ = make_batch(n, 2, 1, K, dsu.FP32_MIXED, 0.2, seed=51, pos=p0)
        b.set_flush_path(path)
        b.set_trace(2)
        b.sweep(2)
        out.append((b.trace(0), b.trace(1)))
        b.close()
    for other in out[1:]:
        for (r0, a0), (r1, a1) in zip(out[0], other):
            m = len(a0) if np.array_equal(a0, a1) else int(np.nonzero(a0 != a1)[0][0])
            assert m > n
            assert_fp32_ratio_stats(rel_err(r0[:m], r1[:m]))


def test_x6_graph_replay_equals_eager():
    require_gpu()
    outs = []
    for graph in (False, True):
        b, _ = make_batch(192, 2, 1, 64, dsu.FP32_MIXED, 0.25, seed=11, graph=graph)
        b.set_flush_path(dsu.PATH_STREAM_X6)
        b.set_trace(3)
        for _ in range(3):
            b.sweep(1)
            b.sync()
        outs.append((b.trace(0), b.trace(1), b.stats()))
        b.close()
    (e0, e1, es), (g0, g1, gs) = outs
    for x, y in ((e0, g0), (e1, g1)):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    assert np.array_equal(es["logdet"], gs["logdet"])


def test_bad_flush_path():
    require_gpu()
    b, _ = make_batch(64, 1, 1, 8, dsu.FP32_MIXED, 0.2, seed=3)
    with pytest.raises(dsu.DsuError) as ex:
        b.set_flush_path(3)
    assert ex.value.code == dsu.EINVAL
    b.close()
