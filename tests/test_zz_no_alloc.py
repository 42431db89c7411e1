"""The allocation-free residual entry point (dsu_batch_residual_noalloc)
against dsu_batch_residual: the same kernels on buffers carved from the
library's static per-GPU scratch array, so the results must be bit-identical,
on two calls in a row with the second one smaller, and the size check must
refuse a batch that needs more scratch than the array has."""
import numpy as np
import pytest

from gpu_util import require_gpu
from paper_1708_00744_amd import dsu, inputs

pytestmark = pytest.mark.gpu

L = 10.0


def batch(n, walkers, spins, K, prec, seed):
    pos = np.stack([inputs.positions(seed, w, spins * n, L).reshape(spins, n, 3) for w in range(walkers)])
    return dsu.Batch(n, pos, [seed] * walkers, list(range(walkers)), 0.2, K, precision=prec, spins=spins, box_l=L)


def same(x, y):
    return np.array_equal(x.view(np.uint64), y.view(np.uint64))


def test_noalloc_residual_equals_allocating_entry_point():
    require_gpu()
    # first call: 3 walkers x 2 spins of n = 520 (ragged), 40 samples; then a
    # smaller one: 1 walker of n = 130, FP64, 16 samples (the array keeps the
    # first call's contents, which the second must not read)
    for (n, walkers, spins, K, prec, samples, sweeps) in ((520, 3, 2, 64, dsu.FP32_MIXED, 40, 2),
                                                          (130, 1, 1, 16, dsu.FP64, 16, 1)):
        with batch(n, walkers, spins, K, prec, 17) as b:
            b.sweep(sweeps)
            r_ref, l_ref = b.residual(samples)
            r_na, l_na = b.residual_noalloc(samples)
            print(f"n={n} dets={b.ndet}: right {r_na.max():.3e} left {l_na.max():.3e}", flush=True)
            assert same(r_na, r_ref) and same(l_na, l_ref)
            assert np.all(r_na > 0) and np.all(l_na > 0)
            # one side only
            r1, none = b.residual_noalloc(samples, left=False)
            assert none is None and same(r1, r_ref)
            none, l1 = b.residual_noalloc(samples, right=False)
            assert none is None and same(l1, l_ref)


def test_noalloc_residual_refuses_oversized_batch():
    """16 determinants of n = 4096 with 64 samples need 16 * 64 * 4096 * 8 =
    32 MiB of sample rows plus the indices and result words: more than the
    array; the call fails before launching anything and the batch stays
    usable."""
    require_gpu()
    with batch(4096, 16, 1, 32, dsu.FP32_MIXED, 5) as b:
        with pytest.raises(dsu.DsuError) as ex:
            b.residual_noalloc(64)
        assert ex.value.code == dsu.EINVAL and "scratch" in str(ex.value)
        r_ref, _ = b.residual(32, left=False)
        r_na, _ = b.residual_noalloc(32, left=False)
        assert same(r_na, r_ref)
