"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def rel_err(x, ref, floor=1e-3):
    """|x - ref| / max(|ref|, floor): a ratio near a node (R -> 0) is compared
    absolutely, elsewhere relatively."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(x - ref) / np.maximum(np.abs(ref), floor)


def marginal(u, r, tol):
    """Decisions u < R^2 whose outcome a relative error `tol` on R^2 could flip."""
    r2 = np.asarray(r) ** 2
    return np.abs(np.asarray(u) - r2) <= tol * np.maximum(r2, np.asarray(u))


# FP32 form: BT, products and flushes in FP32.  A ratio is a dot product of
# an orbital row with a column of the inverse whose terms cancel: its relative
# error is about (FP32 rounding, 6e-8) x (sum |terms| / |R|), which is 1-100
# for most moves and grows near nodes and for ill-conditioned (unequilibrated)
# configurations.  Bounds on the distribution of relative errors:
FP32_MEDIAN, FP32_P99, FP32_MAX = 1e-5, 2e-4, 5e-3


def assert_fp32_ratio_stats(err, median=FP32_MEDIAN, p99=FP32_P99, mx=FP32_MAX):
    err = np.asarray(err)
    stats = (float(np.median(err)), float(np.percentile(err, 99)), float(err.max()))
    assert stats[0] <= median and stats[1] <= p99 and stats[2] <= mx, stats
    return stats
