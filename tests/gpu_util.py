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


# FP32 form: BT, products and flushes in FP32 (unit roundoff u = 2^-24).  A
# ratio is a dot product whose terms cancel, so its error is about
# u x sum|terms| (times a slowly growing accumulation factor), plus what the
# FP32 inverse has picked up since the last FP64 recompute; accepting a move
# with a small ratio scales that inverse error by 1/|R|.  For equilibrated
# configurations (cond(A) of order 1e2-1e3) the relative errors, with the
# 1e-3 floor of rel_err, are bounded as below, with the inverse residual
# max|A^-1 A - I| <= 1e-3 between recomputes.  Unequilibrated (uniform-random)
# configurations are checked against the per-ratio bound instead.
U32 = 2.0 ** -24
FP32_MEDIAN, FP32_P99, FP32_MAX = 1e-5, 2e-4, 1e-2
FP32_RESIDUAL = 1e-3


def assert_fp32_ratio_stats(err, median=FP32_MEDIAN, p99=FP32_P99, mx=FP32_MAX):
    err = np.asarray(err)
    stats = (float(np.median(err)), float(np.percentile(err, 99)), float(err.max()))
    assert stats[0] <= median and stats[1] <= p99 and stats[2] <= mx, stats
    return stats
