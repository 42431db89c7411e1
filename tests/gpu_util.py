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
