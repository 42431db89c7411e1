"""Parity of the complex-orbital walker (dsu_zwalker_*) with the complex oracle.

Twisted plane waves (seeded twist, positions and moves); the oracle applies
each accepted move at once with complex Sherman-Morrison (eq. (2)), the library
delays them (eq. (3) look-ahead, eq. (4) flush).  Same rows and uniforms on
both sides; Metropolis weight |R|^2.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_util import marginal, require_gpu
from paper_1708_00744_amd import dsu, inputs
from test_oracle_pins import _fc_det, _gauss_int_matrix

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
THETA = np.array([0.31, -0.17, 0.42])


def zrel(x, ref, floor=1e-3):
    return abs(x - ref) / max(abs(ref), floor)


def phase_diff(a, b):
    d = (a - b + np.pi) % (2 * np.pi) - np.pi
    return abs(d)


def twisted_system(n, L, seed):
    kv = oracle.zpw_kvectors(n, THETA)
    pos = inputs.positions(seed, 0, n, L)
    return kv, pos, oracle.zpw_matrix(kv, THETA, L, pos)


def run_zwalker(n, K, policy, nmoves, seed, L=4.0, sigma=0.15, mode=None):
    kv, pos, a = twisted_system(n, L, seed)
    ainv, _, _ = oracle.zinverse(a)
    order = inputs.electron_order(seed + 1, n, nmoves)
    g = inputs.normals(seed + 2, (nmoves, 3))
    us = inputs.uniforms(seed + 3, nmoves)
    errs = []
    w = dsu.ZWalker(a, K, policy=policy)
    if mode is not None:
        w.set_flush_kernel(mode)
    for m in range(nmoves):
        e = int(order[m])
        rt = pos[e] + sigma * g[m]
        row = oracle.zpw_row(kv, THETA, L, rt)
        rg = w.propose(e, row)
        ro = oracle.zsm_ratio(ainv, e, row)
        errs.append(zrel(rg, ro))
        acc_o, acc_g = us[m] < abs(ro) ** 2, us[m] < abs(rg) ** 2
        if acc_o != acc_g:
            assert marginal(us[m], abs(ro), 1e-8), (m, rg, ro, us[m])
            break
        if acc_o:
            w.accept()
            oracle.zsm_accept(ainv, a, e, row, ro)
            pos[e] = rt
        else:
            w.reject()
    return w, a, ainv, np.array(errs)


@pytest.mark.parametrize("n", [1, 5, 64, 100, 200])
def test_zcreate_inverts(n):
    require_gpu()
    _, _, a = twisted_system(n, 3.0, 10 + n)
    with dsu.ZWalker(a, 8) as w:
        inv = w.inverse()
        la, ph = w.logdet()
    np.testing.assert_allclose(inv, np.linalg.inv(a), rtol=1e-9, atol=1e-11)
    s, l = np.linalg.slogdet(a)
    assert abs(la - l) < 1e-10 * max(1, abs(l)) and phase_diff(ph, np.angle(s)) < 1e-10


@pytest.mark.parametrize("K,policy,mode", [(1, dsu.FLUSH_K_ACCEPTED, None), (4, dsu.FLUSH_K_PROPOSED, None),
                                           (4, dsu.FLUSH_K_PROPOSED, dsu.FLUSH_VALU),
                                           (16, dsu.FLUSH_K_ACCEPTED, None), (16, dsu.FLUSH_K_ACCEPTED, dsu.FLUSH_VALU),
                                           (40, dsu.FLUSH_K_PROPOSED, dsu.FLUSH_MFMA),
                                           (64, dsu.FLUSH_K_ACCEPTED, None), (64, dsu.FLUSH_K_ACCEPTED, dsu.FLUSH_VALU),
                                           (128, dsu.FLUSH_K_ACCEPTED, None), (200, dsu.FLUSH_K_ACCEPTED, None)])
def test_zratios_decisions_inverse(K, policy, mode):
    """Both flush kernels (matrix cores through the real embedding, and the
    vector-ALU complex kernels; K = 200 exceeds the embedding's 256 slots and
    takes the latter) against the complex oracle."""
    require_gpu()
    n = 96
    w, a, ainv, errs = run_zwalker(n, K, policy, 3 * n, seed=300 + K, mode=mode)
    assert len(errs) > 2 * n and errs.max() < FP64_TOL
    np.testing.assert_allclose(w.inverse(), ainv, rtol=1e-9, atol=1e-10)
    la, ph = w.logdet()
    lo, po = oracle.zslogdet(a)
    assert abs(la - lo) < 1e-9 and phase_diff(ph, po) < 1e-9
    w.close()


def test_zexact_gaussian_integer_ratios():
    """Gaussian-integer rows: every ratio is an exact complex rational."""
    require_gpu()
    n = 5
    a = _gauss_int_matrix(7, n)
    cur = a.copy()
    rng = np.random.default_rng(8)
    with dsu.ZWalker(a, 4) as w:
        for step in range(24):
            e = int(rng.integers(0, n))
            row = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex128)
            new = cur.copy(); new[e] = row
            d0, d1 = _fc_det(cur), _fc_det(new)
            den = d0[0] ** 2 + d0[1] ** 2
            exact = complex(float((d1[0] * d0[0] + d1[1] * d0[1]) / den), float((d1[1] * d0[0] - d1[0] * d0[1]) / den))
            r = w.propose(e, row)
            assert abs(r - exact) <= 1e-11 * max(1.0, abs(exact))
            if d1 != (Fraction(0), Fraction(0)):
                w.accept()
                cur = new
            else:
                w.reject()
        inv = w.inverse()
    np.testing.assert_allclose(inv, np.linalg.inv(cur), rtol=1e-9, atol=1e-11)


def test_zspecial_cases():
    require_gpu()
    n = 30
    _, _, a = twisted_system(n, 3.0, 21)
    with dsu.ZWalker(a, 8) as w:
        assert abs(w.propose(3, a[3]) - 1.0) < 1e-12     # null move
        w.reject()
        assert abs(w.propose(5, a[6])) < 1e-12           # Pauli: equal rows
        with pytest.raises(dsu.DsuError) as ex:
            w.accept()
        assert ex.value.code == dsu.ESINGULAR
        w.reject()
        with pytest.raises(dsu.DsuError) as ex:
            w.accept()
        assert ex.value.code == dsu.ESTATE
        with pytest.raises(dsu.DsuError) as ex:
            w.propose(n, a[0])
        assert ex.value.code == dsu.EINVAL
        # a phase-only change of one row: |R| = 1, arg R = the phase
        r = w.propose(7, np.exp(0.7j) * a[7])
        assert abs(r - np.exp(0.7j)) < 1e-12
        w.accept()
        la0, ph0 = oracle.zslogdet(a)
        la, ph = w.logdet()
        assert abs(la - la0) < 1e-10 and phase_diff(ph, ph0 + 0.7) < 1e-10
        b = a.copy(); b[7] *= np.exp(0.7j)
        np.testing.assert_allclose(w.inverse(), np.linalg.inv(b), rtol=1e-10, atol=1e-12)


def test_zsingular_create():
    require_gpu()
    _, _, a = twisted_system(12, 3.0, 31)
    a[4] = a[9]
    with pytest.raises(dsu.DsuError) as ex:
        dsu.ZWalker(a, 4)
    assert ex.value.code == dsu.ESINGULAR


def test_zrecompute_and_drift():
    require_gpu()
    n = 80
    w, a, ainv, errs = run_zwalker(n, 16, dsu.FLUSH_K_ACCEPTED, 2 * n, seed=41)
    la, ph, drift = w.recompute()
    lo, po = oracle.zslogdet(a)
    assert abs(la - lo) < 1e-10 and phase_diff(ph, po) < 1e-10 and abs(drift) < 1e-9
    np.testing.assert_allclose(w.inverse(), np.linalg.inv(a), rtol=1e-9, atol=1e-11)
    _, _, b = twisted_system(n, 4.0, 42)
    la2, ph2, _ = w.recompute(b)
    s, l = np.linalg.slogdet(b)
    assert abs(la2 - l) < 1e-10 and phase_diff(ph2, np.angle(s)) < 1e-10
    w.close()


def test_zwalker_n1024_k64_matrix_cores():
    """N = 1024, K = 64 with the flush on the matrix cores: 300 moves, every
    ratio against the complex oracle (complex Sherman-Morrison), the final
    inverse against the oracle's, and the flush kernels' results against each
    other: the same walk with the vector-ALU flush lands on the same inverse
    to rounding."""
    require_gpu()
    inv = {}
    for mode in (dsu.FLUSH_MFMA, dsu.FLUSH_VALU):
        w, a, ainv, errs = run_zwalker(1024, 64, dsu.FLUSH_K_ACCEPTED, 300, seed=71, L=10.0, sigma=0.05, mode=mode)
        assert len(errs) == 300 and errs.max() < FP64_TOL
        inv[mode] = w.inverse()
        np.testing.assert_allclose(inv[mode], ainv, rtol=1e-8, atol=1e-9 * np.abs(ainv).max())
        w.close()
    assert np.abs(inv[dsu.FLUSH_MFMA] - inv[dsu.FLUSH_VALU]).max() < 1e-9 * np.abs(ainv).max()


def test_zwalker_n512_sampled():
    """N = 512, K = 64: 400 moves, every ratio against the oracle."""
    require_gpu()
    w, a, ainv, errs = run_zwalker(512, 64, dsu.FLUSH_K_ACCEPTED, 400, seed=51, L=8.0, sigma=0.1)
    assert len(errs) == 400 and errs.max() < FP64_TOL
    np.testing.assert_allclose(w.inverse(), ainv, rtol=1e-8, atol=1e-9)
    w.close()
