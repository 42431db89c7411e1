"""Parity of the host-driven single walker (dsu_walker_*) with the CPU oracle.

The oracle applies every accepted move at once with Sherman-Morrison (eq. (2));
the library delays them (eq. (3) look-ahead, eq. (4) en-bloc update).  Both
see the same seeded rows and uniforms; ratios must agree to the FP64 bound and
decisions must be identical (the paper's equivalence, Sec. II).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_util import assert_fp32_ratio_stats, marginal, rel_err, require_gpu
from paper_1708_00744_amd import dsu, inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def run_walker(n, K, policy, mode, nmoves, seed, precision=dsu.FP64, mix=0.15):
    """Drive walker and oracle through the same proposals; return per-move
    (gpu R, oracle R, u) and the final objects."""
    a = inputs.dense_matrix(seed, n) + 2.0 * np.eye(n)
    ainv, _, _ = oracle.inverse(a)
    order = inputs.electron_order(seed + 1, n, nmoves)
    noise = inputs.rows(seed + 2, nmoves, n)
    us = inputs.uniforms(seed + 3, nmoves)
    rg, ro = np.zeros(nmoves), np.zeros(nmoves)
    w = dsu.Walker(a, K, precision=precision, policy=policy)
    if mode is not None:
        w.set_flush_kernel(mode)
    for m, (e, z, u) in enumerate(zip(order, noise, us)):
        row = (1.0 - mix) * a[e] + mix * z
        rg[m] = w.propose(e, row)
        ro[m] = oracle.sm_ratio(ainv, e, row)
        acc_o = u < ro[m] ** 2
        acc_g = u < rg[m] ** 2
        if acc_g != acc_o:
            assert marginal(u, ro[m], 1e-8 if precision == dsu.FP64 else 1e-3), (m, rg[m], ro[m], u)
            break
        if acc_o:
            w.accept()
            oracle.sm_accept(ainv, a, e, row, ro[m])
        else:
            w.reject()
    return w, a, ainv, rg, ro


@pytest.mark.parametrize("n", [1, 5, 64, 100, 333])
def test_create_inverts(n):
    require_gpu()
    a = inputs.dense_matrix(7 + n, n) + 2.0 * np.eye(n)
    with dsu.Walker(a, 8) as w:
        inv = w.inverse()
        sg, ld = w.logdet()
    np.testing.assert_allclose(inv, np.linalg.inv(a), rtol=1e-9, atol=1e-11)
    s_np, l_np = np.linalg.slogdet(a)
    assert sg == s_np and abs(ld - l_np) < 1e-10 * max(1, abs(l_np))


@pytest.mark.parametrize("K,policy,mode", [
    (1, dsu.FLUSH_K_ACCEPTED, None),
    (4, dsu.FLUSH_K_ACCEPTED, dsu.FLUSH_VALU),
    (4, dsu.FLUSH_K_PROPOSED, dsu.FLUSH_MFMA),
    (16, dsu.FLUSH_K_ACCEPTED, dsu.FLUSH_MFMA),
    (16, dsu.FLUSH_K_PROPOSED, dsu.FLUSH_VALU),
    (40, dsu.FLUSH_K_ACCEPTED, None),
    (64, dsu.FLUSH_K_PROPOSED, None),
    (128, dsu.FLUSH_K_ACCEPTED, None),
    (256, dsu.FLUSH_K_ACCEPTED, None),
])
def test_ratios_decisions_inverse_fp64(K, policy, mode):
    require_gpu()
    n = 96
    w, a, ainv, rg, ro = run_walker(n, K, policy, mode, nmoves=3 * n, seed=100 + K)
    assert rel_err(rg, ro).max() < FP64_TOL
    np.testing.assert_allclose(w.inverse(), ainv, rtol=1e-9, atol=1e-10)
    sg, ld = w.logdet()
    s_o, l_o = oracle.slogdet(a)
    assert sg == s_o and abs(ld - l_o) < 1e-9
    w.close()


def test_exact_rational_ratios():
    """Integer rows: every ratio is an exact rational det(A_new)/det(A)."""
    require_gpu()

    def fdet(m):
        m = [[Fraction(int(x)) for x in r] for r in m]
        d = Fraction(1)
        for k in range(len(m)):
            p = next((i for i in range(k, len(m)) if m[i][k] != 0), None)
            if p is None:
                return Fraction(0)
            if p != k:
                m[k], m[p] = m[p], m[k]
                d = -d
            d *= m[k][k]
            for i in range(k + 1, len(m)):
                f = m[i][k] / m[k][k]
                for j in range(k, len(m)):
                    m[i][j] -= f * m[k][j]
        return d

    n = 6
    a = inputs.integer_matrix(3, n) + 4 * np.eye(n)
    cur = a.copy()
    rows = inputs.rows(5, 24, n, kind="integer")
    order = inputs.electron_order(6, n, 24)
    with dsu.Walker(a, 4) as w:
        for e, row in zip(order, rows):
            new = cur.copy(); new[e] = row
            exact = fdet(new) / fdet(cur)
            r = w.propose(e, row)
            assert abs(r - float(exact)) <= 1e-11 * max(1.0, abs(float(exact)))
            if exact != 0:
                w.accept()
                cur = new
            else:
                w.reject()
        inv = w.inverse()
    np.testing.assert_allclose(inv, np.linalg.inv(cur), rtol=1e-9, atol=1e-11)


def test_special_cases():
    require_gpu()
    n = 40
    a = inputs.dense_matrix(9, n) + 2.0 * np.eye(n)
    with dsu.Walker(a, 8) as w:
        # null move -> 1
        assert abs(w.propose(3, a[3]) - 1.0) < 1e-12
        w.reject()
        # a row equal to another electron's row -> 0, which cannot be accepted;
        # the failed call leaves the walker (and its pending proposal) unchanged
        assert abs(w.propose(5, a[6])) < 1e-12
        with pytest.raises(dsu.DsuError) as ex:
            w.accept()
        assert ex.value.code == dsu.ESINGULAR
        w.reject()
        # no pending proposal now
        with pytest.raises(dsu.DsuError) as ex:
            w.accept()
        assert ex.value.code == dsu.ESTATE
        with pytest.raises(dsu.DsuError) as ex:
            w.propose(n, a[0])
        assert ex.value.code == dsu.EINVAL
        np.testing.assert_allclose(w.inverse(), np.linalg.inv(a), rtol=1e-10, atol=1e-12)


def test_singular_create():
    require_gpu()
    a = inputs.dense_matrix(2, 10)
    a[4] = a[7]
    with pytest.raises(dsu.DsuError) as ex:
        dsu.Walker(a, 4)
    assert ex.value.code == dsu.ESINGULAR


def test_repeat_electron_flushes_first():
    require_gpu()
    n = 32
    a = inputs.dense_matrix(12, n) + 2.0 * np.eye(n)
    ainv, _, _ = oracle.inverse(a)
    rows = inputs.rows(13, 6, n)
    with dsu.Walker(a, 16) as w:
        for i, e in enumerate([3, 7, 3, 3, 7, 9]):
            row = 0.8 * a[e] + 0.2 * rows[i]
            r = w.propose(e, row)
            ro = oracle.sm_ratio(ainv, e, row)
            assert abs(r - ro) < 1e-11 * max(1, abs(ro))
            w.accept()
            oracle.sm_accept(ainv, a, e, row, ro)
        assert w.pending() >= 1
        np.testing.assert_allclose(w.inverse(), ainv, rtol=1e-10, atol=1e-11)


def test_recompute_and_drift():
    require_gpu()
    n = 80
    w, a, ainv, rg, ro = run_walker(n, 16, dsu.FLUSH_K_ACCEPTED, None, nmoves=2 * n, seed=31)
    ld, sg, drift = w.recompute()
    s_o, l_o = oracle.slogdet(a)
    assert sg == s_o and abs(ld - l_o) < 1e-10
    assert abs(drift) < 1e-9
    np.testing.assert_allclose(w.inverse(), np.linalg.inv(a), rtol=1e-9, atol=1e-11)
    # replacing A resets the walker to the new matrix
    b = inputs.dense_matrix(32, n) + 2.0 * np.eye(n)
    ld2, sg2, _ = w.recompute(b)
    assert sg2 == np.linalg.slogdet(b)[0] and abs(ld2 - np.linalg.slogdet(b)[1]) < 1e-10
    w.close()


def test_fp32_mixed_walker():
    require_gpu()
    n = 128
    w, a, ainv, rg, ro = run_walker(n, 32, dsu.FLUSH_K_ACCEPTED, None, nmoves=n, seed=41, precision=dsu.FP32_MIXED)
    m = np.count_nonzero(rg)
    assert_fp32_ratio_stats(rel_err(rg[:m], ro[:m]))
    res = np.abs(w.inverse() @ a - np.eye(n)).max()
    assert res < 1e-3
    w.close()


def test_propose_dev_matches_host():
    torch = require_gpu()
    n = 70
    a = inputs.dense_matrix(51, n) + 2.0 * np.eye(n)
    rows = inputs.rows(52, 5, n)
    with dsu.Walker(a, 8) as w1, dsu.Walker(a, 8) as w2:
        for e, row in enumerate(rows):
            r1 = w1.propose(e, row)
            dev = torch.tensor(row, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            r2 = w2.propose_dev(e, dev.data_ptr())
            assert r1 == r2
            w1.accept(); w2.accept()
        np.testing.assert_array_equal(w1.inverse(), w2.inverse())


def test_plane_wave_c2_size_sampled():
    """N = 1024 (the single-walker FP64 workload): plane-wave rows from the
    oracle's orbitals at seeded positions, K = 64, 300 moves."""
    require_gpu()
    n, L, K = 1024, 10.0, 64
    kv = oracle.pw_kvectors(n)
    pos = inputs.positions(2, 0, n, L)
    a = oracle.pw_matrix(kv, L, pos)
    ainv, _, _ = oracle.inverse(a)
    g = inputs.normals(3, (300, 3))
    us = inputs.uniforms(4, 300)
    errs = []
    with dsu.Walker(a, K) as w:
        for m in range(300):
            e = m
            rt = pos[e] + 0.004 * L * g[m]
            row = oracle.pw_row(kv, L, rt)
            r = w.propose(e, row)
            ro = oracle.sm_ratio(ainv, e, row)
            errs.append(rel_err(r, ro))
            if us[m] < ro * ro:
                assert us[m] < r * r
                w.accept()
                oracle.sm_accept(ainv, a, e, row, ro)
                pos[e] = rt
            else:
                w.reject()
        inv = w.inverse()
    assert max(errs) < FP64_TOL
    np.testing.assert_allclose(inv, ainv, rtol=1e-8, atol=1e-9)
