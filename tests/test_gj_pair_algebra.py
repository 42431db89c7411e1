"""Host-side check of the algebra behind the recompute's panel pairs.

The FP64 recompute inverts A^T in place by blocked Gauss-Jordan with partial
pivoting (panels of columns; each panel factored, then one trailing update
M' = P M + (T - E) Q of the other columns).  The GPU form can factor two
64-column panels R1, R2 one after the other and apply both trailing updates
in one pass:

    M1[:, R2] = (P1 M)[:, R2] + (T1 - E1) Q1[:, R2]      (second panel's input)
    Q2        = M1[P2 rows of R2]                         (its pivot rows)
    M'        = P2 P1 M + P2 (T1 - E1) Q1 + (T2 - E2) Q2  (columns outside R1, R2)
    M'[:, R1] = P2 T1 + (T2 - E2) (P2 T1)[R2],   M'[:, R2] = T2

Here both forms are written with numpy on small matrices (panels of 8 or 16
columns standing in for 64) and must give the same inverse, pivots and
log-determinant, and the inverse must match LAPACK's.  This checks the
identity the kernels implement, not the kernels (the GPU tests compare those
with LAPACK).
"""
import numpy as np
import pytest


def _factor(P, k0, n):
    """In-place Gauss-Jordan on the panel P (rows in current order) with
    partial pivoting over rows >= k; returns the pivots and sum ln|pivot|."""
    piv, logdet = [], 0.0
    for kk in range(P.shape[1]):
        k = k0 + kk
        p = k + int(np.argmax(np.abs(P[k:n, kk])))
        piv.append(p)
        P[[k, p], :] = P[[p, k], :]
        d = P[k, kk]
        logdet += np.log(abs(d))
        rp = P[k, :] / d
        rp[kk] = 1.0 / d
        f = P[:, kk].copy()
        P -= np.outer(f, rp)
        P[:, kk] = -f / d
        P[k, :] = rp
    return piv, logdet


def _rowsrc(piv, k0, n):
    rs = np.arange(n)
    for kk, p in enumerate(piv):
        k = k0 + kk
        rs[k], rs[p] = rs[p], rs[k]
    return rs


def _eye_cols(n, k0, w):
    E = np.zeros((n, w))
    E[k0 + np.arange(w), np.arange(w)] = 1.0
    return E


def _single_step(M, k0, w, n):
    P = M[:, k0:k0 + w].copy()
    piv, ld = _factor(P, k0, n)
    rs = _rowsrc(piv, k0, n)
    out = M[rs, :] + (P - _eye_cols(n, k0, w)) @ M[rs[k0:k0 + w], :]
    out[:, k0:k0 + w] = P
    return out, piv, ld


def _pair_step(M, k0, nb, n):
    R1, R2 = slice(k0, k0 + nb), slice(k0 + nb, k0 + 2 * nb)
    T1 = M[:, R1].copy()
    piv1, ld1 = _factor(T1, k0, n)
    rs1 = _rowsrc(piv1, k0, n)
    E1 = _eye_cols(n, k0, nb)
    qrow = rs1[k0:k0 + nb]
    T2 = M[rs1, R2] + (T1 - E1) @ M[qrow, R2]
    piv2, ld2 = _factor(T2, k0 + nb, n)
    rs2 = _rowsrc(piv2, k0 + nb, n)
    rs12 = rs1[rs2]
    E2 = _eye_cols(n, k0 + nb, nb)
    r = rs2[R2]
    q2 = M[rs12[R2], :] + (T1[r] - E1[r]) @ M[qrow, :]
    out = M[rs12, :] + (T1[rs2] - E1[rs2]) @ M[qrow, :] + (T2 - E2) @ q2
    out[:, R2] = T2
    out[:, R1] = T1[rs2] + (T2 - E2) @ T1[rs2[R2]]
    return out, piv1 + piv2, ld1 + ld2


def _invert(A, nb, pairs):
    n = A.shape[0]
    M, pivs, logdet, k0 = A.T.copy(), [], 0.0, 0
    while k0 < n:
        if pairs and k0 + 2 * nb <= n:
            M, piv, ld = _pair_step(M, k0, nb, n)
            k0 += 2 * nb
        else:
            w = min(nb, n - k0)
            M, piv, ld = _single_step(M, k0, w, n)
            k0 += w
        pivs += piv
        logdet += ld
    perm = np.arange(n)
    for k in range(n - 1, -1, -1):
        p = pivs[k]
        perm[k], perm[p] = perm[p], perm[k]
    return M[:, perm], pivs, logdet


@pytest.mark.parametrize("n,nb", [(64, 8), (100, 8), (96, 16), (200, 16)])
def test_panel_pairs_match_single_panels(n, nb):
    a = np.random.default_rng(n + nb).standard_normal((n, n))
    x1, p1, l1 = _invert(a, nb, pairs=False)
    x2, p2, l2 = _invert(a, nb, pairs=True)
    assert p1 == p2
    ref = np.linalg.inv(a).T  # the in-place form inverts A^T
    scale = np.abs(ref).max()
    assert np.abs(x1 - ref).max() < 1e-11 * scale
    assert np.abs(x2 - ref).max() < 1e-11 * scale
    assert np.abs(x2 - x1).max() < 1e-12 * scale
    assert abs(l1 - l2) < 1e-10 and abs(l2 - np.linalg.slogdet(a)[1]) < 1e-9
