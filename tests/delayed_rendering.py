"""A plain CPU rendering of the delayed update, in FP64 or FP32 -- tolerance
evidence for the GPU tests, never a checker of them.

The batched GPU form works in windows of K consecutive proposals of one
determinant (each electron moves at most once per window, so every proposal
of a window is known before any of its decisions).  Per window it forms the
look-ahead products G[a][b] = U[a] . BT[e0+b] of the proposed orbital rows U
with the window's rows of the transposed stale inverse BT, takes each slot's
ratio as the Schur complement of eq. (3) over the slots accepted before it,
R_a = G[a][a] - G[a, J] C_J^-1 G[J, a]  (C_J = G[J, J]), with C_J^-1 grown by
one bordering step per acceptance (no pivoting: each step divides by the
accepted ratio, which is what makes rounding grow where small ratios are
accepted),
and applies the accepted moves en bloc with the Woodbury formula, eq. (4),
written for BT:  BT <- BT - (BT U_J^T - E) C_J^-T BT[e_J].

This module repeats exactly those steps with numpy, with BT, U and every
product of them held in the chosen precision and the K x K algebra in FP64,
as the GPU's FP32 form does.  Its rounding differs from the GPU's (BLAS
blocking instead of matrix-core tiles) but is of the same kind, so what it
measures -- how far a correct delayed implementation in that precision lands
from the sequential FP64 oracle -- is what the GPU tests may allow.  The
move random numbers and orbital rows come from the oracle (the published
Philox/Box-Muller stream and the plane-wave definition); nothing here comes
from the product library.

exact_ratios() is the definition itself: det(A_new)/det(A) from two LAPACK
LU factorisations per move along a given accept/reject path.
"""
import numpy as np

import oracle


class Rendering:
    def __init__(self, n, sweeps):
        self.ratio = np.zeros(sweeps * n)
        self.accepted = np.zeros(sweeps * n, np.uint8)
        self.u = np.zeros(sweeps * n)
        self.logdet = 0.0
        self.sign = 1
        self.pos = None
        self.bt = None          # final transposed inverse, in the rendering's precision
        self.residual = []      # max |A^-1 A - I| after each sweep (exact FP64 evaluation)

    def inverse(self):
        return np.ascontiguousarray(self.bt.T.astype(np.float64))


def render_delayed(n, L, K, dtype, seed, wid, spin, sigma, pos0, sweeps, force_accept=False, first_sweep=0,
                   residual=False, residual_rows=None, lapack_start=False):
    """Run `sweeps` sweeps of one determinant with delay K in precision
    `dtype` (np.float64 or np.float32) from the positions pos0 (n x 3).
    residual_rows: evaluate the residual only on these rows of A^-1 A - I;
    lapack_start: the starting inverse from LAPACK (large n) instead of the
    oracle's own LU."""
    kv = oracle.pw_kvectors(n)
    pos = np.array(pos0, np.float64).reshape(n, 3).copy()
    if lapack_start:
        a0 = oracle.pw_matrix(kv, L, pos)
        ainv = np.linalg.inv(a0)
        sign, logdet = np.linalg.slogdet(a0)
    else:
        ainv, sign, logdet = oracle.inverse(oracle.pw_matrix(kv, L, pos))
    bt = np.ascontiguousarray(ainv.T).astype(dtype)
    out = Rendering(n, sweeps)
    out.logdet, out.sign = logdet, sign
    for s in range(sweeps):
        sweep = first_sweep + s
        for e0 in range(0, n, K):
            kw = min(K, n - e0)
            prop = np.zeros((kw, 3))
            us = np.zeros(kw)
            rows = np.zeros((kw, n))
            for a in range(kw):
                g, u = oracle.move_randoms(seed, wid, sweep, spin * n + e0 + a)
                prop[a] = pos[e0 + a] + sigma * g
                us[a] = u
                rows[a] = oracle.pw_row(kv, L, prop[a])
            U = rows.astype(dtype)
            Vg = bt[e0:e0 + kw].copy()
            G = (U @ Vg.T).astype(np.float64)
            J = []
            cinv = np.zeros((0, 0))
            for a in range(kw):
                # eq. (3) by the Schur complement, with C_J^-1 kept as a
                # bordered inverse (grown by one row and column per acceptance)
                p, q = G[a, J], G[J, a]
                x, y = cinv @ q, p @ cinv
                r = G[a, a] - p @ x
                m = s * n + e0 + a
                out.ratio[m], out.u[m] = r, us[a]
                if force_accept or us[a] < r * r:
                    k = len(J)
                    grown = np.zeros((k + 1, k + 1))
                    grown[:k, :k] = cinv + np.outer(x, y) / r
                    grown[:k, k] = -x / r
                    grown[k, :k] = -y / r
                    grown[k, k] = 1.0 / r
                    cinv = grown
                    J.append(a)
                    out.accepted[m] = 1
                    out.logdet += np.log(abs(r))
                    out.sign *= 1 if r > 0 else -1
                    pos[e0 + a] = prop[a]
            if J:
                Y = bt @ U[J].T
                Y[e0 + np.asarray(J), np.arange(len(J))] -= dtype(1)
                W = Y @ cinv.T.astype(dtype)
                bt -= W @ Vg[J]
        if residual:
            a_now = oracle.pw_matrix(kv, L, pos)
            rows_r = np.arange(n) if residual_rows is None else np.asarray(residual_rows)
            x = bt.T[rows_r].astype(np.float64) @ a_now
            x[np.arange(len(rows_r)), rows_r] -= 1.0
            out.residual.append(float(np.abs(x).max()))
    out.pos, out.bt = pos, bt
    return out


def exact_ratios(n, L, seed, wid, spin, sigma, pos0, sweeps, accepted, first_sweep=0):
    """det(A_new)/det(A) of every proposal from two LAPACK LU factorisations,
    along the accept/reject path `accepted` (sweeps*n flags)."""
    kv = oracle.pw_kvectors(n)
    pos = np.array(pos0, np.float64).reshape(n, 3).copy()
    a = oracle.pw_matrix(kv, L, pos)
    s0, l0 = np.linalg.slogdet(a)
    out = np.zeros(sweeps * n)
    for sw in range(sweeps):
        for e in range(n):
            m = sw * n + e
            g, _ = oracle.move_randoms(seed, wid, first_sweep + sw, spin * n + e)
            rt = pos[e] + sigma * g
            new = a.copy()
            new[e] = oracle.pw_row(kv, L, rt)
            s1, l1 = np.linalg.slogdet(new)
            out[m] = s1 * s0 * np.exp(l1 - l0)
            if accepted[m]:
                a, pos[e], s0, l0 = new, rt, s1, l1
    return out

