"""ctypes view of oracle/liboracle.so -- the sequential FP64 Sherman-Morrison
oracle of arXiv:1708.00744 (eq. (1) ratio, eq. (2) update, LU for fresh
determinants).  Test infrastructure only: the product path never imports it.

Every function here is argument marshalling; the arithmetic is in
oracle/dsu_oracle.c.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _declare(L):
    L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    L.orc_philox4x64_10.restype = None
    L.orc_uniform53.argtypes = [C.c_uint64]
    L.orc_uniform53.restype = C.c_double
    L.orc_move_randoms.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, _dp, C.POINTER(C.c_double)]
    L.orc_move_randoms.restype = None
    L.orc_pw_kvectors.argtypes = [C.c_int, _ip]
    L.orc_pw_kvectors.restype = C.c_int
    L.orc_pw_row.argtypes = [C.c_int, _ip, C.c_double, _dp, _dp]
    L.orc_pw_row.restype = None
    L.orc_pw_row_grad.argtypes = [C.c_int, _ip, C.c_double, _dp, _dp]
    L.orc_pw_row_grad.restype = None
    L.orc_pw_matrix.argtypes = [C.c_int, _ip, C.c_double, _dp, _dp]
    L.orc_pw_matrix.restype = None
    L.orc_lu.argtypes = [C.c_int, _dp, _ip, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.orc_lu.restype = C.c_int
    L.orc_slogdet.argtypes = [C.c_int, _dp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.orc_slogdet.restype = C.c_int
    L.orc_inverse.argtypes = [C.c_int, _dp, _dp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.orc_inverse.restype = C.c_int
    L.orc_residual.argtypes = [C.c_int, _dp, _dp]
    L.orc_residual.restype = C.c_double
    L.orc_residual_rows.argtypes = [C.c_int, _dp, _dp, C.c_int, _ip]
    L.orc_residual_rows.restype = C.c_double
    L.orc_residual_left_rows.argtypes = [C.c_int, _dp, _dp, C.c_int, _ip]
    L.orc_residual_left_rows.restype = C.c_double
    L.orc_sm_ratio.argtypes = [C.c_int, _dp, C.c_int, _dp]
    L.orc_sm_ratio.restype = C.c_double
    L.orc_sm_ratio_grad.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, _dp]
    L.orc_sm_ratio_grad.restype = C.c_double
    L.orc_sm_accept.argtypes = [C.c_int, _dp, C.c_void_p, C.c_int, _dp, C.c_double, _dp]
    L.orc_sm_accept.restype = None
    _zp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
    L.orc_zpw_kvectors.argtypes = [C.c_int, _dp, _ip]
    L.orc_zpw_kvectors.restype = C.c_int
    L.orc_zpw_row.argtypes = [C.c_int, _ip, _dp, C.c_double, _dp, _zp]
    L.orc_zpw_row.restype = None
    L.orc_zinverse.argtypes = [C.c_int, _zp, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.orc_zinverse.restype = C.c_int
    L.orc_zsm_ratio_out.argtypes = [C.c_int, _zp, C.c_int, _zp, _zp]
    L.orc_zsm_ratio_out.restype = None
    L.orc_zsm_accept_r.argtypes = [C.c_int, _zp, C.c_void_p, C.c_int, _zp, _zp, _zp]
    L.orc_zsm_accept_r.restype = None
    L.orc_md_psi.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_int, _ip, _ip, _ip, _dp, C.POINTER(C.c_double),
                             C.POINTER(C.c_int)]
    L.orc_md_psi.restype = C.c_int
    vp = C.c_void_p
    L.orc_walker_run.argtypes = [C.c_int, C.c_double, C.c_uint64, C.c_uint64, C.c_int, C.c_double,
                                 C.c_int, C.c_int, C.c_int, _dp,
                                 vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.orc_walker_run.restype = C.c_int
    L.orc_walkers_run.argtypes = [C.c_int, C.c_int, C.c_double, _u64p, _u64p, vp, C.c_double,
                                  C.c_int, C.c_int, C.c_int, _dp, vp, vp, vp, vp, vp, _ip]
    L.orc_walkers_run.restype = C.c_int
    L.orc_walker_moves.argtypes = [C.c_int, C.c_double, C.c_uint64, C.c_uint64, C.c_int, C.c_double, C.c_int,
                                   C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, vp]
    L.orc_walker_moves.restype = C.c_int64
    L.orc_walkers_moves.argtypes = [C.c_int, C.c_int, C.c_double, _u64p, _u64p, C.c_double, C.c_int, C.c_int,
                                    C.c_int, C.c_int, _dp, _dp, _dp, _i64p, C.c_void_p]
    L.orc_walkers_moves.restype = C.c_int


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox4x64_10(ctr, key):
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(np.ascontiguousarray(ctr, np.uint64), np.ascontiguousarray(key, np.uint64), out)
    return out


def uniform53(x):
    return lib().orc_uniform53(int(x))


def move_randoms(seed, walker, sweep, slot):
    g = np.zeros(3)
    u = C.c_double()
    lib().orc_move_randoms(seed, walker, sweep, slot, g, C.byref(u))
    return g, u.value


def pw_kvectors(n):
    out = np.zeros((n, 4), np.int32)
    rc = lib().orc_pw_kvectors(n, out)
    if rc != 0:
        raise ValueError("bad n")
    return out


def pw_row(kv, L, r):
    n = kv.shape[0]
    row = np.zeros(n)
    lib().orc_pw_row(n, np.ascontiguousarray(kv, np.int32), float(L), np.ascontiguousarray(r, np.float64), row)
    return row


def pw_row_grad(kv, L, r):
    """(3, n): d phi_j / d r_a of one plane-wave row."""
    n = kv.shape[0]
    d = np.zeros((3, n))
    lib().orc_pw_row_grad(n, np.ascontiguousarray(kv, np.int32), float(L), np.ascontiguousarray(r, np.float64), d)
    return d


def pw_matrix(kv, L, pos):
    n = kv.shape[0]
    a = np.zeros((n, n))
    lib().orc_pw_matrix(n, np.ascontiguousarray(kv, np.int32), float(L), np.ascontiguousarray(pos, np.float64), a)
    return a


def slogdet(a):
    a = np.ascontiguousarray(a, np.float64)
    ld, s = C.c_double(), C.c_int()
    rc = lib().orc_slogdet(a.shape[0], a, C.byref(ld), C.byref(s))
    if rc != 0:
        return 0, -np.inf
    return s.value, ld.value


def inverse(a):
    """(Ainv, sign, logdet); raises on an exactly singular matrix."""
    a = np.ascontiguousarray(a, np.float64)
    n = a.shape[0]
    inv = np.zeros((n, n))
    ld, s = C.c_double(), C.c_int()
    rc = lib().orc_inverse(n, a, inv, C.byref(ld), C.byref(s))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return inv, s.value, ld.value


def residual(ainv, a):
    return lib().orc_residual(a.shape[0], np.ascontiguousarray(ainv), np.ascontiguousarray(a))


def residual_rows(ainv, a, rows):
    """max |(A Ainv - I)[r, j]| over the listed rows r and all columns j."""
    rows = np.ascontiguousarray(rows, np.int32)
    return lib().orc_residual_rows(a.shape[0], np.ascontiguousarray(ainv), np.ascontiguousarray(a), len(rows), rows)


def residual_left_rows(ainv, a, rows):
    """max |(Ainv A - I)[r, j]| over the listed rows r and all columns j."""
    rows = np.ascontiguousarray(rows, np.int32)
    return lib().orc_residual_left_rows(a.shape[0], np.ascontiguousarray(ainv), np.ascontiguousarray(a), len(rows),
                                        rows)


def sm_ratio(ainv, e, phi):
    return lib().orc_sm_ratio(ainv.shape[0], np.ascontiguousarray(ainv), int(e), np.ascontiguousarray(phi, np.float64))


def sm_ratio_grad(ainv, e, phi, dphi):
    """(R, grad R) of eq. (1) for row e -> phi with gradient rows dphi (3, n)."""
    g = np.zeros(3)
    r = lib().orc_sm_ratio_grad(ainv.shape[0], np.ascontiguousarray(ainv), int(e),
                                np.ascontiguousarray(phi, np.float64), np.ascontiguousarray(dphi, np.float64), g)
    return r, g


def sm_accept(ainv, a, e, phi, r):
    """In place: Ainv <- eq. (2) update, A[e,:] <- phi (if a is not None)."""
    n = ainv.shape[0]
    assert ainv.flags.c_contiguous and ainv.dtype == np.float64
    if a is not None:
        assert a.flags.c_contiguous and a.dtype == np.float64
    work = np.zeros(2 * n)
    lib().orc_sm_accept(n, ainv, _ptr(a), int(e), np.ascontiguousarray(phi, np.float64), float(r), work)


class WalkerTrace:
    """Everything orc_walker_run reports for one walker determinant."""

    def __init__(self, n, sweeps):
        self.ratio = np.zeros(sweeps * n)
        self.u = np.zeros(sweeps * n)
        self.accepted = np.zeros(sweeps * n, np.uint8)
        self.logdet_run = np.zeros(sweeps)
        self.sign_run = np.zeros(sweeps, np.int32)
        self.logdet_fresh = np.zeros(sweeps)
        self.sign_fresh = np.zeros(sweeps, np.int32)
        self.residual = np.zeros(sweeps)
        self.pos = np.zeros((n, 3))
        self.ainv = np.zeros((n, n))
        self.n_accepted = np.zeros(1, np.int64)


def walker_run(n, L, seed, walker, spin, sigma, pos, sweeps, first_sweep=0, force_accept=False,
               residual=True, fresh=True):
    """Run `sweeps` Metropolis sweeps of one determinant (eq. (1) + eq. (2))."""
    t = WalkerTrace(n, sweeps)
    pos = np.ascontiguousarray(pos, np.float64).reshape(n, 3)
    rc = lib().orc_walker_run(n, float(L), int(seed), int(walker), int(spin), float(sigma), int(first_sweep),
                              int(sweeps), int(bool(force_accept)), pos,
                              _ptr(t.ratio), _ptr(t.u), _ptr(t.accepted), _ptr(t.logdet_run), _ptr(t.sign_run),
                              _ptr(t.logdet_fresh) if fresh else None, _ptr(t.sign_fresh) if fresh else None,
                              _ptr(t.residual) if residual else None, _ptr(t.pos), _ptr(t.ainv),
                              _ptr(t.n_accepted))
    if rc != 0:
        raise np.linalg.LinAlgError("singular start")
    return t


def walkers_run(n, L, seeds, walker_ids, spins, sigma, pos, sweeps, first_sweep=0, force_accept=False):
    """Independent determinants in OpenMP threads.  Returns (ratio[w, sweeps*n],
    accepted, logdet_run[w, sweeps], pos_out, n_accepted, threads_used)."""
    nw = len(seeds)
    seeds = np.ascontiguousarray(seeds, np.uint64)
    walker_ids = np.ascontiguousarray(walker_ids, np.uint64)
    spins = np.ascontiguousarray(spins, np.int32)
    pos = np.ascontiguousarray(pos, np.float64).reshape(nw, n * 3)
    ratio = np.zeros((nw, sweeps * n))
    acc = np.zeros((nw, sweeps * n), np.uint8)
    ld = np.zeros((nw, sweeps))
    pos_out = np.zeros((nw, n * 3))
    nacc = np.zeros(nw, np.int64)
    status = np.zeros(nw, np.int32)
    threads = lib().orc_walkers_run(nw, n, float(L), seeds, walker_ids, _ptr(spins), float(sigma), int(first_sweep),
                                    int(sweeps), int(bool(force_accept)), pos, _ptr(ratio), _ptr(acc), _ptr(ld),
                                    _ptr(pos_out), _ptr(nacc), status)
    if np.any(status != 0):
        raise np.linalg.LinAlgError("singular start")
    return ratio, acc, ld, pos_out.reshape(nw, n, 3), nacc, threads


def walker_moves(n, L, seed, walker, spin, sigma, sweep, e_first, nmoves, pos, a, ainv, force_accept=False):
    """In place on pos (n x 3), a, ainv: `nmoves` Metropolis moves from the given state.
    Returns (ratios, accepted count)."""
    for x in (pos, a, ainv):
        assert x.flags.c_contiguous and x.dtype == np.float64
    ratios = np.zeros(nmoves)
    nacc = lib().orc_walker_moves(n, float(L), int(seed), int(walker), int(spin), float(sigma), int(sweep),
                                  int(e_first), int(nmoves), int(bool(force_accept)), pos, a, ainv, _ptr(ratios))
    return ratios, nacc


def walkers_moves(n, L, seeds, walker_ids, sigma, sweep, e_first, nmoves, pos, a, ainv, force_accept=False,
                  ratios=None):
    """Many walkers (OpenMP): pos (w, n, 3), a and ainv (w, n, n), all in place;
    ratios (optional, (w, nmoves) FP64) receives every move's ratio.
    Returns (accepted per walker, threads used)."""
    nw = len(seeds)
    for x in (pos, a, ainv) + ((ratios,) if ratios is not None else ()):
        assert x.flags.c_contiguous and x.dtype == np.float64
    if ratios is not None:
        assert ratios.shape == (nw, nmoves)
    nacc = np.zeros(nw, np.int64)
    threads = lib().orc_walkers_moves(nw, n, float(L), np.ascontiguousarray(seeds, np.uint64),
                                      np.ascontiguousarray(walker_ids, np.uint64), float(sigma), int(sweep),
                                      int(e_first), int(nmoves), int(bool(force_accept)), pos, a, ainv, nacc,
                                      ratios.ctypes.data_as(C.c_void_p) if ratios is not None else None)
    return nacc, threads


# ------------------------------------------------------------- complex orbitals
def zpw_kvectors(n, theta):
    """(n, 3) integer vectors of the twisted plane waves, |n + theta|^2 ascending."""
    out = np.zeros((n, 3), np.int32)
    rc = lib().orc_zpw_kvectors(n, np.ascontiguousarray(theta, np.float64), out)
    if rc != 0:
        raise ValueError("bad n")
    return out


def zpw_row(kv, theta, L, r):
    n = kv.shape[0]
    row = np.zeros(n, np.complex128)
    lib().orc_zpw_row(n, np.ascontiguousarray(kv, np.int32), np.ascontiguousarray(theta, np.float64), float(L),
                      np.ascontiguousarray(r, np.float64), row)
    return row


def zpw_matrix(kv, theta, L, pos):
    return np.stack([zpw_row(kv, theta, L, p) for p in pos])


def zinverse(a):
    """(Ainv, log|det|, arg det); raises on an exactly singular matrix."""
    a = np.ascontiguousarray(a, np.complex128)
    n = a.shape[0]
    inv = np.zeros((n, n), np.complex128)
    la, ph = C.c_double(), C.c_double()
    rc = lib().orc_zinverse(n, a, inv.ctypes.data_as(C.c_void_p), C.byref(la), C.byref(ph))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return inv, la.value, ph.value


def zslogdet(a):
    """(log|det|, arg det) by the oracle's LU."""
    a = np.ascontiguousarray(a, np.complex128)
    la, ph = C.c_double(), C.c_double()
    rc = lib().orc_zinverse(a.shape[0], a, None, C.byref(la), C.byref(ph))
    if rc != 0:
        return -np.inf, 0.0
    return la.value, ph.value


def zsm_ratio(ainv, e, phi):
    out = np.zeros(1, np.complex128)
    lib().orc_zsm_ratio_out(ainv.shape[0], np.ascontiguousarray(ainv), int(e), np.ascontiguousarray(phi, np.complex128),
                            out)
    return complex(out[0])


def zsm_accept(ainv, a, e, phi, r):
    """In place: Ainv <- eq. (2) update, A[e,:] <- phi (if a is not None)."""
    n = ainv.shape[0]
    assert ainv.flags.c_contiguous and ainv.dtype == np.complex128
    if a is not None:
        assert a.flags.c_contiguous and a.dtype == np.complex128
    work = np.zeros(2 * n, np.complex128)
    lib().orc_zsm_accept_r(n, ainv, None if a is None else a.ctypes.data_as(C.c_void_p), int(e),
                           np.ascontiguousarray(phi, np.complex128), np.array([r], np.complex128), work)


# ------------------------------------------------------- multideterminant
def md_pack(dets):
    """dets: list of (coef, [(occ, virt), ...]) -> (order, occ, virt, coef) arrays."""
    nd = len(dets)
    order = np.zeros(nd, np.int32)
    occ = np.zeros((nd, 4), np.int32)
    virt = np.zeros((nd, 4), np.int32)
    coef = np.zeros(nd)
    for d, (c, subs) in enumerate(dets):
        order[d] = len(subs)
        coef[d] = c
        for q, (j, v) in enumerate(subs):
            occ[d, q], virt[d, q] = j, v
    return order, occ, virt, coef


def md_psi(a, v, dets):
    """(sign, log|Psi|) of Psi = sum_I c_I det(A_I) by one LU per term."""
    a = np.ascontiguousarray(a, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    order, occ, virt, coef = md_pack(dets)
    la, sg = C.c_double(), C.c_int()
    rc = lib().orc_md_psi(a.shape[0], v.shape[1], a, v, len(dets), order, np.ascontiguousarray(occ.ravel()),
                          np.ascontiguousarray(virt.ravel()), coef, C.byref(la), C.byref(sg))
    if rc != 0:
        raise ValueError("bad excitation list")
    return sg.value, la.value


def md_ratio(a, v, dets, e, phi, vphi):
    """Psi(A with row e -> phi, V with row e -> vphi) / Psi(A, V)."""
    s0, l0 = md_psi(a, v, dets)
    a1, v1 = a.copy(), v.copy()
    a1[e], v1[e] = phi, vphi
    s1, l1 = md_psi(a1, v1, dets)
    return s1 * s0 * np.exp(l1 - l0) if s1 != 0 else 0.0
