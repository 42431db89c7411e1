"""ctypes binding of libdsu (include/dsu.h): argument marshalling only.

Every step of the delayed-update path runs in the HIP kernels behind the C
ABI; nothing here computes.  Importing this module does not need a GPU, but
loading the library requires the built libdsu.so next to this file -- there is
no fallback of any kind.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsu.so")

OK, EINVAL, ENOMEM, ESINGULAR, ESTATE, EDEVICE, EBUDGET = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
FLUSH_K_ACCEPTED, FLUSH_K_PROPOSED = 0, 1
FLUSH_AUTO, FLUSH_VALU, FLUSH_MFMA = 0, 1, 2
PHASE_ROWS, PHASE_G, PHASE_DECIDE, PHASE_FLUSH, PHASE_RECOMPUTE = 0, 1, 2, 3, 4
TIMING_ALL, TIMING_FLUSH = 1, 2
MAX_K = 256

_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ESINGULAR: "ESINGULAR", ESTATE: "ESTATE", EDEVICE: "EDEVICE",
          EBUDGET: "EBUDGET"}


class DsuError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Request(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("n", C.c_int32), ("spins", C.c_int32), ("seed", C.c_uint64),
                ("sigma", C.c_double), ("sweeps", C.c_int32), ("arrival_s", C.c_double),
                ("positions", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("status", C.c_int32), ("sweeps_done", C.c_int32),
                ("admit_s", C.c_double), ("finish_s", C.c_double), ("logdet", C.c_double * 2),
                ("sign", C.c_int32 * 2), ("accepted", C.c_int64)]


_lib = None

# name -> (restype, argtypes)
_vp, _i32, _i64, _dbl, _u64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64, C.c_size_t
_pd, _pi32, _pi64, _pu64, _pu8 = (C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint8))
_pvp = C.POINTER(C.c_void_p)
SIGNATURES = {
    "dsu_last_error": (C.c_char_p, []),
    "dsu_version": (C.c_int, []),
    "dsu_footprint_bytes": (_sz, [_i32, _i32, _i32]),
    "dsu_plane_wave_table": (C.c_int, [_i32, _pi32]),
    "dsu_plane_wave_rows": (C.c_int, [_i32, _dbl, _i32, _pd, _pd]),
    "dsu_walker_create": (C.c_int, [_i32, _i32, _i32, _i32, _pd, _vp, _pvp]),
    "dsu_walker_destroy": (C.c_int, [_vp]),
    "dsu_propose_ratio": (C.c_int, [_vp, _i32, _pd, _pd]),
    "dsu_propose_ratio_dev": (C.c_int, [_vp, _i32, _vp, _pd]),
    "dsu_propose_ratio_grad": (C.c_int, [_vp, _i32, _pd, _pd, _pd, _pd]),
    "dsu_eval_grad": (C.c_int, [_vp, _i32, _pd, _pd]),
    "dsu_accept": (C.c_int, [_vp]),
    "dsu_reject": (C.c_int, [_vp]),
    "dsu_flush": (C.c_int, [_vp]),
    "dsu_recompute_inverse": (C.c_int, [_vp, _pd, _pd, _pi32, _pd]),
    "dsu_get_inverse": (C.c_int, [_vp, _pd]),
    "dsu_get_logdet": (C.c_int, [_vp, _pd, _pi32]),
    "dsu_walker_pending": (C.c_int, [_vp, _pi32]),
    "dsu_walker_set_flush_kernel": (C.c_int, [_vp, _i32]),
    "dsu_walker_set_multidet": (C.c_int, [_vp, _i32, _pd, _i32, _pi32, _pi32, _pi32, _pd]),
    "dsu_propose_ratio_md": (C.c_int, [_vp, _i32, _pd, _pd, _pd, _pd]),
    "dsu_walker_md_value": (C.c_int, [_vp, _pd, _pi32]),
    "dsu_zwalker_create": (C.c_int, [_i32, _i32, _i32, _pd, _vp, _pvp]),
    "dsu_zwalker_destroy": (C.c_int, [_vp]),
    "dsu_zpropose_ratio": (C.c_int, [_vp, _i32, _pd, _pd]),
    "dsu_zaccept": (C.c_int, [_vp]),
    "dsu_zreject": (C.c_int, [_vp]),
    "dsu_zflush": (C.c_int, [_vp]),
    "dsu_zrecompute_inverse": (C.c_int, [_vp, _pd, _pd, _pd, _pd]),
    "dsu_zget_inverse": (C.c_int, [_vp, _pd]),
    "dsu_zget_logdet": (C.c_int, [_vp, _pd, _pd]),
    "dsu_zwalker_pending": (C.c_int, [_vp, _pi32]),
    "dsu_zwalker_set_flush_kernel": (C.c_int, [_vp, _i32]),
    "dsu_batch_create": (C.c_int, [_i32, _i32, _i32, _i32, _i32, _dbl, _pu64, _pu64, _pd, _pd, _i32, _vp, _pvp]),
    "dsu_batch_destroy": (C.c_int, [_vp]),
    "dsu_batch_sweep": (C.c_int, [_vp, _i32, _i32]),
    "dsu_batch_sync": (C.c_int, [_vp]),
    "dsu_batch_recompute": (C.c_int, [_vp, _pd]),
    "dsu_batch_stats": (C.c_int, [_vp, _pd, _pi32, _pi64, _pi64]),
    "dsu_batch_get_positions": (C.c_int, [_vp, _i32, _pd]),
    "dsu_batch_set_sweep": (C.c_int, [_vp, _i64]),
    "dsu_batch_set_watchdog": (C.c_int, [_vp, _i32]),
    "dsu_batch_watchdog_count": (C.c_int, [_vp, _pi64]),
    "dsu_batch_poison_row": (C.c_int, [_vp, _i32, _i32]),
    "dsu_batch_residual": (C.c_int, [_vp, _i32, _pd, _pd]),
    "dsu_batch_residual_noalloc": (C.c_int, [_vp, _i32, _pd, _pd]),
    "dsu_batch_set_residual_watchdog": (C.c_int, [_vp, _i32, _dbl]),
    "dsu_batch_accuracy": (C.c_int, [_vp, _pd, _pd, _pi64]),
    "dsu_batch_set_recompute_tiles": (C.c_int, [_vp, _i32, _i32, _i32]),
    "dsu_batch_get_recompute_tiles": (C.c_int, [_vp, _pi32, _pi32, _pi32]),
    "dsu_batch_get_inverse": (C.c_int, [_vp, _i32, _pd]),
    "dsu_batch_set_trace": (C.c_int, [_vp, _i32]),
    "dsu_batch_get_trace": (C.c_int, [_vp, _i32, _pd, _pu8]),
    "dsu_batch_set_timing": (C.c_int, [_vp, _i32]),
    "dsu_batch_kernel_time": (C.c_int, [_vp, _i32, _pi64, _pd]),
    "dsu_batch_use_graph": (C.c_int, [_vp, _i32]),
    "dsu_batch_set_delay": (C.c_int, [_vp, _i32]),
    "dsu_server_workspace_bytes": (_sz, [_i32]),
    "dsu_server_create": (C.c_int, [_i32, _i32, _dbl, _sz, _i32, _pvp]),
    "dsu_server_destroy": (C.c_int, [_vp]),
    "dsu_server_run": (C.c_int, [_vp, C.POINTER(Request), _i32, C.POINTER(Result), _pd, _i64, _pi64]),
    "dsu_server_add": (C.c_int, [_vp, C.POINTER(Request), _pi32]),
    "dsu_server_step": (C.c_int, [_vp]),
    "dsu_server_result": (C.c_int, [_vp, _i32, C.POINTER(Result), _i32]),
    "dsu_server_usage": (C.c_int, [_vp, C.POINTER(_sz), _pi32]),
}


def lib():
    """Load libdsu.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1708_00744_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise DsuError(rc, lib().dsu_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(_pd)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def footprint_bytes(n, k_delay, precision=FP32_MIXED):
    return int(lib().dsu_footprint_bytes(n, k_delay, precision))


def server_workspace_bytes(n):
    """Budget a serving pool charges for size n's recompute workspace."""
    return int(lib().dsu_server_workspace_bytes(int(n)))


def plane_wave_table(n):
    out = np.zeros((n, 4), np.int32)
    _check(lib().dsu_plane_wave_table(int(n), out.ctypes.data_as(_pi32)))
    return out


def plane_wave_rows(n, box_l, positions):
    """Orbital rows phi_j(r_c) for positions (count, 3), evaluated on the device."""
    pos = _f64(positions).reshape(-1, 3)
    rows = np.zeros((pos.shape[0], n))
    _check(lib().dsu_plane_wave_rows(int(n), float(box_l), pos.shape[0], _dp(pos), _dp(rows)))
    return rows


class Walker:
    """Host-driven single walker (dsu_walker_*)."""

    def __init__(self, slater, k_delay, precision=FP64, policy=FLUSH_K_ACCEPTED, stream=None):
        a = _f64(slater)
        n = a.shape[0]
        if a.shape != (n, n):
            raise ValueError("slater must be square")
        self.n, self.k_delay, self.precision, self.policy = n, k_delay, precision, policy
        h = C.c_void_p()
        _check(lib().dsu_walker_create(n, k_delay, precision, policy, _dp(a), _stream_ptr(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dsu_walker_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def propose(self, electron, row):
        r = C.c_double()
        _check(lib().dsu_propose_ratio(self._h, int(electron), _dp(_f64(row)), C.byref(r)))
        return r.value

    def propose_dev(self, electron, row_ptr):
        r = C.c_double()
        _check(lib().dsu_propose_ratio_dev(self._h, int(electron), C.c_void_p(row_ptr), C.byref(r)))
        return r.value

    def propose_grad(self, electron, row, drows):
        """(R, grad R) for moving `electron` to the row `row` whose gradient
        rows (3, n) are `drows`; the proposal stays pending."""
        r, g = C.c_double(), np.zeros(3)
        d = _f64(drows, (3, self.n))
        _check(lib().dsu_propose_ratio_grad(self._h, int(electron), _dp(_f64(row)), _dp(d), C.byref(r), _dp(g)))
        return r.value, g

    def grad(self, electron, drows):
        """grad_e ln|det A| at the present configuration, given the gradient
        rows (3, n) of the electron's present row."""
        g = np.zeros(3)
        _check(lib().dsu_eval_grad(self._h, int(electron), _dp(_f64(drows, (3, self.n))), _dp(g)))
        return g

    def set_multidet(self, virt, dets):
        """virt: (n, m) virtual orbitals at every electron; dets: list of
        (coef, [(occ, virt), ...]) with up to 4 substitutions each."""
        v = _f64(virt)
        nd = len(dets)
        order = np.zeros(nd, np.int32)
        occ = np.zeros((nd, 4), np.int32)
        vir = np.zeros((nd, 4), np.int32)
        coef = np.zeros(nd)
        for d, (c, subs) in enumerate(dets):
            if len(subs) > 4:
                raise ValueError("at most 4 substitutions per determinant")
            order[d], coef[d] = len(subs), c
            for q, (j, vv) in enumerate(subs):
                occ[d, q], vir[d, q] = j, vv
        _check(lib().dsu_walker_set_multidet(self._h, v.shape[1], _dp(v), nd, order.ctypes.data_as(_pi32),
                                             occ.ctypes.data_as(_pi32), vir.ctypes.data_as(_pi32), _dp(coef)))

    def propose_md(self, electron, row, vrow):
        """(Psi ratio, reference ratio) for moving `electron`; stays pending."""
        r, r0 = C.c_double(), C.c_double()
        _check(lib().dsu_propose_ratio_md(self._h, int(electron), _dp(_f64(row)), _dp(_f64(vrow)), C.byref(r),
                                          C.byref(r0)))
        return r.value, r0.value

    def md_value(self):
        la, sg = C.c_double(), C.c_int32()
        _check(lib().dsu_walker_md_value(self._h, C.byref(la), C.byref(sg)))
        return sg.value, la.value

    def accept(self):
        _check(lib().dsu_accept(self._h))

    def reject(self):
        _check(lib().dsu_reject(self._h))

    def flush(self):
        _check(lib().dsu_flush(self._h))

    def recompute(self, slater=None):
        ld, sg, dr = C.c_double(), C.c_int32(), C.c_double()
        a = None if slater is None else _dp(_f64(slater))
        _check(lib().dsu_recompute_inverse(self._h, a, C.byref(ld), C.byref(sg), C.byref(dr)))
        return ld.value, sg.value, dr.value

    def inverse(self):
        out = np.empty((self.n, self.n))
        _check(lib().dsu_get_inverse(self._h, _dp(out)))
        return out

    def logdet(self):
        ld, sg = C.c_double(), C.c_int32()
        _check(lib().dsu_get_logdet(self._h, C.byref(ld), C.byref(sg)))
        return sg.value, ld.value

    def pending(self):
        k = C.c_int32()
        _check(lib().dsu_walker_pending(self._h, C.byref(k)))
        return k.value

    def set_flush_kernel(self, mode):
        _check(lib().dsu_walker_set_flush_kernel(self._h, mode))


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _zp(a):
    """Pointer to an interleaved (re, im) complex128 array as double*."""
    return a.ctypes.data_as(_pd)


class ZWalker:
    """Host-driven single walker with complex orbitals (dsu_zwalker_*)."""

    def __init__(self, slater, k_delay, policy=FLUSH_K_ACCEPTED, stream=None):
        a = _c128(slater)
        n = a.shape[0]
        if a.shape != (n, n):
            raise ValueError("slater must be square")
        self.n, self.k_delay, self.policy = n, k_delay, policy
        h = C.c_void_p()
        _check(lib().dsu_zwalker_create(n, k_delay, policy, _zp(a), _stream_ptr(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dsu_zwalker_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def propose(self, electron, row):
        r = np.zeros(2)
        _check(lib().dsu_zpropose_ratio(self._h, int(electron), _zp(_c128(row, (self.n,))), _dp(r)))
        return complex(r[0], r[1])

    def accept(self):
        _check(lib().dsu_zaccept(self._h))

    def reject(self):
        _check(lib().dsu_zreject(self._h))

    def flush(self):
        _check(lib().dsu_zflush(self._h))

    def recompute(self, slater=None):
        la, ph, dr = C.c_double(), C.c_double(), C.c_double()
        a = None if slater is None else _zp(_c128(slater, (self.n, self.n)))
        _check(lib().dsu_zrecompute_inverse(self._h, a, C.byref(la), C.byref(ph), C.byref(dr)))
        return la.value, ph.value, dr.value

    def inverse(self):
        out = np.empty((self.n, self.n), np.complex128)
        _check(lib().dsu_zget_inverse(self._h, _zp(out)))
        return out

    def logdet(self):
        la, ph = C.c_double(), C.c_double()
        _check(lib().dsu_zget_logdet(self._h, C.byref(la), C.byref(ph)))
        return la.value, ph.value

    def pending(self):
        k = C.c_int32()
        _check(lib().dsu_zwalker_pending(self._h, C.byref(k)))
        return k.value

    def set_flush_kernel(self, mode):
        _check(lib().dsu_zwalker_set_flush_kernel(self._h, mode))


class Batch:
    """Device-driven batch of walkers of one size n (dsu_batch_*)."""

    def __init__(self, n, positions, seeds, walker_ids, sigma, k_delay, precision=FP32_MIXED, spins=1, box_l=10.0,
                 recompute_every=0, stream=None):
        seeds = np.ascontiguousarray(seeds, np.uint64)
        walkers = len(seeds)
        wids = np.ascontiguousarray(walker_ids, np.uint64)
        sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float64), (walkers,)))
        pos = _f64(positions, (walkers * spins * n * 3,))
        self.n, self.walkers, self.spins, self.ndet = n, walkers, spins, walkers * spins
        self.k_delay, self.precision = k_delay, precision
        h = C.c_void_p()
        _check(lib().dsu_batch_create(walkers, n, spins, k_delay, precision, float(box_l),
                                      seeds.ctypes.data_as(_pu64), wids.ctypes.data_as(_pu64), _dp(sig), _dp(pos),
                                      int(recompute_every), _stream_ptr(stream), C.byref(h)))
        self._h = h
        self._trace_sweeps = 0

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dsu_batch_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def sweep(self, sweeps=1, force_accept=False):
        _check(lib().dsu_batch_sweep(self._h, int(sweeps), int(bool(force_accept))))

    def sync(self):
        _check(lib().dsu_batch_sync(self._h))

    def recompute(self):
        drift = np.zeros(self.ndet)
        _check(lib().dsu_batch_recompute(self._h, _dp(drift)))
        return drift

    def stats(self):
        ld = np.zeros(self.ndet)
        sg = np.zeros(self.ndet, np.int32)
        acc = np.zeros(self.ndet, np.int64)
        sw = np.zeros(self.ndet, np.int64)
        _check(lib().dsu_batch_stats(self._h, _dp(ld), sg.ctypes.data_as(_pi32), acc.ctypes.data_as(_pi64),
                                     sw.ctypes.data_as(_pi64)))
        return {"logdet": ld, "sign": sg, "accepted": acc, "sweeps": sw}

    def set_watchdog(self, enable):
        _check(lib().dsu_batch_set_watchdog(self._h, int(bool(enable))))

    def watchdog_count(self):
        c = C.c_int64()
        _check(lib().dsu_batch_watchdog_count(self._h, C.byref(c)))
        return c.value

    def residual(self, samples=32, right=True, left=True):
        """Sampled (right, left) residuals per determinant: max |A A^-1 - I| and
        max |A^-1 A - I| over `samples` rows each (dsu_batch_residual); a side
        not asked for is None."""
        r = np.zeros(self.ndet) if right else None
        lf = np.zeros(self.ndet) if left else None
        _check(lib().dsu_batch_residual(self._h, int(samples), _dp(r) if right else None, _dp(lf) if left else None))
        return r, lf

    def residual_noalloc(self, samples=32, right=True, left=True):
        """dsu_batch_residual_noalloc: the same residuals, device buffers from
        the library's static per-GPU scratch array."""
        r = np.zeros(self.ndet) if right else None
        lf = np.zeros(self.ndet) if left else None
        _check(lib().dsu_batch_residual_noalloc(self._h, int(samples), _dp(r) if right else None,
                                                _dp(lf) if left else None))
        return r, lf

    def set_residual_watchdog(self, samples, threshold=1e-3):
        _check(lib().dsu_batch_set_residual_watchdog(self._h, int(samples), float(threshold)))

    def set_recompute_tiles(self, panel=0, chunk=0, apply_columns=0):
        """Blocking of the FP64 recompute; 0 keeps the built-in choice."""
        _check(lib().dsu_batch_set_recompute_tiles(self._h, int(panel), int(chunk), int(apply_columns)))

    def recompute_tiles(self):
        p, c, a = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().dsu_batch_get_recompute_tiles(self._h, C.byref(p), C.byref(c), C.byref(a)))
        return {"panel": p.value, "chunk": c.value, "apply_columns": a.value}

    def accuracy(self):
        """Latest sampled right residual of the residual watchdog, drift of the
        latest recompute, and the residual watchdog's recompute count."""
        res, drift = np.zeros(self.ndet), np.zeros(self.ndet)
        cnt = C.c_int64()
        _check(lib().dsu_batch_accuracy(self._h, _dp(res), _dp(drift), C.byref(cnt)))
        return {"residual": res, "drift": drift, "recomputes": cnt.value}

    def poison_row(self, det, row):
        """Test aid: NaN into one row of a determinant's device inverse."""
        _check(lib().dsu_batch_poison_row(self._h, int(det), int(row)))

    def set_sweep(self, sweeps_done):
        """Resume a checkpoint: the next sweep draws as sweep `sweeps_done`."""
        _check(lib().dsu_batch_set_sweep(self._h, int(sweeps_done)))

    def positions(self, det):
        out = np.zeros((self.n, 3))
        _check(lib().dsu_batch_get_positions(self._h, int(det), _dp(out)))
        return out

    def inverse(self, det):
        out = np.zeros((self.n, self.n))
        _check(lib().dsu_batch_get_inverse(self._h, int(det), _dp(out)))
        return out

    def set_trace(self, sweeps):
        _check(lib().dsu_batch_set_trace(self._h, int(sweeps)))
        self._trace_sweeps = int(sweeps)

    def trace(self, det):
        m = self._trace_sweeps * self.n
        r = np.zeros(m)
        a = np.zeros(m, np.uint8)
        _check(lib().dsu_batch_get_trace(self._h, int(det), _dp(r), a.ctypes.data_as(_pu8)))
        return r, a

    def set_timing(self, enable):
        """enable: False/0 off, True/TIMING_ALL every launch, TIMING_FLUSH flush launches only."""
        _check(lib().dsu_batch_set_timing(self._h, int(enable)))

    def kernel_time(self, phase):
        cnt, ms = C.c_int64(), C.c_double()
        _check(lib().dsu_batch_kernel_time(self._h, int(phase), C.byref(cnt), C.byref(ms)))
        return cnt.value, ms.value

    def use_graph(self, enable):
        _check(lib().dsu_batch_use_graph(self._h, int(bool(enable))))

    def set_delay(self, k_delay):
        _check(lib().dsu_batch_set_delay(self._h, int(k_delay)))
        self.k_delay = int(k_delay)


def _request(rid, n, spins, seed, sigma, sweeps, arrival_s, positions):
    pos = _f64(positions, (spins * n * 3,))
    r = Request(int(rid), int(n), int(spins), int(seed), float(sigma), int(sweeps), float(arrival_s),
                pos.ctypes.data_as(_pd))
    return r, pos


def _result_dict(r):
    return {"request_id": r.request_id, "status": r.status, "sweeps_done": r.sweeps_done, "admit_s": r.admit_s,
            "finish_s": r.finish_s, "logdet": [r.logdet[0], r.logdet[1]], "sign": [r.sign[0], r.sign[1]],
            "accepted": r.accepted}


class Server:
    """Serving pool (dsu_server_*): mixed-n walkers admitted by a device-memory
    budget and continuously batched."""

    def __init__(self, k_delay, precision=FP32_MIXED, box_l=10.0, budget_bytes=8 << 30, recompute_every=0):
        h = C.c_void_p()
        _check(lib().dsu_server_create(int(k_delay), int(precision), float(box_l), int(budget_bytes),
                                       int(recompute_every), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dsu_server_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add(self, rid, n, spins, seed, sigma, sweeps, positions):
        r, keep = _request(rid, n, spins, seed, sigma, sweeps, 0.0, positions)
        slot = C.c_int32()
        _check(lib().dsu_server_add(self._h, C.byref(r), C.byref(slot)))
        del keep
        return slot.value

    def step(self):
        _check(lib().dsu_server_step(self._h))

    def result(self, slot, remove=False):
        out = Result()
        _check(lib().dsu_server_result(self._h, int(slot), C.byref(out), int(bool(remove))))
        return _result_dict(out)

    def usage(self):
        used, res = C.c_size_t(), C.c_int32()
        _check(lib().dsu_server_usage(self._h, C.byref(used), C.byref(res)))
        return used.value, res.value

    def run(self, requests, latency_cap=1 << 20):
        """requests: iterable of dicts with request_id, n, spins, seed, sigma,
        sweeps, arrival_s, positions.  Returns (results, sweep latencies in ms)."""
        reqs = list(requests)
        arr = (Request * len(reqs))()
        keep = []
        for i, q in enumerate(reqs):
            r, pos = _request(q["request_id"], q["n"], q["spins"], q["seed"], q["sigma"], q["sweeps"],
                              q["arrival_s"], q["positions"])
            arr[i] = r
            keep.append(pos)
        res = (Result * len(reqs))()
        lat = np.zeros(latency_cap)
        cnt = C.c_int64()
        _check(lib().dsu_server_run(self._h, arr, len(reqs), res, _dp(lat), int(latency_cap), C.byref(cnt)))
        del keep
        return [_result_dict(r) for r in res], lat[:cnt.value]
