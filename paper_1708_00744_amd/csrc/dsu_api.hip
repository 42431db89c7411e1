// dsu_api.hip -- the host-driven single walker of the C ABI (include/dsu.h):
// a host state machine around three kernels (look-ahead ratio, accept with
// bordering, flush) plus the FP64 Gauss-Jordan recompute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "walker.hpp"

using namespace dsu;

using dsu::dalloc;
using dsu::dev_alloc;
using dsu::dfree;
using dsu::fail;
using dsu::GjDesc;
using dsu::GjWork;
using dsu::kpad;
using dsu::make_stream;

// ==========================================================================
// Single walker
// ==========================================================================
struct dsu_walker {
    int n = 0, np = 0, K = 0, kp = 0, prec = 0, policy = 0, flush_mode = DSU_FLUSH_AUTO;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    WalkerDev wd{};
    void *flush_desc = nullptr;     // FlushDesc<T>[1] on the device
    double **a_ptr = nullptr;       // device array {a}
    void **bt_ptr = nullptr;        // device array {bt}
    double *inv_tmp = nullptr;      // n x n FP64 for dsu_get_inverse
    double *row_stage = nullptr;    // mapped pinned host staging: proposal row, then its 3 gradient rows
    const double *row_stage_dev = nullptr;  // its device address
    double *ratio_h = nullptr;      // pinned host words the propose kernel writes R and grad R into
    GjWork gj;
    // host mirror of the state machine
    int k = 0, slots = 0;
    unsigned tag = 0;               // completion tag of the last look-ahead call
    // multideterminant expansion (FP64 walkers): table, excitations, Q
    MdDev md{};
    bool md_on = false, prop_md = false;
    double md_q = 1.0, md_q_pending = 1.0;
    double *vphi_stage = nullptr;           // mapped pinned staging of the virtual row
    const double *vphi_stage_dev = nullptr;
    std::vector<int> idx;
    bool has_prop = false;
    int prop_e = -1;
    double prop_r = 0.0;
    double logdet = 0.0;
    int sign = 1;
};

static size_t elem(int prec) { return dsu::elem_size(prec); }

static void walker_md_free(dsu_walker *w) {
    for (void *p : {(void *)w->md.v, (void *)w->md.t, (void *)w->md.c, (void *)w->md.vphi, (void *)w->md.x,
                    (void *)w->md.order, (void *)w->md.occ, (void *)w->md.virt, (void *)w->md.coef, (void *)w->md.q})
        dfree(p);
    if (w->vphi_stage) (void)hipHostFree(w->vphi_stage);
    w->vphi_stage = nullptr;
    w->vphi_stage_dev = nullptr;
    w->md = MdDev{};
    w->md_on = w->prop_md = false;
}

static void walker_free(dsu_walker *w) {
    if (w->wd.phi != (void *)w->wd.phi64) dfree(w->wd.phi);  // FP64 walkers share one row buffer
    for (void *p : {w->wd.bt, w->wd.u, w->wd.vg, (void *)w->wd.a, (void *)w->wd.phi64, (void *)w->wd.cinv,
                    (void *)w->wd.gdots,
                    (void *)w->wd.dots, (void *)w->wd.t, (void *)w->wd.ratio, (void *)w->wd.idx, (void *)w->wd.counter,
                    w->flush_desc, (void *)w->a_ptr, (void *)w->bt_ptr, (void *)w->inv_tmp})
        dfree(p);
    if (w->ratio_h) (void)hipHostFree(w->ratio_h);
    if (w->row_stage) (void)hipHostFree(w->row_stage);
    walker_md_free(w);
    w->gj.release();
    if (w->own_stream && w->stream) (void)hipStreamDestroy(w->stream);
}

static int walker_recompute(dsu_walker *w, double *fresh_logdet, int *fresh_sign) {
    HIPCHK(launch_load_transpose(w->a_ptr, w->gj.mptr, 1, w->n, w->np, w->np, w->stream));
    const GjDesc *res = nullptr;
    HIPCHK(w->gj.invert(1, w->n, w->stream, &res));
    if (w->prec == DSU_FP64)
        HIPCHK(launch_cast_perm<double>(res, reinterpret_cast<double *const *>(w->bt_ptr), 1, w->n, w->np,
                                        w->stream));
    else
        HIPCHK(launch_cast_perm<float>(res, reinterpret_cast<float *const *>(w->bt_ptr), 1, w->n, w->np,
                                       w->stream));
    double ld = 0.0;
    int sg = 0, st = 0;
    HIPCHK(hipMemcpyAsync(&ld, w->gj.logdet, sizeof(double), hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(&sg, w->gj.sign, sizeof(int), hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(&st, w->gj.status, sizeof(int), hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    if (st != 0) return fail(DSU_ESINGULAR, "Slater matrix is singular");
    *fresh_logdet = ld;
    *fresh_sign = sg;
    return DSU_OK;
}

extern "C" int dsu_walker_create(int32_t n, int32_t k_delay, int32_t precision, int32_t policy,
                                 const double *slater_host, void *hip_stream, dsu_walker **out) {
    if (!out) return fail(DSU_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 32768) return fail(DSU_EINVAL, "n = %d out of range [1, 32768]", n);
    if (k_delay < 1 || k_delay > DSU_MAX_K) return fail(DSU_EINVAL, "k_delay = %d out of range [1, %d]", k_delay, DSU_MAX_K);
    if (precision != DSU_FP64 && precision != DSU_FP32_MIXED) return fail(DSU_EINVAL, "bad precision %d", precision);
    if (policy != DSU_FLUSH_K_ACCEPTED && policy != DSU_FLUSH_K_PROPOSED) return fail(DSU_EINVAL, "bad policy %d", policy);
    if (!slater_host) return fail(DSU_EINVAL, "slater matrix is NULL");
    dsu_walker *w = new dsu_walker();
    w->n = n;
    w->np = round_up(n, 64);
    w->K = k_delay;
    w->kp = kpad(k_delay);
    w->prec = precision;
    w->policy = policy;
    int rc = DSU_OK;
    const size_t s = elem(precision), np = w->np, kp = w->kp;
#define TRY(x)                 \
    do {                       \
        rc = (x);              \
        if (rc != DSU_OK) {    \
            walker_free(w);    \
            delete w;          \
            return rc;         \
        }                      \
    } while (0)
    TRY(make_stream(hip_stream, &w->stream, &w->own_stream));
    TRY(dev_alloc(&w->wd.bt, np * np * s));
    TRY(dev_alloc(&w->wd.u, kp * np * s));
    TRY(dev_alloc(&w->wd.vg, kp * np * s));
    TRY(dalloc(&w->wd.a, np * np));
    // proposal row and its three gradient rows, contiguous (np each)
    TRY(dalloc(&w->wd.phi64, 4 * np));
    if (precision == DSU_FP64) w->wd.phi = w->wd.phi64;
    else TRY(dev_alloc(&w->wd.phi, 4 * np * s));
    w->wd.dphi = static_cast<char *>(w->wd.phi) + np * s;
    TRY(dalloc(&w->wd.gdots, 3 * (kp + 1) + kp));
    TRY(dalloc(&w->wd.cinv, kp * (kp + 1)));
    TRY(dalloc(&w->wd.dots, 1 + 2 * kp));
    TRY(dalloc(&w->wd.t, kp));
    TRY(dalloc(&w->wd.ratio, 1));
    TRY(dalloc(&w->wd.idx, kp));
    TRY(dalloc(&w->wd.counter, 1));
    w->wd.ldc = (int)kp + 1;
    // coherent: the host watches the completion tag while the kernel runs
    if (hipHostMalloc((void **)&w->ratio_h, 5 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        TRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
    std::memset(w->ratio_h, 0, 5 * sizeof(double));
    if (hipHostMalloc((void **)&w->row_stage, 4 * np * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        TRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
    {
        void *dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, w->row_stage, 0) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "hipHostGetDevicePointer failed"));
        w->row_stage_dev = static_cast<const double *>(dptr);
    }
    {
        void *dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, w->ratio_h, 0) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "hipHostGetDevicePointer failed"));
        w->wd.ratio_host = static_cast<double *>(dptr);
    }
    // pointer tables for the batched-style launchers
    TRY(dalloc(&w->a_ptr, 1));
    TRY(dalloc(&w->bt_ptr, 1));
    if (hipMemcpy(w->a_ptr, &w->wd.a, sizeof(double *), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w->bt_ptr, &w->wd.bt, sizeof(void *), hipMemcpyHostToDevice) != hipSuccess)
        TRY(fail(DSU_EDEVICE, "pointer table upload failed"));
    if (precision == DSU_FP64) {
        FlushDesc<double> fd{(double *)w->wd.bt, (const double *)w->wd.u, (const double *)w->wd.vg, w->wd.cinv,
                             w->wd.idx, w->wd.ldc};
        TRY(dev_alloc(&w->flush_desc, sizeof(fd)));
        if (hipMemcpy(w->flush_desc, &fd, sizeof(fd), hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "descriptor upload failed"));
    } else {
        FlushDesc<float> fd{(float *)w->wd.bt, (const float *)w->wd.u, (const float *)w->wd.vg, w->wd.cinv,
                            w->wd.idx, w->wd.ldc};
        TRY(dev_alloc(&w->flush_desc, sizeof(fd)));
        if (hipMemcpy(w->flush_desc, &fd, sizeof(fd), hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "descriptor upload failed"));
    }
    TRY(w->gj.alloc(1, w->np, n));
    if (hipMemcpy2D(w->wd.a, np * sizeof(double), slater_host, n * sizeof(double), n * sizeof(double), n,
                    hipMemcpyHostToDevice) != hipSuccess)
        TRY(fail(DSU_EDEVICE, "matrix upload failed"));
    TRY(walker_recompute(w, &w->logdet, &w->sign));
    w->idx.assign(w->kp, -1);
#undef TRY
    *out = w;
    return DSU_OK;
}

extern "C" int dsu_walker_destroy(dsu_walker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    (void)hipStreamSynchronize(w->stream);
    walker_free(w);
    delete w;
    return DSU_OK;
}

static int walker_do_flush(dsu_walker *w) {
    if (w->k > 0) {
        const int mode = w->flush_mode == DSU_FLUSH_VALU ? 1 : (w->flush_mode == DSU_FLUSH_MFMA ? 0 : (w->k <= 4 ? 1 : 0));
        if (w->prec == DSU_FP64)
            HIPCHK(launch_flush<double>((const FlushDesc<double> *)w->flush_desc, 1, w->n, w->np, w->k, mode, w->stream));
        else
            HIPCHK(launch_flush<float>((const FlushDesc<float> *)w->flush_desc, 1, w->n, w->np, w->k, mode, w->stream));
    }
    w->k = 0;
    w->slots = 0;
    std::fill(w->idx.begin(), w->idx.end(), -1);
    return DSU_OK;
}

extern "C" int dsu_flush(dsu_walker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    return walker_do_flush(w);
}

// Wait for the look-ahead kernel of call `tag`: it writes the tag to mapped
// host memory after its results, so watching that word returns as soon as the
// results are there.  After 2 s of no tag the stream is synchronised instead,
// which reports a failed kernel.
static int walker_wait(dsu_walker *w, unsigned tag) {
    const volatile double *h = w->ratio_h;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0;; ++spin) {
        if (h[4] == (double)tag) return DSU_OK;
        if ((spin & 4095u) == 4095u && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) break;
    }
    HIPCHK(hipStreamSynchronize(w->stream));
    if (h[4] != (double)tag) return fail(DSU_EDEVICE, "look-ahead kernel did not report");
    return DSU_OK;
}

static int walker_propose_common(dsu_walker *w, int e, double *ratio_out, double *grad_out = nullptr) {
    // an electron may hold at most one pending move: apply the window first
    for (int j = 0; j < w->k; ++j)
        if (w->idx[j] == e) {
            CHK(walker_do_flush(w));
            break;
        }
    const int gm = grad_out ? 1 : 0;
    const unsigned tag = ++w->tag;
    if (w->prec == DSU_FP64) HIPCHK(launch_walker_propose<double>(&w->wd, w->n, w->np, w->k, e, gm, -1, tag, w->stream));
    else HIPCHK(launch_walker_propose<float>(&w->wd, w->n, w->np, w->k, e, gm, -1, tag, w->stream));
    CHK(walker_wait(w, tag));
    const volatile double *h = w->ratio_h;
    const double r = h[0];
    w->has_prop = true;
    w->prop_e = e;
    w->prop_r = r;
    if (ratio_out) *ratio_out = r;
    if (grad_out)
        for (int a = 0; a < 3; ++a) grad_out[a] = h[1 + a];
    return DSU_OK;
}

// Stage `nrows` host rows (n FP64 each) at row `first` of the walker's
// 4-row block (0 = proposal, 1..3 = gradient rows), zero padded to np, and
// convert them to the walker's precision.
static int walker_stage_rows(dsu_walker *w, int first, int nrows, const double *const *rows) {
    // every earlier copy out of the staging buffer was followed on the stream
    // by a look-ahead kernel the host waited for, so the buffer is free
    const size_t np = w->np;
    double *st = w->row_stage + first * np;
    for (int r = 0; r < nrows; ++r) {
        std::memcpy(st + r * np, rows[r], sizeof(double) * w->n);
        std::memset(st + r * np + w->n, 0, sizeof(double) * (np - w->n));
    }
    // read over the host link by one small kernel (no runtime copy)
    HIPCHK(launch_rows_from_host(w->row_stage_dev + first * np, w->wd.phi64 + first * np,
                                 w->prec == DSU_FP64 ? nullptr : static_cast<float *>(w->wd.phi) + first * np,
                                 (int)(nrows * np), w->stream));
    return DSU_OK;
}

extern "C" int dsu_propose_ratio(dsu_walker *w, int32_t electron, const double *phi_host, double *ratio_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (w->md_on) return fail(DSU_ESTATE, "multideterminant walker: propose with dsu_propose_ratio_md");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_host) return fail(DSU_EINVAL, "row is NULL");
    CHK(walker_stage_rows(w, 0, 1, &phi_host));
    return walker_propose_common(w, electron, ratio_out);
}

extern "C" int dsu_propose_ratio_grad(dsu_walker *w, int32_t electron, const double *phi_host, const double *dphi_host,
                                      double *ratio_out, double *grad_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (w->md_on) return fail(DSU_ESTATE, "multideterminant walker: propose with dsu_propose_ratio_md");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_host || !dphi_host || !grad_out) return fail(DSU_EINVAL, "NULL argument");
    const double *rows[4] = {phi_host, dphi_host, dphi_host + w->n, dphi_host + 2 * (size_t)w->n};
    CHK(walker_stage_rows(w, 0, 4, rows));
    return walker_propose_common(w, electron, ratio_out, grad_out);
}

extern "C" int dsu_eval_grad(dsu_walker *w, int32_t electron, const double *dphi_host, double *grad_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!dphi_host || !grad_out) return fail(DSU_EINVAL, "NULL argument");
    const double *rows[3] = {dphi_host, dphi_host + w->n, dphi_host + 2 * (size_t)w->n};
    CHK(walker_stage_rows(w, 1, 3, rows));
    int m = -1;  // pending slot holding this electron's accepted move, if any
    for (int j = 0; j < w->k; ++j)
        if (w->idx[j] == electron) m = j;
    const unsigned tag = ++w->tag;
    if (w->prec == DSU_FP64)
        HIPCHK(launch_walker_propose<double>(&w->wd, w->n, w->np, w->k, electron, 2, m, tag, w->stream));
    else HIPCHK(launch_walker_propose<float>(&w->wd, w->n, w->np, w->k, electron, 2, m, tag, w->stream));
    CHK(walker_wait(w, tag));
    const volatile double *h = w->ratio_h;
    for (int a = 0; a < 3; ++a) grad_out[a] = h[1 + a];
    return DSU_OK;
}

extern "C" int dsu_propose_ratio_dev(dsu_walker *w, int32_t electron, const void *phi_dev, double *ratio_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (w->md_on) return fail(DSU_ESTATE, "multideterminant walker: propose with dsu_propose_ratio_md");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_dev) return fail(DSU_EINVAL, "row is NULL");
    if (w->prec == DSU_FP64) {
        HIPCHK(launch_row_to((const double *)phi_dev, w->wd.phi64, 0, w->n, w->np, w->stream));
    } else {
        HIPCHK(hipMemsetAsync(w->wd.phi, 0, sizeof(float) * w->np, w->stream));
        HIPCHK(hipMemcpyAsync(w->wd.phi, phi_dev, sizeof(float) * w->n, hipMemcpyDeviceToDevice, w->stream));
        HIPCHK(launch_row_to((const double *)w->wd.phi, w->wd.phi64, 2, w->n, w->np, w->stream));
    }
    return walker_propose_common(w, electron, ratio_out);
}

static int walker_slot_used(dsu_walker *w) {
    ++w->slots;
    const bool full = w->policy == DSU_FLUSH_K_ACCEPTED ? (w->k >= w->K) : (w->slots >= w->K);
    if (full) return walker_do_flush(w);
    return DSU_OK;
}

extern "C" int dsu_accept(dsu_walker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->has_prop) return fail(DSU_ESTATE, "no pending proposal");
    const double r = w->prop_r;
    const double floor = w->prec == DSU_FP64 ? RatioFloor<double>::value : RatioFloor<float>::value;
    if (!(std::fabs(r) > floor) || !std::isfinite(r)) return fail(DSU_ESINGULAR, "ratio %g cannot be accepted", r);
    if (w->prop_md && !(std::fabs(w->md_q_pending) > 0.0 && std::isfinite(w->md_q_pending)))
        return fail(DSU_ESINGULAR, "the expansion vanishes at the proposed configuration");
    if (w->prec == DSU_FP64) HIPCHK(launch_walker_accept<double>(&w->wd, w->n, w->np, w->k, w->kp, w->prop_e, w->stream));
    else HIPCHK(launch_walker_accept<float>(&w->wd, w->n, w->np, w->k, w->kp, w->prop_e, w->stream));
    if (w->prop_md) {
        HIPCHK(launch_md_accept(&w->md, w->n, w->np, w->prop_e, w->stream));
        w->md_q = w->md_q_pending;
        w->prop_md = false;
    }
    w->idx[w->k] = w->prop_e;
    ++w->k;
    w->logdet += std::log(std::fabs(r));
    if (r < 0) w->sign = -w->sign;
    w->has_prop = false;
    return walker_slot_used(w);
}

extern "C" int dsu_reject(dsu_walker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->has_prop) return fail(DSU_ESTATE, "no pending proposal");
    w->has_prop = false;
    w->prop_md = false;
    if (w->policy == DSU_FLUSH_K_PROPOSED) return walker_slot_used(w);
    return DSU_OK;
}

static int walker_md_refresh(dsu_walker *w);

extern "C" int dsu_recompute_inverse(dsu_walker *w, const double *slater_host_or_null, double *logdet_out,
                                     int32_t *sign_out, double *drift_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (slater_host_or_null)
        HIPCHK(hipMemcpy2DAsync(w->wd.a, w->np * sizeof(double), slater_host_or_null, w->n * sizeof(double),
                                w->n * sizeof(double), w->n, hipMemcpyHostToDevice, w->stream));
    double ld;
    int sg;
    CHK(walker_recompute(w, &ld, &sg));
    if (w->md_on) {
        if (slater_host_or_null) {
            walker_md_free(w);  // the virtual rows belong to the old configuration
        } else {
            CHK(walker_md_refresh(w));
        }
    }
    if (drift_out) *drift_out = w->logdet - ld;
    w->logdet = ld;
    w->sign = sg;
    w->k = 0;
    w->slots = 0;
    w->has_prop = false;
    std::fill(w->idx.begin(), w->idx.end(), -1);
    if (logdet_out) *logdet_out = ld;
    if (sign_out) *sign_out = sg;
    return DSU_OK;
}

extern "C" int dsu_get_inverse(dsu_walker *w, double *out_host) {
    if (!w || !out_host) return fail(DSU_EINVAL, "NULL argument");
    CHK(walker_do_flush(w));
    if (!w->inv_tmp) CHK(dalloc(&w->inv_tmp, (size_t)w->n * w->n));
    if (w->prec == DSU_FP64) HIPCHK(launch_untranspose<double>((const double *)w->wd.bt, w->inv_tmp, w->n, w->np, w->stream));
    else HIPCHK(launch_untranspose<float>((const float *)w->wd.bt, w->inv_tmp, w->n, w->np, w->stream));
    HIPCHK(hipMemcpyAsync(out_host, w->inv_tmp, sizeof(double) * w->n * w->n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    return DSU_OK;
}

extern "C" int dsu_get_logdet(dsu_walker *w, double *logdet, int32_t *sign) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (logdet) *logdet = w->logdet;
    if (sign) *sign = w->sign;
    return DSU_OK;
}

extern "C" int dsu_walker_pending(dsu_walker *w, int32_t *k_out) {
    if (!w || !k_out) return fail(DSU_EINVAL, "NULL argument");
    *k_out = w->k;
    return DSU_OK;
}

extern "C" int dsu_walker_set_flush_kernel(dsu_walker *w, int32_t mode) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (mode < DSU_FLUSH_AUTO || mode > DSU_FLUSH_MFMA) return fail(DSU_EINVAL, "bad flush mode %d", mode);
    if (mode == DSU_FLUSH_VALU && w->K > 64) return fail(DSU_EINVAL, "VALU flush supports k <= 64");
    w->flush_mode = mode;
    return DSU_OK;
}


// ==========================================================================
// Multideterminant expansion on a single reference (FP64 walkers)
// ==========================================================================
// Table T = A^{-1} V from the present (flushed) inverse, and Q of the present table.
static int walker_md_refresh(dsu_walker *w) {
    HIPCHK(launch_md_table(&w->wd, &w->md, w->n, w->np, w->stream));
    const unsigned tag = ++w->tag;
    HIPCHK(launch_md_init(&w->wd, &w->md, tag, w->stream));
    CHK(walker_wait(w, tag));
    const double q = ((const volatile double *)w->ratio_h)[2];
    if (!(std::fabs(q) > 0.0) || !std::isfinite(q)) return fail(DSU_ESINGULAR, "the expansion vanishes (Q = %g)", q);
    w->md_q = q;
    return DSU_OK;
}

extern "C" int dsu_walker_set_multidet(dsu_walker *w, int32_t m, const double *virt_host, int32_t ndet,
                                       const int32_t *order, const int32_t *occ, const int32_t *virt,
                                       const double *coef) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (w->prec != DSU_FP64) return fail(DSU_EINVAL, "multideterminant expansions need an FP64 walker");
    if (m < 1 || m > 4096) return fail(DSU_EINVAL, "m = %d out of range [1, 4096]", m);
    if (ndet < 1 || ndet > (1 << 20)) return fail(DSU_EINVAL, "ndet = %d out of range", ndet);
    if (!virt_host || !order || !occ || !virt || !coef) return fail(DSU_EINVAL, "NULL argument");
    for (int d = 0; d < ndet; ++d) {
        const int o = order[d];
        if (o < 0 || o > 4) return fail(DSU_EINVAL, "determinant %d: order %d outside [0, 4]", d, o);
        for (int a = 0; a < o; ++a) {
            const int j = occ[4 * d + a], v = virt[4 * d + a];
            if (j < 0 || j >= w->n || v < 0 || v >= m) return fail(DSU_EINVAL, "determinant %d: index out of range", d);
            for (int b = 0; b < a; ++b)
                if (occ[4 * d + b] == j || virt[4 * d + b] == v)
                    return fail(DSU_EINVAL, "determinant %d: repeated orbital", d);
        }
    }
    walker_md_free(w);
    CHK(walker_do_flush(w));
    w->has_prop = false;
    const size_t np = w->np;
    int rc = DSU_OK;
#define MDTRY(x)                  \
    do {                          \
        rc = (x);                 \
        if (rc != DSU_OK) {       \
            walker_md_free(w);    \
            return rc;            \
        }                         \
    } while (0)
    MDTRY(dalloc(&w->md.v, np * m));
    MDTRY(dalloc(&w->md.t, np * m));
    MDTRY(dalloc(&w->md.c, np));
    MDTRY(dalloc(&w->md.vphi, (size_t)m));
    MDTRY(dalloc(&w->md.x, (size_t)m));
    MDTRY(dalloc(&w->md.order, (size_t)ndet));
    MDTRY(dalloc(&w->md.occ, 4 * (size_t)ndet));
    MDTRY(dalloc(&w->md.virt, 4 * (size_t)ndet));
    MDTRY(dalloc(&w->md.coef, (size_t)ndet));
    MDTRY(dalloc(&w->md.q, 2));
    if (hipHostMalloc((void **)&w->vphi_stage, sizeof(double) * m, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        MDTRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
    {
        void *dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, w->vphi_stage, 0) != hipSuccess)
            MDTRY(fail(DSU_EDEVICE, "hipHostGetDevicePointer failed"));
        w->vphi_stage_dev = static_cast<const double *>(dptr);
    }
    w->md.m = m;
    w->md.ndet = ndet;
    if (hipMemcpy(w->md.v, virt_host, sizeof(double) * w->n * m, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w->md.order, order, sizeof(int) * ndet, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w->md.occ, occ, sizeof(int) * 4 * ndet, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w->md.virt, virt, sizeof(int) * 4 * ndet, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w->md.coef, coef, sizeof(double) * ndet, hipMemcpyHostToDevice) != hipSuccess)
        MDTRY(fail(DSU_EDEVICE, "expansion upload failed"));
    MDTRY(walker_md_refresh(w));
#undef MDTRY
    w->md_on = true;
    return DSU_OK;
}

extern "C" int dsu_propose_ratio_md(dsu_walker *w, int32_t electron, const double *phi_host, const double *vphi_host,
                                    double *ratio_out, double *ratio_ref_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->md_on) return fail(DSU_ESTATE, "no multideterminant expansion set");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_host || !vphi_host) return fail(DSU_EINVAL, "row is NULL");
    CHK(walker_stage_rows(w, 0, 1, &phi_host));
    std::memcpy(w->vphi_stage, vphi_host, sizeof(double) * w->md.m);
    HIPCHK(launch_rows_from_host(w->vphi_stage_dev, w->md.vphi, nullptr, w->md.m, w->stream));
    // an electron may hold at most one pending move: apply the window first
    for (int j = 0; j < w->k; ++j)
        if (w->idx[j] == electron) {
            CHK(walker_do_flush(w));
            break;
        }
    const unsigned t1 = ++w->tag;
    HIPCHK(launch_walker_propose<double>(&w->wd, w->n, w->np, w->k, electron, 0, -1, t1, w->stream));
    const unsigned t2 = ++w->tag;
    HIPCHK(launch_md_propose(&w->wd, &w->md, w->n, w->np, w->k, electron, t2, w->stream));
    CHK(walker_wait(w, t2));
    const volatile double *h = w->ratio_h;
    const double total = h[0], r = h[1], q = h[2];
    w->has_prop = true;
    w->prop_e = electron;
    w->prop_r = r;
    w->prop_md = true;
    w->md_q_pending = q;
    if (ratio_out) *ratio_out = total;
    if (ratio_ref_out) *ratio_ref_out = r;
    return DSU_OK;
}

extern "C" int dsu_walker_md_value(dsu_walker *w, double *logabs, int32_t *sign) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->md_on) return fail(DSU_ESTATE, "no multideterminant expansion set");
    if (logabs) *logabs = w->logdet + std::log(std::fabs(w->md_q));
    if (sign) *sign = w->md_q < 0 ? -w->sign : w->sign;
    return DSU_OK;
}
