// dsu_api.hip -- host side of libdsu: the C ABI declared in include/dsu.h.
//
// Single walker: a host state machine around three kernels (look-ahead ratio,
// accept/bordering, flush) plus the FP64 Gauss-Jordan recompute.
// Batch: lock-step windows of K proposals over many determinants; per window
// four launches (proposal rows, look-ahead products, decisions, flush).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dsu.h"
#include "dsu_internal.hpp"

using namespace dsu;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                                           \
    do {                                                                                                    \
        hipError_t e_ = (x);                                                                                \
        if (e_ != hipSuccess)                                                                               \
            return fail(e_ == hipErrorOutOfMemory ? DSU_ENOMEM : DSU_EDEVICE, "%s: %s (%s:%d)", #x,         \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                         \
    } while (0)
#define CHK(x)                          \
    do {                                \
        int r_ = (x);                   \
        if (r_ != DSU_OK) return r_;    \
    } while (0)

extern "C" const char *dsu_last_error(void) { return g_err.c_str(); }
extern "C" int dsu_version(void) { return 100; }

// Smallest supported padded delay (one of the MFMA tile-count buckets).
static int kpad(int k) {
    int p = 16;
    while (p < k) p *= 2;
    return p;
}

static int dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return DSU_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(DSU_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    e = hipMemset(*p, 0, bytes);
    if (e != hipSuccess) return fail(DSU_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
    return DSU_OK;
}
template <typename P> static int dalloc(P **p, size_t count) {
    return dev_alloc(reinterpret_cast<void **>(p), count * sizeof(P));
}
static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

// ------------------------------------------------------- plane-wave table
// Orbitals by shells s = |n|^2 = 0, 1, 2, ...; inside a shell the integer
// vectors with first nonzero component positive, in ascending (nx, ny, nz);
// n = 0 gives the constant, every other vector cos then sin.
int dsu::build_kvectors(int n, int4 *out) {
    if (n <= 0) return -1;
    int j = 0;
    out[j++] = make_int4(0, 0, 0, 0);
    for (int s = 1; j < n; ++s) {
        const int r = (int)std::floor(std::sqrt((double)s)) + 1;
        for (int x = -r; x <= r && j < n; ++x)
            for (int y = -r; y <= r && j < n; ++y) {
                const int rest = s - x * x - y * y;
                if (rest < 0) continue;
                const int z0 = (int)std::lround(std::sqrt((double)rest));
                if (z0 * z0 != rest) continue;
                const int zs[2] = {-z0, z0};
                for (int q = 0; q < (z0 == 0 ? 1 : 2) && j < n; ++q) {
                    const int z = zs[q];
                    const bool rep = x > 0 || (x == 0 && (y > 0 || (y == 0 && z > 0)));
                    if (!rep) continue;
                    out[j++] = make_int4(x, y, z, 1);
                    if (j < n) out[j++] = make_int4(x, y, z, 2);
                }
            }
    }
    return 0;
}

// -------------------------------------------------- Gauss-Jordan workspace
struct GjWork {
    int g = 0, np = 0, nb = 32;
    double *m = nullptr, *panel = nullptr, *w = nullptr, *q = nullptr, *logdet = nullptr;
    int *piv = nullptr, *perm = nullptr, *sign = nullptr, *status = nullptr;
    GjDesc *gdesc = nullptr;
    RankDesc *rdesc = nullptr;
    double **mptr = nullptr;
    int alloc(int groups, int np_, int n) {
        g = groups;
        np = np_;
        nb = n >= 512 ? 64 : (n >= 64 ? 32 : 16);
        const size_t np2 = (size_t)np * np;
        CHK(dalloc(&m, np2 * g));
        CHK(dalloc(&panel, (size_t)np * nb * g));
        CHK(dalloc(&w, (size_t)np * nb * g));
        CHK(dalloc(&q, (size_t)np * nb * g));
        CHK(dalloc(&logdet, g));
        CHK(dalloc(&piv, (size_t)np * g));
        CHK(dalloc(&perm, (size_t)np * g));
        CHK(dalloc(&sign, g));
        CHK(dalloc(&status, g));
        CHK(dalloc(&gdesc, g));
        CHK(dalloc(&rdesc, g));
        CHK(dalloc(&mptr, g));
        std::vector<GjDesc> gd(g);
        std::vector<RankDesc> rd(g);
        std::vector<double *> mp(g);
        for (int i = 0; i < g; ++i) {
            gd[i] = GjDesc{m + np2 * i, panel + (size_t)np * nb * i, w + (size_t)np * nb * i,
                           q + (size_t)np * nb * i, piv + (size_t)np * i, perm + (size_t)np * i,
                           logdet + i, sign + i, status + i};
            rd[i] = RankDesc{gd[i].m, gd[i].w, gd[i].q};
            mp[i] = gd[i].m;
        }
        HIPCHK(hipMemcpy(gdesc, gd.data(), sizeof(GjDesc) * g, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(rdesc, rd.data(), sizeof(RankDesc) * g, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(mptr, mp.data(), sizeof(double *) * g, hipMemcpyHostToDevice));
        return DSU_OK;
    }
    void release() {
        for (void *p : {(void *)m, (void *)panel, (void *)w, (void *)q, (void *)logdet, (void *)piv, (void *)perm,
                        (void *)sign, (void *)status, (void *)gdesc, (void *)rdesc, (void *)mptr})
            dfree(p);
        m = panel = w = q = logdet = nullptr;
        piv = perm = sign = status = nullptr;
        gdesc = nullptr;
        rdesc = nullptr;
        mptr = nullptr;
    }
};

static int make_stream(void *given, hipStream_t *s, bool *own) {
    if (given) {
        *s = (hipStream_t)given;
        *own = false;
        return DSU_OK;
    }
    HIPCHK(hipStreamCreateWithFlags(s, hipStreamNonBlocking));
    *own = true;
    return DSU_OK;
}

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
    double *row_stage = nullptr;    // pinned host staging for proposal rows
    double *ratio_h = nullptr;      // pinned host word the propose kernel writes R into
    GjWork gj;
    // host mirror of the state machine
    int k = 0, slots = 0;
    std::vector<int> idx;
    bool has_prop = false;
    int prop_e = -1;
    double prop_r = 0.0;
    double logdet = 0.0;
    int sign = 1;
};

static size_t elem(int prec) { return prec == DSU_FP64 ? sizeof(double) : sizeof(float); }

static void walker_free(dsu_walker *w) {
    for (void *p : {w->wd.bt, w->wd.u, w->wd.vg, (void *)w->wd.a, w->wd.phi, (void *)w->wd.phi64, (void *)w->wd.cinv,
                    (void *)w->wd.dots, (void *)w->wd.t, (void *)w->wd.ratio, (void *)w->wd.idx, (void *)w->wd.counter,
                    w->flush_desc, (void *)w->a_ptr, (void *)w->bt_ptr, (void *)w->inv_tmp})
        dfree(p);
    if (w->ratio_h) (void)hipHostFree(w->ratio_h);
    if (w->row_stage) (void)hipHostFree(w->row_stage);
    w->gj.release();
    if (w->own_stream && w->stream) (void)hipStreamDestroy(w->stream);
}

static int walker_recompute(dsu_walker *w, double *fresh_logdet, int *fresh_sign) {
    HIPCHK(launch_load_transpose(w->a_ptr, w->gj.mptr, 1, w->n, w->np, w->np, w->stream));
    HIPCHK(launch_gj_invert(w->gj.gdesc, w->gj.rdesc, 1, w->n, w->np, w->gj.nb, w->stream));
    if (w->prec == DSU_FP64)
        HIPCHK(launch_cast_perm<double>(w->gj.gdesc, reinterpret_cast<double *const *>(w->bt_ptr), 1, w->n, w->np,
                                        w->stream));
    else
        HIPCHK(launch_cast_perm<float>(w->gj.gdesc, reinterpret_cast<float *const *>(w->bt_ptr), 1, w->n, w->np,
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
    TRY(dalloc(&w->wd.phi64, np));
    if (precision == DSU_FP64) w->wd.phi = w->wd.phi64;
    else TRY(dev_alloc(&w->wd.phi, np * s));
    TRY(dalloc(&w->wd.cinv, kp * (kp + 1)));
    TRY(dalloc(&w->wd.dots, 1 + 2 * kp));
    TRY(dalloc(&w->wd.t, kp));
    TRY(dalloc(&w->wd.ratio, 1));
    TRY(dalloc(&w->wd.idx, kp));
    TRY(dalloc(&w->wd.counter, 1));
    w->wd.ldc = (int)kp + 1;
    if (hipHostMalloc((void **)&w->ratio_h, sizeof(double), hipHostMallocMapped) != hipSuccess)
        TRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
    if (hipHostMalloc((void **)&w->row_stage, np * sizeof(double), hipHostMallocDefault) != hipSuccess)
        TRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
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

static int walker_propose_common(dsu_walker *w, int e, double *ratio_out) {
    // an electron may hold at most one pending move: apply the window first
    for (int j = 0; j < w->k; ++j)
        if (w->idx[j] == e) {
            CHK(walker_do_flush(w));
            break;
        }
    if (w->prec == DSU_FP64) HIPCHK(launch_walker_propose<double>(&w->wd, w->n, w->np, w->k, e, w->stream));
    else HIPCHK(launch_walker_propose<float>(&w->wd, w->n, w->np, w->k, e, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    const double r = *(volatile double *)w->ratio_h;
    w->has_prop = true;
    w->prop_e = e;
    w->prop_r = r;
    if (ratio_out) *ratio_out = r;
    return DSU_OK;
}

extern "C" int dsu_propose_ratio(dsu_walker *w, int32_t electron, const double *phi_host, double *ratio_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_host) return fail(DSU_EINVAL, "row is NULL");
    // the staging buffer may still feed a previous copy: wait for the stream
    HIPCHK(hipStreamSynchronize(w->stream));
    std::memcpy(w->row_stage, phi_host, sizeof(double) * w->n);
    std::memset(w->row_stage + w->n, 0, sizeof(double) * (w->np - w->n));
    HIPCHK(hipMemcpyAsync(w->wd.phi64, w->row_stage, sizeof(double) * w->np, hipMemcpyHostToDevice, w->stream));
    if (w->prec != DSU_FP64) HIPCHK(launch_row_to(w->wd.phi64, w->wd.phi, 1, w->n, w->np, w->stream));
    return walker_propose_common(w, electron, ratio_out);
}

extern "C" int dsu_propose_ratio_dev(dsu_walker *w, int32_t electron, const void *phi_dev, double *ratio_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
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
    if (!(std::isfinite(r)) || r == 0.0) return fail(DSU_ESINGULAR, "ratio %g cannot be accepted", r);
    if (w->prec == DSU_FP64) HIPCHK(launch_walker_accept<double>(&w->wd, w->n, w->np, w->k, w->kp, w->prop_e, w->stream));
    else HIPCHK(launch_walker_accept<float>(&w->wd, w->n, w->np, w->k, w->kp, w->prop_e, w->stream));
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
    if (w->policy == DSU_FLUSH_K_PROPOSED) return walker_slot_used(w);
    return DSU_OK;
}

extern "C" int dsu_recompute_inverse(dsu_walker *w, const double *slater_host_or_null, double *logdet_out,
                                     int32_t *sign_out, double *drift_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (slater_host_or_null)
        HIPCHK(hipMemcpy2DAsync(w->wd.a, w->np * sizeof(double), slater_host_or_null, w->n * sizeof(double),
                                w->n * sizeof(double), w->n, hipMemcpyHostToDevice, w->stream));
    double ld;
    int sg;
    CHK(walker_recompute(w, &ld, &sg));
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
// Batched form
// ==========================================================================
static int choose_nsplit(int np) {
    int s = np / 512;
    if (s < 1) s = 1;
    while (s > 1 && (np % s != 0 || (np / s) % 64 != 0)) --s;
    return s;
}

extern "C" size_t dsu_footprint_bytes(int32_t n, int32_t k_delay, int32_t precision) {
    if (n < 1 || k_delay < 1 || k_delay > DSU_MAX_K || (precision != DSU_FP64 && precision != DSU_FP32_MIXED)) return 0;
    const size_t s = elem(precision), np = round_up(n, 64), kp = kpad(k_delay);
    const size_t nsplit = choose_nsplit((int)np);
    size_t b = np * np * s + 2 * kp * np * s + nsplit * kp * kp * s + kp * kp * 8 + kp * 4 * 8 + (size_t)n * 3 * 8 +
               kp * 4 + sizeof(DetState);
    if (kp > 64) b += kp * (kp + 1) * 8;   // G outside LDS
    if (kp > 128) b += kp * (kp + 1) * 8;  // C^{-1} outside LDS
    return b;
}

enum { PH_ROWS = 0, PH_G = 1, PH_DECIDE = 2, PH_FLUSH = 3, PH_RECOMPUTE = 4, PH_COUNT = 5 };

struct dsu_batch {
    int walkers = 0, spins = 1, ndet = 0, n = 0, np = 0, K = 0, kp = 0, prec = 0, recompute_every = 0, nsplit = 1;
    double L = 0, twopi_l = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // per-determinant arrays, determinant-major
    void *bt = nullptr, *u = nullptr, *vg = nullptr, *gpart = nullptr;
    double *cfl = nullptr, *cwork = nullptr, *gwork = nullptr, *prop = nullptr, *pos = nullptr;
    int *idx = nullptr;
    DetState *st = nullptr;
    int4 *kvec = nullptr;
    void *ddesc = nullptr, *fdesc = nullptr;
    double **pos_ptr = nullptr;
    void **bt_ptr = nullptr;
    double *drift = nullptr;
    double *inv_tmp = nullptr;
    GjWork gj;
    // trace
    double *trace_r = nullptr;
    uint8_t *trace_a = nullptr;
    long long trace_cap = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    long long t_count[PH_COUNT] = {0};
    double t_ms[PH_COUNT] = {0};
    // graph
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_force = -1;
    long long sweeps_done = 0;
};

template <typename T> static void fill_descs(dsu_batch *b, std::vector<DetDesc<T>> &dd, std::vector<FlushDesc<T>> &fd,
                                             const uint64_t *seeds, const uint64_t *wids, const double *sigma) {
    const size_t np = b->np, kp = b->kp;
    dd.resize(b->ndet);
    fd.resize(b->ndet);
    for (int i = 0; i < b->ndet; ++i) {
        const int w = i / b->spins;
        DetDesc<T> &d = dd[i];
        d.bt = (T *)b->bt + np * np * i;
        d.u = (T *)b->u + kp * np * i;
        d.vg = (T *)b->vg + kp * np * i;
        d.gpart = (T *)b->gpart + (size_t)b->nsplit * kp * kp * i;
        d.cfl = b->cfl + kp * kp * i;
        d.cwork = b->cwork ? b->cwork + kp * (kp + 1) * i : nullptr;
        d.gwork = b->gwork ? b->gwork + kp * (kp + 1) * i : nullptr;
        d.prop = b->prop + kp * 4 * i;
        d.pos = b->pos + (size_t)b->n * 3 * i;
        d.idx = b->idx + kp * i;
        d.st = b->st + i;
        d.trace_r = nullptr;
        d.trace_a = nullptr;
        d.trace_cap = 0;
        d.seed = seeds[w];
        d.wid = wids[w];
        d.sigma = sigma[w];
        d.spin = i % b->spins;
        fd[i] = FlushDesc<T>{d.bt, d.u, d.vg, d.cfl, d.idx, (int)kp};
    }
}

static void batch_free(dsu_batch *b) {
    for (void *p : {b->bt, b->u, b->vg, b->gpart, (void *)b->cfl, (void *)b->cwork, (void *)b->gwork, (void *)b->prop,
                    (void *)b->pos, (void *)b->idx, (void *)b->st, (void *)b->kvec, b->ddesc, b->fdesc,
                    (void *)b->pos_ptr, (void *)b->bt_ptr, (void *)b->drift, (void *)b->inv_tmp, (void *)b->trace_r,
                    (void *)b->trace_a})
        dfree(p);
    b->gj.release();
    for (auto &e : b->ev_free) (void)hipEventDestroy(e);
    for (auto &e : b->ev_used) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

static int ev_get(dsu_batch *b, hipEvent_t *e) {
    if (!b->ev_free.empty()) {
        *e = b->ev_free.back();
        b->ev_free.pop_back();
        return DSU_OK;
    }
    HIPCHK(hipEventCreate(e));
    return DSU_OK;
}

// Launch `fn` on the batch stream, bracketed by events when timing is on.
template <typename F> static int timed(dsu_batch *b, int phase, F fn) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing) {
        CHK(ev_get(b, &e0));
        CHK(ev_get(b, &e1));
        HIPCHK(hipEventRecord(e0, b->stream));
    }
    HIPCHK(fn());
    if (b->timing) {
        HIPCHK(hipEventRecord(e1, b->stream));
        b->ev_used.push_back({phase, {e0, e1}});
    }
    return DSU_OK;
}

static int batch_harvest_events(dsu_batch *b) {
    if (b->ev_used.empty()) return DSU_OK;
    HIPCHK(hipStreamSynchronize(b->stream));
    for (auto &e : b->ev_used) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e.second.first, e.second.second));
        b->t_ms[e.first] += ms;
        b->t_count[e.first] += 1;
        b->ev_free.push_back(e.second.first);
        b->ev_free.push_back(e.second.second);
    }
    b->ev_used.clear();
    return DSU_OK;
}

template <typename T> static int batch_recompute_t(dsu_batch *b, bool want_drift) {
    const DetDesc<T> *dd = (const DetDesc<T> *)b->ddesc;
    for (int g0 = 0; g0 < b->ndet; g0 += b->gj.g) {
        const int cnt = std::min(b->gj.g, b->ndet - g0);
        CHK(timed(b, PH_RECOMPUTE, [&] {
            hipError_t e = launch_build_pw_transpose(b->pos_ptr + g0, b->gj.mptr, cnt, b->n, b->np, b->kvec, b->twopi_l,
                                                     b->stream);
            if (e != hipSuccess) return e;
            e = launch_gj_invert(b->gj.gdesc, b->gj.rdesc, cnt, b->n, b->np, b->gj.nb, b->stream);
            if (e != hipSuccess) return e;
            e = launch_cast_perm<T>(b->gj.gdesc, (T *const *)(b->bt_ptr + g0), cnt, b->n, b->np, b->stream);
            if (e != hipSuccess) return e;
            return launch_reset_state<T>(dd + g0, b->gj.gdesc, want_drift ? b->drift + g0 : nullptr, cnt, b->stream);
        }));
        std::vector<int> st(cnt);
        HIPCHK(hipMemcpyAsync(st.data(), b->gj.status, sizeof(int) * cnt, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        for (int i = 0; i < cnt; ++i)
            if (st[i] != 0) return fail(DSU_ESINGULAR, "determinant %d: Slater matrix is singular", g0 + i);
    }
    return DSU_OK;
}

static int batch_recompute(dsu_batch *b, bool want_drift) {
    return b->prec == DSU_FP64 ? batch_recompute_t<double>(b, want_drift) : batch_recompute_t<float>(b, want_drift);
}

template <typename T> static int batch_enqueue_sweep_t(dsu_batch *b, int force) {
    const DetDesc<T> *dd = (const DetDesc<T> *)b->ddesc;
    const FlushDesc<T> *fd = (const FlushDesc<T> *)b->fdesc;
    for (int e0 = 0; e0 < b->n; e0 += b->K) {
        const int kw = std::min(b->K, b->n - e0);
        const int last = e0 + kw == b->n;
        CHK(timed(b, PH_ROWS, [&] {
            return launch_window_rows<T>(dd, b->ndet, b->n, b->np, b->kp, e0, kw, b->kvec, b->twopi_l, b->L, b->stream);
        }));
        CHK(timed(b, PH_G, [&] { return launch_window_g<T>(dd, b->ndet, b->n, b->np, b->kp, e0, kw, b->nsplit, b->stream); }));
        CHK(timed(b, PH_DECIDE, [&] {
            return launch_window_decide<T>(dd, b->ndet, b->n, b->kp, e0, kw, b->nsplit, force, last, b->stream);
        }));
        CHK(timed(b, PH_FLUSH, [&] { return launch_window_flush<T>(dd, fd, b->ndet, b->n, b->np, kw, b->stream); }));
    }
    return DSU_OK;
}

static int batch_enqueue_sweep(dsu_batch *b, int force) {
    return b->prec == DSU_FP64 ? batch_enqueue_sweep_t<double>(b, force) : batch_enqueue_sweep_t<float>(b, force);
}

extern "C" int dsu_batch_create(int32_t walkers, int32_t n, int32_t spins, int32_t k_delay, int32_t precision,
                                double box_L, const uint64_t *seeds, const uint64_t *walker_ids, const double *sigma,
                                const double *positions_host, int32_t recompute_every, void *hip_stream,
                                dsu_batch **out) {
    if (!out) return fail(DSU_EINVAL, "out is NULL");
    *out = nullptr;
    if (walkers < 1) return fail(DSU_EINVAL, "walkers = %d", walkers);
    if (n < 1 || n > 32768) return fail(DSU_EINVAL, "n = %d out of range [1, 32768]", n);
    if (spins != 1 && spins != 2) return fail(DSU_EINVAL, "spins must be 1 or 2");
    if (k_delay < 1 || k_delay > DSU_MAX_K) return fail(DSU_EINVAL, "k_delay = %d out of range [1, %d]", k_delay, DSU_MAX_K);
    if (precision != DSU_FP64 && precision != DSU_FP32_MIXED) return fail(DSU_EINVAL, "bad precision %d", precision);
    if (!(box_L > 0)) return fail(DSU_EINVAL, "box_L must be positive");
    if (!seeds || !walker_ids || !sigma || !positions_host) return fail(DSU_EINVAL, "NULL input array");
    if (recompute_every < 0) return fail(DSU_EINVAL, "recompute_every < 0");
    dsu_batch *b = new dsu_batch();
    b->walkers = walkers;
    b->spins = spins;
    b->ndet = walkers * spins;
    b->n = n;
    b->np = round_up(n, 64);
    b->K = k_delay;
    b->kp = kpad(k_delay);
    b->prec = precision;
    b->recompute_every = recompute_every;
    b->nsplit = choose_nsplit(b->np);
    b->L = box_L;
    b->twopi_l = 2.0 * M_PI / box_L;
    int rc = DSU_OK;
#define TRY(x)               \
    do {                     \
        rc = (x);            \
        if (rc != DSU_OK) {  \
            batch_free(b);   \
            delete b;        \
            return rc;       \
        }                    \
    } while (0)
    const size_t s = elem(precision), np = b->np, kp = b->kp, nd = b->ndet;
    TRY(make_stream(hip_stream, &b->stream, &b->own_stream));
    TRY(dev_alloc(&b->bt, nd * np * np * s));
    TRY(dev_alloc(&b->u, nd * kp * np * s));
    TRY(dev_alloc(&b->vg, nd * kp * np * s));
    TRY(dev_alloc(&b->gpart, nd * b->nsplit * kp * kp * s));
    TRY(dalloc(&b->cfl, nd * kp * kp));
    if (kp > 128) TRY(dalloc(&b->cwork, nd * kp * (kp + 1)));
    if (kp > 64) TRY(dalloc(&b->gwork, nd * kp * (kp + 1)));
    TRY(dalloc(&b->prop, nd * kp * 4));
    TRY(dalloc(&b->pos, nd * (size_t)n * 3));
    TRY(dalloc(&b->idx, nd * kp));
    TRY(dalloc(&b->st, nd));
    TRY(dalloc(&b->kvec, (size_t)n));
    TRY(dalloc(&b->pos_ptr, nd));
    TRY(dalloc(&b->bt_ptr, nd));
    TRY(dalloc(&b->drift, nd));
    {
        std::vector<int4> kv(n);
        build_kvectors(n, kv.data());
        if (hipMemcpy(b->kvec, kv.data(), sizeof(int4) * n, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "kvec upload failed"));
        if (hipMemcpy(b->pos, positions_host, sizeof(double) * nd * n * 3, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "positions upload failed"));
        std::vector<double *> pp(nd);
        std::vector<void *> bp(nd);
        for (size_t i = 0; i < nd; ++i) {
            pp[i] = b->pos + (size_t)n * 3 * i;
            bp[i] = (char *)b->bt + np * np * s * i;
        }
        if (hipMemcpy(b->pos_ptr, pp.data(), sizeof(double *) * nd, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->bt_ptr, bp.data(), sizeof(void *) * nd, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "pointer table upload failed"));
        std::vector<DetState> st(nd);
        for (auto &x : st) x = DetState{0.0, 1, 0, 0, 0, 0};
        if (hipMemcpy(b->st, st.data(), sizeof(DetState) * nd, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "state upload failed"));
    }
    if (precision == DSU_FP64) {
        std::vector<DetDesc<double>> dd;
        std::vector<FlushDesc<double>> fd;
        fill_descs<double>(b, dd, fd, seeds, walker_ids, sigma);
        TRY(dev_alloc(&b->ddesc, sizeof(dd[0]) * nd));
        TRY(dev_alloc(&b->fdesc, sizeof(fd[0]) * nd));
        if (hipMemcpy(b->ddesc, dd.data(), sizeof(dd[0]) * nd, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->fdesc, fd.data(), sizeof(fd[0]) * nd, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "descriptor upload failed"));
    } else {
        std::vector<DetDesc<float>> dd;
        std::vector<FlushDesc<float>> fd;
        fill_descs<float>(b, dd, fd, seeds, walker_ids, sigma);
        TRY(dev_alloc(&b->ddesc, sizeof(dd[0]) * nd));
        TRY(dev_alloc(&b->fdesc, sizeof(fd[0]) * nd));
        if (hipMemcpy(b->ddesc, dd.data(), sizeof(dd[0]) * nd, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->fdesc, fd.data(), sizeof(fd[0]) * nd, hipMemcpyHostToDevice) != hipSuccess)
            TRY(fail(DSU_EDEVICE, "descriptor upload failed"));
    }
    // recompute workspace: as many determinants at once as fit in ~8 GiB
    {
        const size_t per = np * np * 8 + np * 64 * 8 * 3;
        size_t g = (size_t)8 << 30;
        g = std::max<size_t>(1, g / per);
        g = std::min<size_t>(g, nd);
        TRY(b->gj.alloc((int)g, b->np, n));
    }
    TRY(batch_recompute(b, false));
#undef TRY
    *out = b;
    return DSU_OK;
}

extern "C" int dsu_batch_destroy(dsu_batch *b) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
    return DSU_OK;
}

static int batch_build_graph(dsu_batch *b, int force) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const bool tm = b->timing;
    b->timing = false;
    int rc = batch_enqueue_sweep(b, force);
    b->timing = tm;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != DSU_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(DSU_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_force = force;
    return DSU_OK;
}

extern "C" int dsu_batch_sweep(dsu_batch *b, int32_t sweeps, int32_t force_accept) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (sweeps < 0) return fail(DSU_EINVAL, "sweeps < 0");
    const int force = force_accept ? 1 : 0;
    for (int s = 0; s < sweeps; ++s) {
        if (b->recompute_every > 0 && b->sweeps_done > 0 && b->sweeps_done % b->recompute_every == 0)
            CHK(batch_recompute(b, false));
        if (b->use_graph && !b->timing) {
            if (!b->gexec || b->graph_force != force) CHK(batch_build_graph(b, force));
            HIPCHK(hipGraphLaunch(b->gexec, b->stream));
        } else {
            CHK(batch_enqueue_sweep(b, force));
        }
        ++b->sweeps_done;
    }
    return DSU_OK;
}

extern "C" int dsu_batch_sync(dsu_batch *b) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->stream));
    return DSU_OK;
}

extern "C" int dsu_batch_recompute(dsu_batch *b, double *drift_out) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    CHK(batch_recompute(b, drift_out != nullptr));
    if (drift_out) {
        HIPCHK(hipMemcpyAsync(drift_out, b->drift, sizeof(double) * b->ndet, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return DSU_OK;
}

extern "C" int dsu_batch_stats(dsu_batch *b, double *logdet, int32_t *sign, int64_t *accepted, int64_t *sweeps_done) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    std::vector<DetState> st(b->ndet);
    HIPCHK(hipMemcpyAsync(st.data(), b->st, sizeof(DetState) * b->ndet, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->ndet; ++i) {
        if (logdet) logdet[i] = st[i].logdet;
        if (sign) sign[i] = st[i].sign;
        if (accepted) accepted[i] = st[i].accepted;
        if (sweeps_done) sweeps_done[i] = st[i].sweep;
    }
    return DSU_OK;
}

extern "C" int dsu_batch_get_positions(dsu_batch *b, int32_t det, double *out_host) {
    if (!b || !out_host) return fail(DSU_EINVAL, "NULL argument");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    HIPCHK(hipMemcpyAsync(out_host, b->pos + (size_t)b->n * 3 * det, sizeof(double) * b->n * 3, hipMemcpyDeviceToHost,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DSU_OK;
}

extern "C" int dsu_batch_get_inverse(dsu_batch *b, int32_t det, double *out_host) {
    if (!b || !out_host) return fail(DSU_EINVAL, "NULL argument");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    if (!b->inv_tmp) CHK(dalloc(&b->inv_tmp, (size_t)b->n * b->n));
    const size_t off = (size_t)b->np * b->np * det;
    if (b->prec == DSU_FP64)
        HIPCHK(launch_untranspose<double>((const double *)b->bt + off, b->inv_tmp, b->n, b->np, b->stream));
    else
        HIPCHK(launch_untranspose<float>((const float *)b->bt + off, b->inv_tmp, b->n, b->np, b->stream));
    HIPCHK(hipMemcpyAsync(out_host, b->inv_tmp, sizeof(double) * b->n * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DSU_OK;
}

template <typename T> static int batch_set_trace_t(dsu_batch *b) {
    std::vector<DetDesc<T>> dd(b->ndet);
    HIPCHK(hipMemcpy(dd.data(), b->ddesc, sizeof(dd[0]) * b->ndet, hipMemcpyDeviceToHost));
    for (int i = 0; i < b->ndet; ++i) {
        dd[i].trace_r = b->trace_r ? b->trace_r + (size_t)b->trace_cap * i : nullptr;
        dd[i].trace_a = b->trace_a ? b->trace_a + (size_t)b->trace_cap * i : nullptr;
        dd[i].trace_cap = b->trace_r ? b->trace_cap : 0;
    }
    HIPCHK(hipMemcpy(b->ddesc, dd.data(), sizeof(dd[0]) * b->ndet, hipMemcpyHostToDevice));
    return DSU_OK;
}

extern "C" int dsu_batch_set_trace(dsu_batch *b, int32_t sweeps) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (sweeps < 0) return fail(DSU_EINVAL, "sweeps < 0");
    HIPCHK(hipStreamSynchronize(b->stream));
    dfree(b->trace_r);
    dfree(b->trace_a);
    b->trace_r = nullptr;
    b->trace_a = nullptr;
    b->trace_cap = (long long)sweeps * b->n;
    if (sweeps > 0) {
        CHK(dalloc(&b->trace_r, (size_t)b->trace_cap * b->ndet));
        CHK(dalloc(&b->trace_a, (size_t)b->trace_cap * b->ndet));
    }
    std::vector<DetState> st(b->ndet);
    HIPCHK(hipMemcpy(st.data(), b->st, sizeof(DetState) * b->ndet, hipMemcpyDeviceToHost));
    for (auto &x : st) x.trace_pos = 0;
    HIPCHK(hipMemcpy(b->st, st.data(), sizeof(DetState) * b->ndet, hipMemcpyHostToDevice));
    return b->prec == DSU_FP64 ? batch_set_trace_t<double>(b) : batch_set_trace_t<float>(b);
}

extern "C" int dsu_batch_get_trace(dsu_batch *b, int32_t det, double *ratio_host, uint8_t *accepted_host) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    if (!b->trace_r) return fail(DSU_ESTATE, "tracing is off");
    if (ratio_host)
        HIPCHK(hipMemcpyAsync(ratio_host, b->trace_r + (size_t)b->trace_cap * det, sizeof(double) * b->trace_cap,
                              hipMemcpyDeviceToHost, b->stream));
    if (accepted_host)
        HIPCHK(hipMemcpyAsync(accepted_host, b->trace_a + (size_t)b->trace_cap * det, b->trace_cap,
                              hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DSU_OK;
}

extern "C" int dsu_batch_set_timing(dsu_batch *b, int32_t enable) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    CHK(batch_harvest_events(b));
    b->timing = enable != 0;
    for (int p = 0; p < PH_COUNT; ++p) {
        b->t_ms[p] = 0;
        b->t_count[p] = 0;
    }
    return DSU_OK;
}

extern "C" int dsu_batch_kernel_time(dsu_batch *b, int32_t phase, int64_t *launches, double *total_ms) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (phase < 0 || phase >= PH_COUNT) return fail(DSU_EINVAL, "bad phase %d", phase);
    CHK(batch_harvest_events(b));
    if (launches) *launches = b->t_count[phase];
    if (total_ms) *total_ms = b->t_ms[phase];
    return DSU_OK;
}

extern "C" int dsu_batch_use_graph(dsu_batch *b, int32_t enable) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    b->use_graph = enable != 0;
    return DSU_OK;
}
