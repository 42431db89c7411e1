// bucket.hip -- the lock-step engine of the batched form, and the dsu_batch
// entry points built on it.
//
// A sweep of every member determinant is a chain of windows of K proposals
// (electrons e0..e0+kw-1), three launches per window:
//   props  : draw the next window's kw moves and evaluate their proposed
//            orbital rows U (k_window_rows, beside the decisions on a second
//            stream)
//   decide : sequential Metropolis decisions with the bordered inverse of
//            eq. (3)'s C matrix (k_window_decide_gj / k_window_decide), the
//            look-ahead products G taken from the previous pass over BT
//   flush  : one pass over BT: the en-bloc Woodbury update of eq. (4), and,
//            while each chunk of the new BT is on chip, the next window's
//            look-ahead products (k_flush_stream32 / k_flush_stream)
#include "bucket.hpp"

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <mutex>

namespace dsu {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

BucketShape BucketShape::make(int n, int kmax, int prec) {
    BucketShape s;
    s.n = n;
    s.np = round_up(n, 64);
    s.kmax = kmax;
    s.kp = kpad(kmax);
    s.prec = prec;
    return s;
}

// Piece sizes in carve order.
static constexpr int kPieces = 15;
static void pieces(const BucketShape &s, size_t out[kPieces]) {
    const size_t e = elem_size(s.prec), np = s.np, kp = s.kp;
    out[0] = np * np * e;                           // bt
    out[1] = kp * np * e;                           // u
    out[2] = kp * np * e;                           // vg
    out[3] = kp * kp * 8;                           // cfl
    out[4] = kp > 128 ? kp * (kp + 1) * 8 : 0;      // cwork
    out[5] = kp > 64 ? kp * (kp + 1) * 8 : 0;       // gwork
    out[6] = kp * 4 * 8;                            // prop
    out[7] = (size_t)s.n * 3 * 8;                   // pos
    out[8] = kp * 4;                                // idx
    out[9] = sizeof(DetState);                      // st
    out[10] = kp * np * e;                          // u2
    out[11] = kp * np * e;                          // vg2
    out[12] = np * kp * e;                          // y
    out[13] = kp * 4 * 8;                           // prop2
    out[14] = s.prec == DSU_FP32_MIXED ? kp * kp * 4 : 0;  // cfl32
}

size_t BucketShape::det_bytes() const {
    size_t p[kPieces], b = 0;
    pieces(*this, p);
    for (size_t x : p) b += align256(x);
    return b;
}

DetSlot BucketShape::carve(char *base) const {
    size_t p[kPieces];
    pieces(*this, p);
    char *c = base;
    void *ptr[kPieces];
    for (int i = 0; i < kPieces; ++i) {
        ptr[i] = p[i] ? (void *)c : nullptr;
        c += align256(p[i]);
    }
    DetSlot d;
    d.bt = ptr[0];
    d.u = ptr[1];
    d.vg = ptr[2];
    d.cfl = (double *)ptr[3];
    d.cwork = (double *)ptr[4];
    d.gwork = (double *)ptr[5];
    d.prop = (double *)ptr[6];
    d.pos = (double *)ptr[7];
    d.idx = (int *)ptr[8];
    d.st = (DetState *)ptr[9];
    d.u2 = ptr[10];
    d.vg2 = ptr[11];
    d.y = ptr[12];
    d.prop2 = (double *)ptr[13];
    d.cfl32 = (float *)ptr[14];
    return d;
}

int Bucket::init(const BucketShape &shape, int k_delay, double box_l, void *stream_or_null, int gj_group,
                 void *gj_block) {
    sh = shape;
    K = k_delay;
    L = box_l;
    twopi_l = 2.0 * M_PI / box_l;
    CHK(make_stream(stream_or_null, &stream, &own_stream));
    HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    for (hipEvent_t &e : ev_ring_) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    CHK(dalloc(&kvec, (size_t)sh.n));
    std::vector<int4> kv(sh.n);
    build_kvectors(sh.n, kv.data());
    HIPCHK(hipMemcpy(kvec, kv.data(), sizeof(int4) * sh.n, hipMemcpyHostToDevice));
    kmax_comp = 0;
    for (const int4 &k : kv) kmax_comp = std::max({kmax_comp, std::abs(k.x), std::abs(k.y), std::abs(k.z)});
    CHK(gj_.alloc(std::max(1, gj_group), sh.np, sh.n, gj_block));
    return DSU_OK;
}

void Bucket::release() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (side) (void)hipStreamSynchronize(side);
    drop_graph();
    for (void *p : {(void *)kvec, ddesc_, fdesc_, sub_ddesc_, (void *)sub_pos_, (void *)sub_bt_, (void *)drift_,
                    (void *)res_rows_, (void *)res_eidx_, (void *)res_bits_})
        dfree(p);
    if (res_host_) (void)hipHostFree(res_host_);
    res_rows_ = nullptr;
    res_eidx_ = nullptr;
    res_bits_ = nullptr;
    res_host_ = nullptr;
    res_cap_ = 0;
    if (status_h_) (void)hipHostFree(status_h_);
    if (stage_h_) (void)hipHostFree(stage_h_);
    status_h_ = nullptr;
    stage_h_ = nullptr;
    pending_.clear();
    kvec = nullptr;
    ddesc_ = fdesc_ = sub_ddesc_ = nullptr;
    sub_pos_ = nullptr;
    sub_bt_ = nullptr;
    drift_ = nullptr;
    cap_ = 0;
    gj_.release();
    for (hipEvent_t &e : ev_ring_) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (side) (void)hipStreamDestroy(side);
    side = nullptr;
    for (auto &e : ev_free_) (void)hipEventDestroy(e);
    for (auto &e : ev_used_) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    ev_free_.clear();
    ev_used_.clear();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    stream = nullptr;
}

static size_t stage_bytes_per() {
    return std::max(sizeof(DetDesc<double>), sizeof(DetDesc<float>)) + sizeof(double *) + sizeof(void *);
}

int Bucket::ensure_capacity(int n) {
    if (n <= cap_) return DSU_OK;
    int c = std::max(n, cap_ * 2);
    // pending recompute statuses survive the move (the stream has passed them:
    // callers grow the arrays only between sweeps, after a synchronisation)
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<int> keep(status_h_ ? status_h_ : nullptr, status_h_ ? status_h_ + pending_.size() : nullptr);
    for (void *p : {ddesc_, fdesc_, sub_ddesc_, (void *)sub_pos_, (void *)sub_bt_, (void *)drift_}) dfree(p);
    if (status_h_) (void)hipHostFree(status_h_);
    if (stage_h_) (void)hipHostFree(stage_h_);
    status_h_ = nullptr;
    stage_h_ = nullptr;
    const size_t dsz = std::max(sizeof(DetDesc<double>), sizeof(DetDesc<float>));
    const size_t fsz = std::max(sizeof(FlushDesc<double>), sizeof(FlushDesc<float>));
    CHK(dev_alloc(&ddesc_, dsz * c));
    CHK(dev_alloc(&fdesc_, fsz * c));
    CHK(dev_alloc(&sub_ddesc_, dsz * c));
    CHK(dalloc(&sub_pos_, c));
    CHK(dalloc(&sub_bt_, c));
    CHK(dalloc(&drift_, c));
    HIPCHK(hipHostMalloc((void **)&status_h_, sizeof(int) * c));
    HIPCHK(hipHostMalloc((void **)&stage_h_, stage_bytes_per() * c));
    std::copy(keep.begin(), keep.end(), status_h_);
    cap_ = c;
    return DSU_OK;
}

template <typename T> static DetDesc<T> to_desc(const DetSlot &s) {
    DetDesc<T> d;
    d.bt = (T *)s.bt;
    d.u = (T *)s.u;
    d.vg = (T *)s.vg;
    d.cfl = s.cfl;
    d.cfl32 = s.cfl32;
    d.cwork = s.cwork;
    d.gwork = s.gwork;
    d.prop = s.prop;
    d.pos = s.pos;
    d.idx = s.idx;
    d.st = s.st;
    d.trace_r = s.trace_r;
    d.trace_a = s.trace_a;
    d.trace_cap = s.trace_cap;
    d.seed = s.seed;
    d.wid = s.wid;
    d.sigma = s.sigma;
    d.spin = s.spin;
    d.u2 = (T *)s.u2;
    d.vg2 = (T *)s.vg2;
    d.y = (T *)s.y;
    d.prop2 = s.prop2;
    return d;
}

template <typename T> int Bucket::upload_t() {
    std::vector<DetDesc<T>> dd(dets.size());
    std::vector<FlushDesc<T>> fd(dets.size());
    for (size_t i = 0; i < dets.size(); ++i) {
        dd[i] = to_desc<T>(dets[i]);
        fd[i] = FlushDesc<T>{dd[i].bt, dd[i].u, dd[i].vg, dd[i].cfl, dd[i].idx, sh.kp};
    }
    if (!dets.empty()) {
        HIPCHK(hipMemcpyAsync(ddesc_, dd.data(), sizeof(dd[0]) * dd.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(fdesc_, fd.data(), sizeof(fd[0]) * fd.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    return DSU_OK;
}

int Bucket::set_dets(const std::vector<DetSlot> &d) {
    HIPCHK(hipStreamSynchronize(stream));
    dets = d;
    CHK(ensure_capacity((int)dets.size()));
    drop_graph();
    return sh.prec == DSU_FP64 ? upload_t<double>() : upload_t<float>();
}

int Bucket::set_delay(int k) {
    if (k < 1 || k > sh.kmax) return fail(DSU_EINVAL, "delay %d outside [1, %d] of this batch", k, sh.kmax);
    HIPCHK(hipStreamSynchronize(stream));
    HIPCHK(hipStreamSynchronize(side));
    K = k;
    drop_graph();
    return DSU_OK;
}

void Bucket::drop_graph() {
    // a launched graph may still be running on either stream: destroy it only
    // once both have drained
    if (gexec_ || graph_) {
        if (stream) (void)hipStreamSynchronize(stream);
        if (side) (void)hipStreamSynchronize(side);
    }
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    gexec_ = nullptr;
    graph_ = nullptr;
    graph_force_ = -1;
}

template <typename F> int Bucket::timed(int phase, F fn, hipStream_t on) {
    if (!on) on = stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool ev = timing == 1 || (timing == 2 && phase == PH_FLUSH);
    if (ev) {
        for (hipEvent_t *e : {&e0, &e1}) {
            if (!ev_free_.empty()) {
                *e = ev_free_.back();
                ev_free_.pop_back();
            } else {
                HIPCHK(hipEventCreate(e));
            }
        }
        HIPCHK(hipEventRecord(e0, on));
    }
    HIPCHK(fn());
    if (ev) {
        HIPCHK(hipEventRecord(e1, on));
        ev_used_.push_back({phase, {e0, e1}});
    }
    return DSU_OK;
}

int Bucket::harvest_events() {
    if (ev_used_.empty()) return DSU_OK;
    HIPCHK(hipStreamSynchronize(stream));
    HIPCHK(hipStreamSynchronize(side));
    for (auto &e : ev_used_) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e.second.first, e.second.second));
        t_ms[e.first] += ms;
        t_count[e.first] += 1;
        ev_free_.push_back(e.second.first);
        ev_free_.push_back(e.second.second);
    }
    ev_used_.clear();
    return DSU_OK;
}

// Streaming sweep: prime (proposals of window 0, y = BT U^T for all rows,
// decisions of window 0), then per window w: proposals of w+1, one-pass flush
// of w producing y for w+1, decisions of w+1.
template <typename T> int Bucket::enqueue_sweep_stream_t(int force) {
    const DetDesc<T> *dd = (const DetDesc<T> *)ddesc_;
    const int nd = (int)dets.size();
    const int kt = kpad(K);
    const int nwin = (sh.n + K - 1) / K;
    auto kw_of = [&](int w) { return std::min(K, sh.n - w * K); };
    CHK(timed(PH_ROWS, [&] {
        return launch_window_props<T>(dd, nd, sh.n, sh.np, kt, 0, kw_of(0), kvec, twopi_l, 0, 1, kmax_comp, stream);
    }));
    CHK(timed(PH_G, [&] { return launch_window_prime<T>(dd, nd, sh.np, kt, sh.kp, 0, stream); }));
    int ring = 0;
    for (int w = 0; w < nwin; ++w) {
        const int cur = w & 1, nxt = cur ^ 1;
        const bool has_next = w + 1 < nwin;
        const int e0 = w * K, e0n = (w + 1) * K, kwn = has_next ? kw_of(w + 1) : 0;
        // The next window's proposals depend only on sweep-start positions of
        // its own electrons: draw them on the side stream while this window is
        // decided.  Their U/proposal buffers were last read by the previous
        // flush, which the fork point follows.
        hipEvent_t fork = ev_ring_[ring++ & 7], join = ev_ring_[ring++ & 7];
        if (has_next) {
            HIPCHK(hipEventRecord(fork, stream));
            HIPCHK(hipStreamWaitEvent(side, fork, 0));
            CHK(timed(PH_ROWS, [&] {
                return launch_window_props<T>(dd, nd, sh.n, sh.np, kt, e0n, kwn, kvec, twopi_l, nxt, 0, kmax_comp,
                                              side);
            }, side));
            HIPCHK(hipEventRecord(join, side));
        }
        CHK(timed(PH_DECIDE, [&] {
            return launch_window_decide<T>(dd, nd, kt, sh.kp, e0, kw_of(w), force, w + 1 == nwin, cur, stream);
        }));
        if (has_next) HIPCHK(hipStreamWaitEvent(stream, join, 0));
        CHK(timed(PH_FLUSH, [&] {
            return launch_flush_stream<T>(dd, nd, sh.np, kt, sh.kp, kw_of(w), cur, has_next ? 1 : 0, e0n, kwn, stream);
        }));
    }
    return DSU_OK;
}

int Bucket::enqueue_sweep(int force) {
    return sh.prec == DSU_FP64 ? enqueue_sweep_stream_t<double>(force) : enqueue_sweep_stream_t<float>(force);
}

int Bucket::build_graph(int force) {
    drop_graph();
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    const int tm = timing;
    timing = 0;
    int rc = enqueue_sweep(force);
    timing = tm;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &g);
    if (rc != DSU_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(DSU_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    graph_ = g;
    HIPCHK(hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0));
    graph_force_ = force;
    return DSU_OK;
}

int Bucket::sweep(int force) {
    if (dets.empty()) return DSU_OK;
    if (use_graph && !timing) {
        if (!gexec_ || graph_force_ != force) CHK(build_graph(force));
        HIPCHK(hipGraphLaunch(gexec_, stream));
        return DSU_OK;
    }
    return enqueue_sweep(force);
}

template <typename T> int Bucket::recompute_async_t(const std::vector<int> &which) {
    if (which.empty()) return DSU_OK;
    const int base = (int)pending_.size(), cnt_all = (int)which.size();
    if (base + cnt_all > cap_) return fail(DSU_ESTATE, "more pending recomputes than members");
    // descriptors staged in pinned memory at this call's own offset, so that
    // calls pending together do not overwrite each other's uploads
    DetDesc<T> *hd = (DetDesc<T> *)stage_h_;
    double **hp = (double **)(stage_h_ + std::max(sizeof(DetDesc<double>), sizeof(DetDesc<float>)) * cap_);
    void **hb = (void **)((char *)hp + sizeof(double *) * cap_);
    for (int i = 0; i < cnt_all; ++i) {
        const DetSlot &s = dets[which[i]];
        hd[base + i] = to_desc<T>(s);
        hp[base + i] = s.pos;
        hb[base + i] = s.bt;
    }
    DetDesc<T> *dd = (DetDesc<T> *)sub_ddesc_ + base;
    HIPCHK(hipMemcpyAsync(dd, hd + base, sizeof(DetDesc<T>) * cnt_all, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(sub_pos_ + base, hp + base, sizeof(double *) * cnt_all, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(sub_bt_ + base, hb + base, sizeof(void *) * cnt_all, hipMemcpyHostToDevice, stream));
    for (int g0 = 0; g0 < cnt_all; g0 += gj_.g) {
        const int cnt = std::min(gj_.g, cnt_all - g0);
        CHK(timed(PH_RECOMPUTE, [&] {
            hipError_t e =
                launch_build_pw_transpose(sub_pos_ + base + g0, gj_.mptr, cnt, sh.n, sh.np, kvec, twopi_l, stream);
            if (e != hipSuccess) return e;
            const GjDesc *res = nullptr;
            e = gj_.invert(cnt, sh.n, stream, &res);
            if (e != hipSuccess) return e;
            e = launch_cast_perm<T>(res, (T *const *)(sub_bt_ + base + g0), cnt, sh.n, sh.np, stream);
            if (e != hipSuccess) return e;
            return launch_reset_state<T>(dd + g0, res, drift_ + base + g0, cnt, stream);
        }));
        HIPCHK(hipMemcpyAsync(status_h_ + base + g0, gj_.status, sizeof(int) * cnt, hipMemcpyDeviceToHost, stream));
    }
    pending_.insert(pending_.end(), which.begin(), which.end());
    return DSU_OK;
}

int Bucket::recompute_async(const std::vector<int> &which) {
    return sh.prec == DSU_FP64 ? recompute_async_t<double>(which) : recompute_async_t<float>(which);
}

void Bucket::check_recompute(std::vector<int> *singular) {
    for (size_t i = 0; i < pending_.size(); ++i)
        if (status_h_[i] != 0 && singular) singular->push_back(pending_[i]);
    pending_.clear();
}

int Bucket::residual(int samples, std::vector<double> *right, std::vector<double> *left) {
    const int nd = (int)dets.size();
    if (right) right->assign(nd, 0.0);
    if (left) left->assign(nd, 0.0);
    if (nd == 0 || (!right && !left)) return DSU_OK;
    if (samples < 1 || samples > 64 || samples > sh.n)
        return fail(DSU_EINVAL, "residual samples %d outside [1, min(64, n = %d)]", samples, sh.n);
    HIPCHK(hipStreamSynchronize(stream));
    if (nd > res_cap_) {
        for (void *p : {(void *)res_rows_, (void *)res_eidx_, (void *)res_bits_}) dfree(p);
        if (res_host_) (void)hipHostFree(res_host_);
        res_rows_ = nullptr;
        res_eidx_ = nullptr;
        res_bits_ = nullptr;
        res_host_ = nullptr;
        res_cap_ = 0;
        CHK(dalloc(&res_rows_, (size_t)nd * 64 * sh.np));
        CHK(dalloc(&res_eidx_, (size_t)nd * 64));
        CHK(dalloc(&res_bits_, (size_t)2 * nd));
        HIPCHK(hipHostMalloc((void **)&res_host_, sizeof(unsigned long long) * 2 * nd));
        res_cap_ = nd;
    }
    const bool f64 = sh.prec == DSU_FP64;
    if (right) {
        HIPCHK(f64 ? launch_resid<double>((const DetDesc<double> *)ddesc_, nd, sh.n, sh.np, samples, kvec, twopi_l,
                                          res_rows_, res_eidx_, res_bits_, stream)
                   : launch_resid<float>((const DetDesc<float> *)ddesc_, nd, sh.n, sh.np, samples, kvec, twopi_l,
                                         res_rows_, res_eidx_, res_bits_, stream));
    }
    if (left) {
        HIPCHK(f64 ? launch_resid_left<double>((const DetDesc<double> *)ddesc_, nd, sh.n, sh.np, samples, kvec,
                                               twopi_l, kmax_comp, res_bits_ + nd, stream)
                   : launch_resid_left<float>((const DetDesc<float> *)ddesc_, nd, sh.n, sh.np, samples, kvec,
                                              twopi_l, kmax_comp, res_bits_ + nd, stream));
    }
    HIPCHK(hipMemcpyAsync(res_host_, res_bits_, sizeof(unsigned long long) * 2 * nd, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int i = 0; i < nd; ++i) {
        double v;
        if (right) {
            std::memcpy(&v, &res_host_[i], sizeof(v));
            (*right)[i] = v;
        }
        if (left) {
            std::memcpy(&v, &res_host_[nd + i], sizeof(v));
            (*left)[i] = v;
        }
    }
    return DSU_OK;
}

static int resid_pad(int samples) { return samples <= 16 ? 16 : (samples <= 32 ? 32 : 64); }

size_t Bucket::residual_scratch_bytes(int samples) const {
    const size_t nd = dets.size(), sp = (size_t)resid_pad(samples);
    return align256(2 * nd * sizeof(unsigned long long)) + align256(nd * sp * sizeof(int)) +
           nd * sp * (size_t)sh.np * sizeof(double);
}

int Bucket::residual_into(int samples, double *right_host, double *left_host, void *scratch, size_t scratch_bytes) {
    const int nd = (int)dets.size();
    if (nd == 0 || (!right_host && !left_host)) return DSU_OK;
    if (samples < 1 || samples > 64 || samples > sh.n)
        return fail(DSU_EINVAL, "residual samples %d outside [1, min(64, n = %d)]", samples, sh.n);
    const size_t need = residual_scratch_bytes(samples);
    if (need > scratch_bytes)
        return fail(DSU_EINVAL,
                    "%d determinants of n = %d with %d samples need %zu bytes of residual scratch; the "
                    "allocation-free entry point has %zu (use dsu_batch_residual)",
                    nd, sh.n, samples, need, scratch_bytes);
    // layout: result words (right, then left), sample indices, sample rows
    char *base = static_cast<char *>(scratch);
    unsigned long long *bits = reinterpret_cast<unsigned long long *>(base);
    const size_t sp = (size_t)resid_pad(samples);
    int *eidx = reinterpret_cast<int *>(base + align256(2 * (size_t)nd * sizeof(unsigned long long)));
    double *rows = reinterpret_cast<double *>(reinterpret_cast<char *>(eidx) + align256((size_t)nd * sp * sizeof(int)));
    const bool f64 = sh.prec == DSU_FP64;
    if (right_host) {
        HIPCHK(f64 ? launch_resid<double>((const DetDesc<double> *)ddesc_, nd, sh.n, sh.np, samples, kvec, twopi_l,
                                          rows, eidx, bits, stream)
                   : launch_resid<float>((const DetDesc<float> *)ddesc_, nd, sh.n, sh.np, samples, kvec, twopi_l, rows,
                                         eidx, bits, stream));
        HIPCHK(hipMemcpyAsync(right_host, bits, sizeof(double) * nd, hipMemcpyDeviceToHost, stream));
    }
    if (left_host) {
        HIPCHK(f64 ? launch_resid_left<double>((const DetDesc<double> *)ddesc_, nd, sh.n, sh.np, samples, kvec,
                                               twopi_l, kmax_comp, bits + nd, stream)
                   : launch_resid_left<float>((const DetDesc<float> *)ddesc_, nd, sh.n, sh.np, samples, kvec,
                                              twopi_l, kmax_comp, bits + nd, stream));
        HIPCHK(hipMemcpyAsync(left_host, bits + nd, sizeof(double) * nd, hipMemcpyDeviceToHost, stream));
    }
    // the words are the bit patterns of the doubles: copied as they are
    HIPCHK(hipStreamSynchronize(stream));
    return DSU_OK;
}

int Bucket::recompute(const std::vector<int> &which, double *drift_host) {
    if (which.empty()) return DSU_OK;
    HIPCHK(hipStreamSynchronize(stream));
    check_recompute(nullptr);
    CHK(recompute_async(which));
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<int> bad;
    check_recompute(&bad);
    if (!bad.empty()) return fail(DSU_ESINGULAR, "determinant %d: Slater matrix is singular", bad[0]);
    if (drift_host) {
        HIPCHK(hipMemcpyAsync(drift_host, drift_, sizeof(double) * which.size(), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    return DSU_OK;
}

// Plane-wave table: orbitals by shells s = |n|^2 = 0, 1, 2, ...; inside a
// shell the integer vectors whose first nonzero component is positive, in
// ascending (nx, ny, nz); n = 0 gives the constant, every other vector cos
// then sin.
int build_kvectors(int n, int4 *out) {
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

}  // namespace dsu

// ==========================================================================
// Plane-wave utilities
// ==========================================================================
extern "C" int dsu_plane_wave_table(int32_t n, int32_t *out4) {
    if (n < 1 || n > 32768 || !out4) return dsu::fail(DSU_EINVAL, "bad arguments");
    std::vector<int4> kv(n);
    dsu::build_kvectors(n, kv.data());
    for (int j = 0; j < n; ++j) {
        out4[4 * j + 0] = kv[j].x;
        out4[4 * j + 1] = kv[j].y;
        out4[4 * j + 2] = kv[j].z;
        out4[4 * j + 3] = kv[j].w;
    }
    return DSU_OK;
}

extern "C" int dsu_plane_wave_rows(int32_t n, double box_L, int32_t count, const double *positions_host,
                                   double *rows_host) {
    using namespace dsu;
    if (n < 1 || n > 32768 || count < 0 || !(box_L > 0)) return fail(DSU_EINVAL, "bad arguments");
    if (count == 0) return DSU_OK;
    if (!positions_host || !rows_host) return fail(DSU_EINVAL, "NULL array");
    std::vector<int4> kv(n);
    build_kvectors(n, kv.data());
    int4 *dk = nullptr;
    double *dp = nullptr, *dr = nullptr;
    hipStream_t s = nullptr;
    bool own = false;
    int rc = make_stream(nullptr, &s, &own);
    if (rc == DSU_OK) rc = dalloc(&dk, (size_t)n);
    if (rc == DSU_OK) rc = dalloc(&dp, (size_t)count * 3);
    if (rc == DSU_OK) rc = dalloc(&dr, (size_t)count * n);
    hipError_t e = hipSuccess;
    if (rc == DSU_OK) e = hipMemcpyAsync(dk, kv.data(), sizeof(int4) * n, hipMemcpyHostToDevice, s);
    if (rc == DSU_OK && e == hipSuccess)
        e = hipMemcpyAsync(dp, positions_host, sizeof(double) * count * 3, hipMemcpyHostToDevice, s);
    if (rc == DSU_OK && e == hipSuccess) e = launch_pw_rows(dp, dr, n, count, dk, 2.0 * M_PI / box_L, s);
    if (rc == DSU_OK && e == hipSuccess)
        e = hipMemcpyAsync(rows_host, dr, sizeof(double) * count * n, hipMemcpyDeviceToHost, s);
    if (rc == DSU_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc == DSU_OK && e != hipSuccess) rc = fail(DSU_EDEVICE, "plane-wave rows: %s", hipGetErrorString(e));
    dfree(dk);
    dfree(dp);
    dfree(dr);
    if (own && s) (void)hipStreamDestroy(s);
    return rc;
}

// ==========================================================================
// dsu_batch: one bucket over one contiguous block of determinant storage.
// ==========================================================================
using namespace dsu;

struct dsu_batch {
    Bucket bk;
    int walkers = 0, spins = 1, ndet = 0, recompute_every = 0;
    char *store = nullptr;
    double *trace_r = nullptr;
    uint8_t *trace_a = nullptr;
    long long trace_cap = 0;
    double *inv_tmp = nullptr;
    long long sweeps_done = 0;
    // watchdog: recompute members whose count of zero / non-finite ratios grew
    bool watchdog = false;
    std::vector<int> bad_seen;
    long long watchdog_recomputes = 0;
    // residual watchdog: sampled residual after every sweep, recompute above threshold
    int resid_samples = 0;
    double resid_threshold = 0.0;
    long long resid_recomputes = 0;
    std::vector<double> last_right, last_drift;
};

// Recompute the listed members, keeping each one's running-minus-fresh log|det|.
static int batch_recompute_some(dsu_batch *b, const std::vector<int> &which) {
    if (which.empty()) return DSU_OK;
    std::vector<double> drift(which.size());
    CHK(b->bk.recompute(which, drift.data()));
    for (size_t i = 0; i < which.size(); ++i) b->last_drift[which[i]] = drift[i];
    return DSU_OK;
}

static int batch_read_bad(dsu_batch *b, std::vector<int> *bad) {
    bad->resize(b->ndet);
    for (int i = 0; i < b->ndet; ++i) {
        DetState st;
        HIPCHK(hipMemcpy(&st, b->bk.dets[i].st, sizeof(st), hipMemcpyDeviceToHost));
        (*bad)[i] = st.bad;
    }
    return DSU_OK;
}

static void batch_free(dsu_batch *b) {
    b->bk.release();
    dfree(b->store);
    dfree(b->trace_r);
    dfree(b->trace_a);
    dfree(b->inv_tmp);
}

static std::vector<int> all_indices(int n) {
    std::vector<int> v(n);
    for (int i = 0; i < n; ++i) v[i] = i;
    return v;
}

extern "C" size_t dsu_footprint_bytes(int32_t n, int32_t k_delay, int32_t precision) {
    if (n < 1 || n > 32768 || k_delay < 1 || k_delay > DSU_MAX_K ||
        (precision != DSU_FP64 && precision != DSU_FP32_MIXED))
        return 0;
    return BucketShape::make(n, k_delay, precision).det_bytes();
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
    b->recompute_every = recompute_every;
    b->last_right.assign(b->ndet, 0.0);
    b->last_drift.assign(b->ndet, 0.0);
    const BucketShape sh = BucketShape::make(n, k_delay, precision);
    // recompute as many determinants at once as fit in ~16 GiB of workspace
    const size_t per = GjWork::bytes_per(sh.np, n);
    int group = (int)std::min<size_t>((size_t)b->ndet, std::max<size_t>(1, ((size_t)16 << 30) / per));
    int rc = b->bk.init(sh, k_delay, box_L, hip_stream, group);
    if (rc == DSU_OK) rc = dev_alloc((void **)&b->store, sh.det_bytes() * b->ndet);
    if (rc != DSU_OK) {
        batch_free(b);
        delete b;
        return rc;
    }
    std::vector<DetSlot> slots(b->ndet);
    std::vector<DetState> st(b->ndet);
    for (int i = 0; i < b->ndet; ++i) {
        const int w = i / spins;
        DetSlot &s = slots[i];
        s = sh.carve(b->store + sh.det_bytes() * i);
        s.seed = seeds[w];
        s.wid = walker_ids[w];
        s.sigma = sigma[w];
        s.spin = i % spins;
        st[i] = DetState{0.0, 1, 0, 0, 0, 0};
        if (hipMemcpy(s.pos, positions_host + (size_t)n * 3 * i, sizeof(double) * n * 3, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(s.st, &st[i], sizeof(DetState), hipMemcpyHostToDevice) != hipSuccess) {
            batch_free(b);
            delete b;
            return fail(DSU_EDEVICE, "upload of walker state failed");
        }
    }
    rc = b->bk.set_dets(slots);
    if (rc == DSU_OK) rc = b->bk.recompute(all_indices(b->ndet), nullptr);
    if (rc != DSU_OK) {
        batch_free(b);
        delete b;
        return rc;
    }
    *out = b;
    return DSU_OK;
}

extern "C" int dsu_batch_destroy(dsu_batch *b) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    batch_free(b);
    delete b;
    return DSU_OK;
}

extern "C" int dsu_batch_sweep(dsu_batch *b, int32_t sweeps, int32_t force_accept) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (sweeps < 0) return fail(DSU_EINVAL, "sweeps < 0");
    for (int s = 0; s < sweeps; ++s) {
        if (b->recompute_every > 0 && b->sweeps_done > 0 && b->sweeps_done % b->recompute_every == 0)
            CHK(batch_recompute_some(b, all_indices(b->ndet)));
        CHK(b->bk.sweep(force_accept ? 1 : 0));
        ++b->sweeps_done;
        if (b->resid_samples > 0) {
            CHK(b->bk.residual(b->resid_samples, &b->last_right, nullptr));
            std::vector<int> which;
            for (int i = 0; i < b->ndet; ++i)
                if (!(b->last_right[i] <= b->resid_threshold)) which.push_back(i);
            CHK(batch_recompute_some(b, which));
            b->resid_recomputes += (long long)which.size();
        }
        if (b->watchdog) {
            HIPCHK(hipStreamSynchronize(b->bk.stream));
            std::vector<int> bad, which;
            CHK(batch_read_bad(b, &bad));
            for (int i = 0; i < b->ndet; ++i)
                if (bad[i] > b->bad_seen[i]) which.push_back(i);
            if (!which.empty()) {
                CHK(batch_recompute_some(b, which));
                b->watchdog_recomputes += (long long)which.size();
            }
            b->bad_seen = bad;
        }
    }
    return DSU_OK;
}

extern "C" int dsu_batch_set_watchdog(dsu_batch *b, int32_t enable) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    b->watchdog = enable != 0;
    if (b->watchdog) CHK(batch_read_bad(b, &b->bad_seen));
    return DSU_OK;
}

extern "C" int dsu_batch_residual(dsu_batch *b, int32_t samples, double *right_host, double *left_host) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (!right_host && !left_host) return fail(DSU_EINVAL, "both outputs are NULL");
    std::vector<double> r, l;
    CHK(b->bk.residual(samples, right_host ? &r : nullptr, left_host ? &l : nullptr));
    if (right_host) std::copy(r.begin(), r.end(), right_host);
    if (left_host) std::copy(l.begin(), l.end(), left_host);
    return DSU_OK;
}

// --------------------------------------------------------------------------
// Allocation-free residual: the device buffers of dsu_batch_residual carved
// from one file-scope array.  Each GPU holds its own copy of the array, so its
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels and copies: in host code
// the array's name is a host-side stand-in, not a device address.
static constexpr size_t kResidScratchBytes = (size_t)32 << 20;  // 32 MiB per device
static __device__ __align__(256) unsigned char scratch[kResidScratchBytes];
static std::mutex g_scratch_mu;
static constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices] = {};

static int resid_scratch(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DSU_EDEVICE, "device %d outside the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DSU_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DSU_OK;
}

extern "C" int dsu_batch_residual_noalloc(dsu_batch *b, int32_t samples, double *right_host, double *left_host) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (!right_host && !left_host) return fail(DSU_EINVAL, "both outputs are NULL");
    void *p = nullptr;
    CHK(resid_scratch(&p));
    return b->bk.residual_into(samples, right_host, left_host, p, kResidScratchBytes);
}

extern "C" int dsu_batch_set_residual_watchdog(dsu_batch *b, int32_t samples, double threshold) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (samples < 0 || samples > 64 || samples > b->bk.sh.n)
        return fail(DSU_EINVAL, "residual samples %d outside [0, min(64, n = %d)]", samples, b->bk.sh.n);
    if (samples > 0 && !(threshold > 0.0)) return fail(DSU_EINVAL, "residual threshold must be positive");
    b->resid_samples = samples;
    b->resid_threshold = threshold;
    return DSU_OK;
}

extern "C" int dsu_batch_set_recompute_tiles(dsu_batch *b, int32_t panel, int32_t chunk, int32_t apply_columns) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    const int np = b->bk.sh.np;
    const GjTiles def = gj_tiles_default(b->bk.sh.n, np);
    GjTiles t;
    t.nb = panel ? panel : def.nb;
    t.cw = chunk ? chunk : def.cw;
    t.cpb = apply_columns ? apply_columns : def.cpb;
    if (t.nb != 16 && t.nb != 32 && t.nb != 64 && t.nb != 128)
        return fail(DSU_EINVAL, "panel width %d not 0, 16, 32, 64 or 128", panel);
    if (t.cw != 32 && t.cw != 64) return fail(DSU_EINVAL, "update chunk %d not 0, 32 or 64", chunk);
    if (t.cw == 64 && np % 128)
        return fail(DSU_EINVAL, "update chunk 64 needs the padded size (%d) to be a multiple of 128", np);
    if (t.cpb != 1 && t.cpb != 4) return fail(DSU_EINVAL, "apply columns %d not 0, 1 or 4", apply_columns);
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    b->bk.set_recompute_tiles(t);
    return DSU_OK;
}

extern "C" int dsu_batch_get_recompute_tiles(dsu_batch *b, int32_t *panel, int32_t *chunk, int32_t *apply_columns) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    const GjTiles t = b->bk.recompute_tiles();
    if (panel) *panel = t.nb;
    if (chunk) *chunk = t.cw;
    if (apply_columns) *apply_columns = t.cpb;
    return DSU_OK;
}

extern "C" int dsu_batch_accuracy(dsu_batch *b, double *residual_out, double *drift_out,
                                  int64_t *residual_recomputes) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (residual_out) std::copy(b->last_right.begin(), b->last_right.end(), residual_out);
    if (drift_out) std::copy(b->last_drift.begin(), b->last_drift.end(), drift_out);
    if (residual_recomputes) *residual_recomputes = b->resid_recomputes;
    return DSU_OK;
}

extern "C" int dsu_batch_watchdog_count(dsu_batch *b, int64_t *recomputes) {
    if (!b || !recomputes) return fail(DSU_EINVAL, "NULL argument");
    *recomputes = b->watchdog_recomputes;
    return DSU_OK;
}

extern "C" int dsu_batch_poison_row(dsu_batch *b, int32_t det, int32_t row) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    if (row < 0 || row >= b->bk.sh.n) return fail(DSU_EINVAL, "row %d out of range", row);
    const size_t es = elem_size(b->bk.sh.prec), np = b->bk.sh.np;
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    // all-ones bytes: a NaN in either precision
    HIPCHK(hipMemset(static_cast<char *>(b->bk.dets[det].bt) + (size_t)row * np * es, 0xff, np * es));
    return DSU_OK;
}

extern "C" int dsu_batch_sync(dsu_batch *b) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    return DSU_OK;
}

extern "C" int dsu_batch_recompute(dsu_batch *b, double *drift_out) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    CHK(batch_recompute_some(b, all_indices(b->ndet)));
    if (drift_out) std::copy(b->last_drift.begin(), b->last_drift.end(), drift_out);
    return DSU_OK;
}

extern "C" int dsu_batch_set_delay(dsu_batch *b, int32_t k_delay) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    return b->bk.set_delay(k_delay);
}

extern "C" int dsu_batch_stats(dsu_batch *b, double *logdet, int32_t *sign, int64_t *accepted, int64_t *sweeps_done) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    for (int i = 0; i < b->ndet; ++i) {
        DetState st;
        HIPCHK(hipMemcpy(&st, b->bk.dets[i].st, sizeof(st), hipMemcpyDeviceToHost));
        if (logdet) logdet[i] = st.logdet;
        if (sign) sign[i] = st.sign;
        if (accepted) accepted[i] = st.accepted;
        if (sweeps_done) sweeps_done[i] = st.sweep;
    }
    return DSU_OK;
}

extern "C" int dsu_batch_set_sweep(dsu_batch *b, int64_t sweeps_done) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (sweeps_done < 0) return fail(DSU_EINVAL, "sweeps_done %lld < 0", (long long)sweeps_done);
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    for (int i = 0; i < b->ndet; ++i) {
        const long long v = sweeps_done;
        HIPCHK(hipMemcpy(reinterpret_cast<char *>(b->bk.dets[i].st) + offsetof(DetState, sweep), &v, sizeof(v),
                         hipMemcpyHostToDevice));
    }
    return DSU_OK;
}

extern "C" int dsu_batch_get_positions(dsu_batch *b, int32_t det, double *out_host) {
    if (!b || !out_host) return fail(DSU_EINVAL, "NULL argument");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    HIPCHK(hipMemcpyAsync(out_host, b->bk.dets[det].pos, sizeof(double) * b->bk.sh.n * 3, hipMemcpyDeviceToHost,
                          b->bk.stream));
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    return DSU_OK;
}

extern "C" int dsu_batch_get_inverse(dsu_batch *b, int32_t det, double *out_host) {
    if (!b || !out_host) return fail(DSU_EINVAL, "NULL argument");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    const int n = b->bk.sh.n, np = b->bk.sh.np;
    if (!b->inv_tmp) CHK(dalloc(&b->inv_tmp, (size_t)n * n));
    if (b->bk.sh.prec == DSU_FP64)
        HIPCHK(launch_untranspose<double>((const double *)b->bk.dets[det].bt, b->inv_tmp, n, np, b->bk.stream));
    else
        HIPCHK(launch_untranspose<float>((const float *)b->bk.dets[det].bt, b->inv_tmp, n, np, b->bk.stream));
    HIPCHK(hipMemcpyAsync(out_host, b->inv_tmp, sizeof(double) * n * n, hipMemcpyDeviceToHost, b->bk.stream));
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    return DSU_OK;
}

extern "C" int dsu_batch_set_trace(dsu_batch *b, int32_t sweeps) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (sweeps < 0) return fail(DSU_EINVAL, "sweeps < 0");
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    dfree(b->trace_r);
    dfree(b->trace_a);
    b->trace_r = nullptr;
    b->trace_a = nullptr;
    b->trace_cap = (long long)sweeps * b->bk.sh.n;
    if (sweeps > 0) {
        CHK(dalloc(&b->trace_r, (size_t)b->trace_cap * b->ndet));
        CHK(dalloc(&b->trace_a, (size_t)b->trace_cap * b->ndet));
    }
    std::vector<DetSlot> slots = b->bk.dets;
    for (int i = 0; i < b->ndet; ++i) {
        slots[i].trace_r = b->trace_r ? b->trace_r + (size_t)b->trace_cap * i : nullptr;
        slots[i].trace_a = b->trace_a ? b->trace_a + (size_t)b->trace_cap * i : nullptr;
        slots[i].trace_cap = b->trace_r ? b->trace_cap : 0;
        DetState st;
        HIPCHK(hipMemcpy(&st, slots[i].st, sizeof(st), hipMemcpyDeviceToHost));
        st.trace_pos = 0;
        HIPCHK(hipMemcpy(slots[i].st, &st, sizeof(st), hipMemcpyHostToDevice));
    }
    return b->bk.set_dets(slots);
}

extern "C" int dsu_batch_get_trace(dsu_batch *b, int32_t det, double *ratio_host, uint8_t *accepted_host) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (det < 0 || det >= b->ndet) return fail(DSU_EINVAL, "det %d out of range", det);
    if (!b->trace_r) return fail(DSU_ESTATE, "tracing is off");
    if (ratio_host)
        HIPCHK(hipMemcpyAsync(ratio_host, b->trace_r + (size_t)b->trace_cap * det, sizeof(double) * b->trace_cap,
                              hipMemcpyDeviceToHost, b->bk.stream));
    if (accepted_host)
        HIPCHK(hipMemcpyAsync(accepted_host, b->trace_a + (size_t)b->trace_cap * det, b->trace_cap,
                              hipMemcpyDeviceToHost, b->bk.stream));
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    return DSU_OK;
}

extern "C" int dsu_batch_set_timing(dsu_batch *b, int32_t enable) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (enable < 0 || enable > 2) return fail(DSU_EINVAL, "timing level %d (0, 1 or 2)", enable);
    CHK(b->bk.harvest_events());
    b->bk.timing = enable;
    for (int p = 0; p < PH_COUNT; ++p) {
        b->bk.t_ms[p] = 0;
        b->bk.t_count[p] = 0;
    }
    return DSU_OK;
}

extern "C" int dsu_batch_kernel_time(dsu_batch *b, int32_t phase, int64_t *launches, double *total_ms) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    if (phase < 0 || phase >= PH_COUNT) return fail(DSU_EINVAL, "bad phase %d", phase);
    CHK(b->bk.harvest_events());
    if (launches) *launches = b->bk.t_count[phase];
    if (total_ms) *total_ms = b->bk.t_ms[phase];
    return DSU_OK;
}

extern "C" int dsu_batch_use_graph(dsu_batch *b, int32_t enable) {
    if (!b) return fail(DSU_EINVAL, "batch is NULL");
    b->bk.use_graph = enable != 0;
    return DSU_OK;
}

