// dsu_server.hip -- the serving pool: walkers of mixed size admitted by a
// device-memory budget and continuously batched.
//
// * One device allocation of `budget` bytes is the arena every walker's
//   state (inverses, delayed buffers, positions) is carved from (first fit,
//   coalescing free list).  A request waits until its footprint fits.
// * Walkers of the same n share a Bucket (lock-step windows, one launch per
//   phase for all of them) on the bucket's own stream; buckets of different
//   n run concurrently on the device.
// * Membership changes only between a bucket's sweeps: arrivals join and
//   finished walkers leave at the next sweep boundary of their bucket, while
//   the other buckets keep running.
// * Every walker draws from its own counter-based stream keyed by (request
//   seed, request id), so its result does not depend on what else is resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "bucket.hpp"

using namespace dsu;

namespace {

// First-fit allocator over [0, size) with coalescing.
class Arena {
  public:
    size_t size = 0, used = 0;
    void reset(size_t sz) {
        size = sz;
        used = 0;
        free_.clear();
        if (sz) free_[0] = sz;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Resident {
    uint64_t request_id = 0;
    int n = 0, spins = 1, sweeps_target = 0, sweeps_done = 0;
    size_t off = 0, bytes = 0;
    std::vector<DetSlot> dets;
    double admit_s = 0.0, last_s = 0.0;
    int result_index = -1;
    int status = DSU_OK;  // DSU_ESINGULAR once an inverse of the walker came out singular
};

struct BucketState {
    Bucket bk;
    std::vector<int> members;  // slot ids, in descriptor order
    bool busy = false;
    bool dirty = false;
    hipEvent_t done = nullptr;
    size_t ws_off = 0, ws_bytes = 0;  // the recompute workspace, carved from the arena
};

// Determinants recomputed per pass in a serving bucket.
constexpr int kServerGjGroup = 4;

// Arena bytes a bucket of size n takes for its recompute workspace.
static size_t bucket_ws_bytes(int n) {
    const int np = round_up(n, 64);
    return GjWork::block_bytes(kServerGjGroup, np, n);
}

}  // namespace

struct dsu_server {
    int K = 0, prec = 0, recompute_every = 0;
    double L = 0.0;
    size_t budget = 0;
    char *arena_base = nullptr;
    Arena arena;
    std::map<int, std::unique_ptr<BucketState>> buckets;
    std::map<int, Resident> resident;  // slot -> walker
    int next_slot = 0;
};

static int bucket_for(dsu_server *s, int n, BucketState **out) {
    auto it = s->buckets.find(n);
    if (it != s->buckets.end()) {
        *out = it->second.get();
        return DSU_OK;
    }
    std::unique_ptr<BucketState> b(new BucketState());
    const BucketShape sh = BucketShape::make(n, s->K, s->prec);
    // the recompute workspace (four determinants per pass) is charged to the
    // budget: carved from the arena, held while the server lives
    b->ws_bytes = bucket_ws_bytes(n);
    if (!s->arena.alloc(b->ws_bytes, &b->ws_off))
        return fail(DSU_EBUDGET, "recompute workspace of size %d does not fit the free budget now", n);
    // descriptor room for 64
    int rc = b->bk.init(sh, s->K, s->L, nullptr, kServerGjGroup, s->arena_base + b->ws_off);
    if (rc == DSU_OK) rc = b->bk.reserve(64);
    if (rc != DSU_OK) {
        b->bk.release();
        s->arena.release(b->ws_off, b->ws_bytes);
        return rc;
    }
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        b->bk.release();
        s->arena.release(b->ws_off, b->ws_bytes);
        return fail(DSU_EDEVICE, "hipEventCreate failed");
    }
    *out = b.get();
    s->buckets[n] = std::move(b);
    return DSU_OK;
}

static size_t walker_bytes(int n, int spins, int K, int prec) {
    return BucketShape::make(n, K, prec).det_bytes() * (size_t)spins;
}

// Upload the member list of a bucket (it must be idle).
static int refresh_bucket(dsu_server *s, BucketState *b) {
    std::vector<DetSlot> d;
    for (int slot : b->members)
        for (const DetSlot &x : s->resident[slot].dets) d.push_back(x);
    b->dirty = false;
    return b->bk.set_dets(d);
}

// Admit one request (its bucket must be idle).  DSU_EBUDGET if it does not fit now.
static int admit(dsu_server *s, const dsu_request &r, double now_s, int result_index, int *slot_out) {
    if (r.n < 1 || r.n > 32768 || (r.spins != 1 && r.spins != 2) || r.sweeps < 0 || !r.positions)
        return fail(DSU_EINVAL, "bad request %llu", (unsigned long long)r.request_id);
    const size_t bytes = walker_bytes(r.n, r.spins, s->K, s->prec);
    // a walker of a size not resident yet also brings its bucket's workspace
    const size_t ws = s->buckets.count(r.n) ? 0 : bucket_ws_bytes(r.n);
    if (bytes + ws > s->budget)
        return fail(DSU_EINVAL, "request %llu needs %zu bytes (walker %zu, recompute workspace %zu), budget %zu",
                    (unsigned long long)r.request_id, bytes + ws, bytes, ws, s->budget);
    size_t off = 0;
    if (!s->arena.alloc(bytes, &off)) return fail(DSU_EBUDGET, "request does not fit the free budget now");
    BucketState *b = nullptr;
    int rc = bucket_for(s, r.n, &b);
    if (rc != DSU_OK) {
        s->arena.release(off, bytes);
        return rc;
    }
    const BucketShape &sh = b->bk.sh;
    Resident w;
    w.request_id = r.request_id;
    w.n = r.n;
    w.spins = r.spins;
    w.sweeps_target = r.sweeps;
    w.off = off;
    w.bytes = bytes;
    w.admit_s = now_s;
    w.last_s = now_s;
    w.result_index = result_index;
    char *base = s->arena_base + off;
    hipStream_t st = b->bk.stream;
    HIPCHK(hipMemsetAsync(base, 0, bytes, st));
    const DetState init{0.0, 1, 0, 0, 0, 0};
    for (int sp = 0; sp < r.spins; ++sp) {
        DetSlot d = sh.carve(base + sh.det_bytes() * sp);
        d.seed = r.seed;
        d.wid = r.request_id;
        d.sigma = r.sigma;
        d.spin = sp;
        HIPCHK(hipMemcpyAsync(d.pos, r.positions + (size_t)sp * r.n * 3, sizeof(double) * r.n * 3,
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d.st, &init, sizeof(DetState), hipMemcpyHostToDevice, st));
        w.dets.push_back(d);
    }
    HIPCHK(hipStreamSynchronize(st));
    const int slot = s->next_slot++;
    s->resident[slot] = w;
    b->members.push_back(slot);
    rc = refresh_bucket(s, b);
    if (rc == DSU_OK) {
        // FP64 inverse of the new walker's determinants (the last members),
        // enqueued ahead of the bucket's next sweep; a singular start is
        // reported when that sweep completes.
        std::vector<int> which;
        for (int i = 0; i < r.spins; ++i) which.push_back((int)b->bk.dets.size() - r.spins + i);
        rc = b->bk.recompute_async(which);
    }
    if (rc != DSU_OK) {
        b->members.pop_back();
        s->resident.erase(slot);
        s->arena.release(off, bytes);
        (void)refresh_bucket(s, b);
        return rc;
    }
    if (slot_out) *slot_out = slot;
    return DSU_OK;
}

static int read_result(dsu_server *s, int slot, dsu_result *out) {
    Resident &w = s->resident[slot];
    out->request_id = w.request_id;
    out->status = w.status;
    out->sweeps_done = w.sweeps_done;
    out->admit_s = w.admit_s;
    out->finish_s = w.last_s;
    out->accepted = 0;
    out->logdet[0] = out->logdet[1] = 0.0;
    out->sign[0] = out->sign[1] = 0;
    for (int sp = 0; sp < w.spins; ++sp) {
        DetState st;
        HIPCHK(hipMemcpy(&st, w.dets[sp].st, sizeof(st), hipMemcpyDeviceToHost));
        out->logdet[sp] = st.logdet;
        out->sign[sp] = st.sign;
        out->accepted += st.accepted;
    }
    return DSU_OK;
}

// Release idle buckets without members, with their recompute workspace
// (charged to the budget only while a walker of that size is resident).
static void drop_empty_buckets(dsu_server *s) {
    for (auto it = s->buckets.begin(); it != s->buckets.end();) {
        BucketState *b = it->second.get();
        if (b->busy || !b->members.empty()) {
            ++it;
            continue;
        }
        b->bk.release();  // waits for the bucket's streams
        if (b->done) (void)hipEventDestroy(b->done);
        s->arena.release(b->ws_off, b->ws_bytes);
        it = s->buckets.erase(it);
    }
}

static void retire(dsu_server *s, int slot) {
    Resident &w = s->resident[slot];
    s->arena.release(w.off, w.bytes);
    auto it = s->buckets.find(w.n);
    if (it != s->buckets.end()) {
        auto &m = it->second->members;
        m.erase(std::remove(m.begin(), m.end(), slot), m.end());
        it->second->dirty = true;
    }
    s->resident.erase(slot);
}

// After a completed sweep of bucket b: recompute the walkers that are due.
static int recompute_due(dsu_server *s, BucketState *b) {
    if (s->recompute_every <= 0) return DSU_OK;
    std::vector<int> which;
    int pos = 0;
    for (int slot : b->members) {
        const Resident &w = s->resident[slot];
        const bool due = w.sweeps_done > 0 && w.sweeps_done < w.sweeps_target &&
                         w.sweeps_done % s->recompute_every == 0;
        for (int sp = 0; sp < w.spins; ++sp, ++pos)
            if (due) which.push_back(pos);
    }
    return b->bk.recompute_async(which);
}

static int slot_of_det(dsu_server *s, BucketState *b, int pos);

// After bucket b's stream has passed its pending recomputes: flag the walkers
// whose inverse came out singular; returns their slots.
static std::vector<int> flag_singular(dsu_server *s, BucketState *b) {
    std::vector<int> bad, slots;
    b->bk.check_recompute(&bad);
    for (int pos : bad) {
        const int slot = slot_of_det(s, b, pos);
        if (slot >= 0 && std::find(slots.begin(), slots.end(), slot) == slots.end()) {
            slots.push_back(slot);
            s->resident[slot].status = DSU_ESINGULAR;
        }
    }
    return slots;
}

// Slot of the walker that owns determinant `pos` of bucket b (descriptor order).
static int slot_of_det(dsu_server *s, BucketState *b, int pos) {
    for (int slot : b->members) {
        const int sp = s->resident[slot].spins;
        if (pos < sp) return slot;
        pos -= sp;
    }
    return -1;
}

extern "C" size_t dsu_server_workspace_bytes(int32_t n) {
    if (n < 1 || n > 32768) return 0;
    return bucket_ws_bytes(n);
}

extern "C" int dsu_server_create(int32_t k_delay, int32_t precision, double box_L, size_t budget_bytes,
                                 int32_t recompute_every, dsu_server **out) {
    if (!out) return fail(DSU_EINVAL, "out is NULL");
    *out = nullptr;
    if (k_delay < 1 || k_delay > DSU_MAX_K) return fail(DSU_EINVAL, "k_delay = %d out of range", k_delay);
    if (precision != DSU_FP64 && precision != DSU_FP32_MIXED) return fail(DSU_EINVAL, "bad precision %d", precision);
    if (!(box_L > 0)) return fail(DSU_EINVAL, "box_L must be positive");
    if (budget_bytes < 4096) return fail(DSU_EINVAL, "budget too small");
    if (recompute_every < 0) return fail(DSU_EINVAL, "recompute_every < 0");
    dsu_server *s = new dsu_server();
    s->K = k_delay;
    s->prec = precision;
    s->L = box_L;
    s->budget = budget_bytes;
    s->recompute_every = recompute_every;
    hipError_t e = hipMalloc((void **)&s->arena_base, budget_bytes);
    if (e != hipSuccess) {
        delete s;
        return fail(DSU_ENOMEM, "arena of %zu bytes: %s", budget_bytes, hipGetErrorString(e));
    }
    s->arena.reset(budget_bytes);
    *out = s;
    return DSU_OK;
}

extern "C" int dsu_server_destroy(dsu_server *s) {
    if (!s) return fail(DSU_EINVAL, "server is NULL");
    for (auto &kv : s->buckets) {
        kv.second->bk.release();
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    }
    s->buckets.clear();
    dfree(s->arena_base);
    delete s;
    return DSU_OK;
}

extern "C" int dsu_server_add(dsu_server *s, const dsu_request *req, int32_t *slot_out) {
    if (!s || !req) return fail(DSU_EINVAL, "NULL argument");
    auto it = s->buckets.find(req->n);
    if (it != s->buckets.end() && it->second->busy) return fail(DSU_ESTATE, "bucket busy");
    int slot = -1;
    CHK(admit(s, *req, 0.0, -1, &slot));
    BucketState *b = s->buckets[req->n].get();
    HIPCHK(hipStreamSynchronize(b->bk.stream));
    const std::vector<int> bad = flag_singular(s, b);
    if (std::find(bad.begin(), bad.end(), slot) != bad.end()) {
        retire(s, slot);
        drop_empty_buckets(s);
        return fail(DSU_ESINGULAR, "request %llu: Slater matrix is singular", (unsigned long long)req->request_id);
    }
    if (slot_out) *slot_out = slot;
    return DSU_OK;
}

extern "C" int dsu_server_step(dsu_server *s) {
    if (!s) return fail(DSU_EINVAL, "server is NULL");
    for (auto &kv : s->buckets) {
        BucketState *b = kv.second.get();
        if (b->dirty) CHK(refresh_bucket(s, b));
        if (b->members.empty()) continue;
        CHK(b->bk.sweep(0));
        HIPCHK(hipEventRecord(b->done, b->bk.stream));
        b->busy = true;
    }
    for (auto &kv : s->buckets) {
        BucketState *b = kv.second.get();
        if (!b->busy) continue;
        HIPCHK(hipEventSynchronize(b->done));
        b->busy = false;
        (void)flag_singular(s, b);
        for (int slot : b->members) s->resident[slot].sweeps_done += 1;
        CHK(recompute_due(s, b));
    }
    return DSU_OK;
}

extern "C" int dsu_server_result(dsu_server *s, int32_t slot, dsu_result *out, int32_t remove) {
    if (!s || !out) return fail(DSU_EINVAL, "NULL argument");
    if (!s->resident.count(slot)) return fail(DSU_EINVAL, "no walker in slot %d", slot);
    const int n = s->resident[slot].n;
    auto it = s->buckets.find(n);
    if (it != s->buckets.end() && it->second->busy) return fail(DSU_ESTATE, "bucket busy");
    CHK(read_result(s, slot, out));
    if (remove) {
        retire(s, slot);
        drop_empty_buckets(s);
    }
    return DSU_OK;
}

extern "C" int dsu_server_usage(dsu_server *s, size_t *used_bytes, int32_t *resident_walkers) {
    if (!s) return fail(DSU_EINVAL, "server is NULL");
    if (used_bytes) *used_bytes = s->arena.used;
    if (resident_walkers) *resident_walkers = (int32_t)s->resident.size();
    return DSU_OK;
}

extern "C" int dsu_server_run(dsu_server *s, const dsu_request *reqs, int32_t count, dsu_result *results,
                              double *sweep_latency_ms, int64_t latency_cap, int64_t *latency_count) {
    if (!s || (count > 0 && (!reqs || !results))) return fail(DSU_EINVAL, "NULL argument");
    if (!s->resident.empty()) return fail(DSU_ESTATE, "server already has resident walkers");
    typedef std::chrono::steady_clock clk;
    const auto t0 = clk::now();
    auto now_s = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
    int next = 0, completed = 0;
    int64_t nlat = 0;
    std::deque<int> waiting;
    for (int i = 0; i < count; ++i) {
        results[i] = dsu_result{};
        results[i].request_id = reqs[i].request_id;
        results[i].status = DSU_EBUDGET;
    }
    while (completed < count) {
        const double t = now_s();
        while (next < count && reqs[order[next]].arrival_s <= t) waiting.push_back(order[next++]);
        // sweep completions
        for (auto &kv : s->buckets) {
            BucketState *b = kv.second.get();
            if (!b->busy) continue;
            const hipError_t q = hipEventQuery(b->done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return fail(DSU_EDEVICE, "hipEventQuery: %s", hipGetErrorString(q));
            b->busy = false;
            const double td = now_s();
            // walkers whose (re)computed inverse came out singular leave with that status
            for (int slot : flag_singular(s, b)) {
                CHK(read_result(s, slot, &results[s->resident[slot].result_index]));
                retire(s, slot);
                ++completed;
            }
            std::vector<int> finished;
            for (int slot : b->members) {
                Resident &w = s->resident[slot];
                w.sweeps_done += 1;
                if (sweep_latency_ms && nlat < latency_cap) sweep_latency_ms[nlat] = 1e3 * (td - w.last_s);
                ++nlat;
                w.last_s = td;
                if (w.sweeps_done >= w.sweeps_target) finished.push_back(slot);
            }
            for (int slot : finished) {
                dsu_result &res = results[s->resident[slot].result_index];
                CHK(read_result(s, slot, &res));
                retire(s, slot);
                ++completed;
            }
            CHK(recompute_due(s, b));
        }
        drop_empty_buckets(s);
        // admission, first fit in arrival order, into idle buckets
        for (auto it = waiting.begin(); it != waiting.end();) {
            const dsu_request &r = reqs[*it];
            auto bit = s->buckets.find(r.n);
            if (bit != s->buckets.end() && bit->second->busy) {
                ++it;
                continue;
            }
            if (walker_bytes(r.n, r.spins, s->K, s->prec) + bucket_ws_bytes(r.n) > s->budget || r.sweeps == 0) {
                results[*it].status = r.sweeps == 0 ? DSU_OK : DSU_EBUDGET;
                results[*it].admit_s = results[*it].finish_s = now_s();
                ++completed;
                it = waiting.erase(it);
                continue;
            }
            int slot = -1;
            const int rc = admit(s, r, now_s(), *it, &slot);
            if (rc == DSU_EBUDGET) {
                ++it;
                continue;
            }
            if (rc != DSU_OK) return rc;
            it = waiting.erase(it);
        }
        // launch the next sweep of every idle, non-empty bucket
        bool any_busy = false;
        for (auto &kv : s->buckets) {
            BucketState *b = kv.second.get();
            if (!b->busy) {
                if (b->dirty) CHK(refresh_bucket(s, b));
                if (!b->members.empty()) {
                    CHK(b->bk.sweep(0));
                    HIPCHK(hipEventRecord(b->done, b->bk.stream));
                    b->busy = true;
                }
            }
            any_busy = any_busy || b->busy;
        }
        if (!any_busy) {
            if (next < count) {
                const double wait = reqs[order[next]].arrival_s - now_s();
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            } else if (!waiting.empty() && s->resident.empty()) {
                return fail(DSU_EBUDGET, "waiting requests cannot be admitted into an empty pool");
            }
        } else {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    if (latency_count) *latency_count = std::min(nlat, latency_cap);
    return DSU_OK;
}
