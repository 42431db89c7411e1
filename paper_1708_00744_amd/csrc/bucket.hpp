// bucket.hpp -- a lock-step group of same-size determinants of the batched
// form.  A bucket owns the launch machinery (descriptor arrays, stream,
// recompute workspace, optional hipGraph of a sweep, kernel timing); the
// determinants' storage belongs to whoever created them (one contiguous
// block for dsu_batch, an arena for dsu_server), so members can join and
// leave between sweeps.
#pragma once
#include <utility>
#include <vector>

#include "host_common.hpp"

namespace dsu {

// Device storage of one determinant.
struct DetSlot {
    void *bt = nullptr, *u = nullptr, *vg = nullptr, *u2 = nullptr, *vg2 = nullptr, *y = nullptr;
    double *cfl = nullptr, *cwork = nullptr, *gwork = nullptr, *prop = nullptr, *pos = nullptr, *prop2 = nullptr;
    float *cfl32 = nullptr;
    int *idx = nullptr;
    DetState *st = nullptr;
    double *trace_r = nullptr;
    uint8_t *trace_a = nullptr;
    long long trace_cap = 0;
    uint64_t seed = 0, wid = 0;
    double sigma = 0.0;
    int spin = 0;
};

// Sizes shared by every determinant of a bucket.
struct BucketShape {
    int n = 0, np = 0, kmax = 0, kp = 0, prec = 0;
    static BucketShape make(int n, int kmax, int prec);
    size_t det_bytes() const;            // one determinant's storage, 256-byte aligned pieces
    DetSlot carve(char *base) const;     // split a det_bytes() block into its arrays
};

enum { PH_ROWS = 0, PH_G = 1, PH_DECIDE = 2, PH_FLUSH = 3, PH_RECOMPUTE = 4, PH_COUNT = 5 };

class Bucket {
  public:
    BucketShape sh;
    int K = 0;  // current delay (<= sh.kmax)
    double L = 0.0, twopi_l = 0.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;  // proposals of the next window, beside the current window's decisions
    int4 *kvec = nullptr;
    int kmax_comp = 0;  // largest |component| of the plane-wave integer vectors
    std::vector<DetSlot> dets;
    bool use_graph = false;
    int timing = 0;  // 0 off, 1 events around every launch, 2 around flush launches only

    // gj_block (optional): GjWork::block_bytes(gj_group, np, n) bytes of the
    // caller's device memory for the recompute workspace (else allocated here).
    int init(const BucketShape &shape, int k_delay, double box_l, void *stream_or_null, int gj_group,
             void *gj_block = nullptr);
    void release();
    // Replace the member list (descriptors re-uploaded, graph invalidated).
    int set_dets(const std::vector<DetSlot> &d);
    int set_delay(int k);
    // One sweep of every member, stream ordered.
    int sweep(int force_accept);
    // FP64 recompute of the listed members (indices into dets); waits for it
    // and reports a singular matrix.  drift_dev (optional, per listed member)
    // receives running-minus-fresh log|det|.
    int recompute(const std::vector<int> &which, double *drift_host);
    // The same, only enqueued on the bucket's stream: nothing waits.  Status
    // words land in pinned host memory; once the stream has passed this point,
    // check_recompute() lists the members (indices into dets) found singular.
    // Several calls may be pending at once; members must not be reordered
    // until they are checked.
    int recompute_async(const std::vector<int> &which);
    void check_recompute(std::vector<int> *singular);
    // Sampled residuals of every member, A rebuilt from the positions: right =
    // max over `samples` rows of |A A^{-1} - I| (launch_resid), left = the same
    // for A^{-1} A - I (launch_resid_left); either may be NULL.  Waits.
    int residual(int samples, std::vector<double> *right, std::vector<double> *left);
    // The same into caller memory, with every device buffer carved from
    // `scratch` (scratch_bytes long): nothing allocated.  right_host and
    // left_host receive one double per member (either may be NULL).
    int residual_into(int samples, double *right_host, double *left_host, void *scratch, size_t scratch_bytes);
    // Scratch residual_into needs for the present members.
    size_t residual_scratch_bytes(int samples) const;
    // Pre-size the descriptor arrays for n members.
    int reserve(int n) { return ensure_capacity(n); }
    // Blocking of the FP64 recompute (panel width, update chunk, apply columns).
    GjTiles recompute_tiles() const { return gj_.tiles; }
    void set_recompute_tiles(const GjTiles &t) { gj_.tiles = t; }
    int harvest_events();
    long long t_count[PH_COUNT] = {0};
    double t_ms[PH_COUNT] = {0};

  private:
    int cap_ = 0;
    void *ddesc_ = nullptr, *fdesc_ = nullptr;
    void *sub_ddesc_ = nullptr;
    double **sub_pos_ = nullptr;
    void **sub_bt_ = nullptr;
    double *drift_ = nullptr;
    int *status_h_ = nullptr;      // pinned: one status word per pending recompute
    char *stage_h_ = nullptr;      // pinned: descriptor staging of pending recomputes
    std::vector<int> pending_;
    double *res_rows_ = nullptr;              // residual scratch, sized for res_cap_ members
    int *res_eidx_ = nullptr;
    unsigned long long *res_bits_ = nullptr;
    unsigned long long *res_host_ = nullptr;  // pinned
    int res_cap_ = 0;
    GjWork gj_;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t gexec_ = nullptr;
    int graph_force_ = -1;
    std::vector<hipEvent_t> ev_free_;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used_;

    int ensure_capacity(int n);
    int enqueue_sweep(int force_accept);
    int build_graph(int force_accept);
    void drop_graph();
    hipEvent_t ev_ring_[8] = {};
    template <typename F> int timed(int phase, F fn, hipStream_t on = nullptr);
    template <typename T> int upload_t();
    template <typename T> int enqueue_sweep_stream_t(int force_accept);
    template <typename T> int recompute_async_t(const std::vector<int> &which);
};

}  // namespace dsu
