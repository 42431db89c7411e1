/*
 * dsu.h -- C ABI of libdsu, the MI355X (gfx950) delayed Slater-determinant
 * update library (McDaniel, D'Azevedo, Li, Wong, Kent, arXiv:1708.00744).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrix convention: the Slater matrix A has one ROW per electron,
 *    A[i][j] = phi_j(r_i), FP64, row-major.  This is the transpose of the
 *    paper's layout (Sec. I puts electrons in columns); determinants and
 *    ratios are identical.  Moving electron e replaces row e of A.
 *  - The library keeps the transposed inverse BT = (A^{-1})^T on the device,
 *    so column e of A^{-1} (needed by the ratio, eq. (1)) is a contiguous row.
 *  - Every call returns DSU_OK (0) or a negative status; on error the object
 *    is unchanged and dsu_last_error() returns a thread-local message.
 *    No call throws across the ABI.
 *  - Ownership: the caller keeps every array it passes; the library copies
 *    what it needs during the call.  All device memory behind a handle is
 *    owned by the library and released by the matching *_destroy.
 *  - Pointers named *_host are host memory; *_dev are device memory.
 *  - Calls on one handle must be serialised by the caller; distinct handles
 *    may be used from distinct threads.
 *  - Streams: `hip_stream` is a hipStream_t (e.g. torch's
 *    current_stream().cuda_stream) or NULL, in which case the handle creates
 *    its own non-blocking stream of default priority.  Work is stream
 *    ordered; calls that return numbers to the host synchronise that stream.
 */
#ifndef DSU_H
#define DSU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- status codes */
enum {
    DSU_OK = 0,
    DSU_EINVAL = -1,     /* bad argument (size, index, pointer, enum)          */
    DSU_ENOMEM = -2,     /* device or host allocation failed                    */
    DSU_ESINGULAR = -3,  /* matrix singular, or a zero / non-finite ratio     */
    DSU_ESTATE = -4,     /* call not valid in the handle's current state        */
    DSU_EDEVICE = -5,    /* a HIP runtime call failed                           */
    DSU_EBUDGET = -6     /* request does not fit the pool's device-memory budget */
};

/* Precision forms. */
enum {
    DSU_FP64 = 0,        /* inverse, ratios and flushes in FP64                 */
    DSU_FP32_MIXED = 1   /* BT, ratios, flushes in FP32 (FP32 accumulation);
                            A, log-determinant, K x K bordering and every
                            recompute of the inverse in FP64                  */
};

/* What counts toward the delay K (Sec. II, handling of rejected moves). */
enum {
    DSU_FLUSH_K_ACCEPTED = 0, /* flush after K accepted moves                   */
    DSU_FLUSH_K_PROPOSED = 1  /* flush after K proposals; a rejected move takes
                                 a slot but contributes nothing (a zero-rank
                                 term), so every flush is uniform work          */
};

/* Flush kernel selection for the single-walker form. */
enum {
    DSU_FLUSH_AUTO = 0,  /* VALU for k <= 4, matrix cores above                  */
    DSU_FLUSH_VALU = 1,  /* vector-ALU rank-k kernel                             */
    DSU_FLUSH_MFMA = 2   /* fused matrix-core (MFMA) rank-k kernel               */
};

#define DSU_MAX_K 256    /* largest supported delay */

const char *dsu_last_error(void);
/* Library version (major*10000 + minor*100 + patch). */
int dsu_version(void);

/* Bytes of device memory one determinant of size n needs in the batched
 * form (inverse, delayed buffers, window scratch), excluding the shared
 * recompute workspace.  0 on a bad argument. */
size_t dsu_footprint_bytes(int32_t n, int32_t k_delay, int32_t precision);

/* Plane-wave orbitals phi_j(r) = 1, cos(k.r), sin(k.r), k = (2 pi / L) n
 * (n integer; shells of |n|^2 in ascending order, inside a shell the vectors
 * whose first nonzero component is positive in ascending (nx, ny, nz); n = 0
 * gives the constant, every other vector cos then sin).  The batched form
 * uses these as the N single-particle functions of the Slater matrix
 * (Sec. I).  dsu_plane_wave_table writes {nx, ny, nz, kind} per orbital
 * (kind 0 = 1, 1 = cos, 2 = sin; host only, no device needed).
 * dsu_plane_wave_rows evaluates rows_host[c][j] = phi_j(positions_host[c])
 * for `count` positions (count*3 FP64 in, count*n FP64 out) on the device. */
int dsu_plane_wave_table(int32_t n, int32_t *out4);
int dsu_plane_wave_rows(int32_t n, double box_L, int32_t count, const double *positions_host, double *rows_host);

/* ======================================================================
 * Single walker, host-driven: the paper's procedure one call per step.
 * ====================================================================== */
typedef struct dsu_walker dsu_walker;

/* Create a walker from the Slater matrix `slater_host` (n*n FP64, row i =
 * electron i).  Computes A^{-1} and log|det A| in FP64 on the device
 * (blocked Gauss-Jordan with partial pivoting: the explicit route of
 * Sec. I).  k_delay in [1, DSU_MAX_K]; k_delay = 1 is plain Sherman-Morrison,
 * eq. (2).  DSU_ESINGULAR if A is singular to working precision (a pivot at
 * or below n * 2^-52 times the largest pivot). */
int dsu_walker_create(int32_t n, int32_t k_delay, int32_t precision, int32_t policy,
                      const double *slater_host, void *hip_stream, dsu_walker **out);
int dsu_walker_destroy(dsu_walker *w);

/* Ratio det(A_new)/det(A) for replacing row `electron` by `phi_host` (n FP64
 * values): eq. (1) against the stale inverse, corrected for the k pending
 * accepted moves by the generalised lemma, eq. (3) (look-ahead,
 * R = r0 - p^T C_k^{-1} q).  The proposal stays pending until dsu_accept or
 * dsu_reject; a new proposal replaces it.  If `electron` already has a pending
 * accepted move, the pending moves are flushed first.  Synchronises. */
int dsu_propose_ratio(dsu_walker *w, int32_t electron, const double *phi_host, double *ratio_out);
/* Same, with the row already on the device in the walker's precision
 * (double for DSU_FP64, float for DSU_FP32_MIXED), n values. */
int dsu_propose_ratio_dev(dsu_walker *w, int32_t electron, const void *phi_dev, double *ratio_out);

/* Ratio and its gradient with respect to the proposed position: the
 * drift-diffusion move of DMC (Sec. II: short time steps, high acceptance)
 * needs grad R / R at the proposed point.  The determinant is linear in the
 * replaced row, so the eq. (3) look-ahead applied to the three derivative
 * rows gives grad R with the same C_k^{-1} q as R (3 more products of
 * length n against BT row e and each pending Vg row).  dphi_host is 3*n FP64,
 * row-major: dphi_host[a*n + j] = d phi_j / d r_a (a = x, y, z) at the
 * proposed position.  grad_out receives 3 values (grad R, not grad R / R).
 * The proposal stays pending exactly as for dsu_propose_ratio (same repeat
 * rule, same dsu_accept / dsu_reject).  Synchronises.  DSU_EINVAL on a NULL
 * pointer or an electron out of range. */
int dsu_propose_ratio_grad(dsu_walker *w, int32_t electron, const double *phi_host, const double *dphi_host,
                           double *ratio_out, double *grad_out);
/* Drift at the present configuration: grad_e ln|det A| = dphi . A_k^{-1}[:, e]
 * with dphi (3*n FP64, as above) the gradient rows of electron `electron`'s
 * present row, A_k the matrix with every pending accepted move applied (the
 * same look-ahead; if the electron itself holds a pending move, its slot's
 * unit vector is taken out of the right-hand side).  Reads only: a pending
 * proposal stays pending and nothing is flushed.  Synchronises. */
int dsu_eval_grad(dsu_walker *w, int32_t electron, const double *dphi_host, double *grad_out);

/* Accept the pending proposal: queue it in the delayed buffer (Sec. II),
 * border the K x K inverse, update A's row and the running log-determinant.
 * When the delay limit is reached the queued moves are applied en bloc by
 * the Woodbury formula, eq. (4).  DSU_ESTATE without a pending proposal;
 * DSU_ESINGULAR (walker unchanged) if the ratio is not finite or |R| <= 1e-12
 * (1e-6 in DSU_FP32_MIXED): the updated matrix would be numerically singular,
 * and a Metropolis test accepts such a move with probability R^2 below 1e-24
 * (1e-12).  The batched form rejects such proposals the same way. */
int dsu_accept(dsu_walker *w);
/* Drop the pending proposal.  Under DSU_FLUSH_K_PROPOSED it still takes a
 * slot toward K. */
int dsu_reject(dsu_walker *w);
/* Apply the k pending moves now (eq. (4)); no-op when k = 0. */
int dsu_flush(dsu_walker *w);
/* Recompute A^{-1} from scratch in FP64 (Sec. III's direct calculation).  If
 * `slater_host_or_null` is given it replaces A first.  Pending moves are
 * already part of A, so the delayed buffer is cleared.  Writes the fresh
 * log|det| and sign when the pointers are non-NULL; `drift_out` (optional)
 * receives running-minus-fresh log|det| before re-basing. */
int dsu_recompute_inverse(dsu_walker *w, const double *slater_host_or_null, double *logdet_out,
                          int32_t *sign_out, double *drift_out);
/* Flush, then copy A^{-1} (natural layout, n*n FP64) to the host. */
int dsu_get_inverse(dsu_walker *w, double *out_host);
/* Running log|det A| and its sign (FP64, maintained from accepted ratios). */
int dsu_get_logdet(dsu_walker *w, double *logdet, int32_t *sign);
/* Number of accepted moves waiting in the delayed buffer. */
int dsu_walker_pending(dsu_walker *w, int32_t *k_out);
/* Choose the flush kernel (DSU_FLUSH_*) -- for the VALU/MFMA crossover study. */
int dsu_walker_set_flush_kernel(dsu_walker *w, int32_t mode);

/* Multideterminant expansion on a single reference (FP64 walkers; the
 * combination with single-reference multideterminant schemes noted at the end
 * of Sec. II).  Psi = sum_I coef[I] det(A_I): A_I is the walker's Slater
 * matrix with the occupied orbitals occ[4I .. 4I+order[I]) replaced by the
 * virtual orbitals virt[4I .. 4I+order[I]) (order 0 = the reference itself,
 * order <= 4, no orbital repeated within a determinant).  virt_host holds the
 * m virtual orbitals at every electron, n*m FP64, row i = electron i.  The
 * library keeps the table T = A^{-1} V; det(A_I)/det(A) is the determinant
 * of a submatrix of T of size order[I], and a move changes T by a rank-1 term
 * built from the delayed inverse's column of the moved electron (the eq. (3)
 * look-ahead), so the reference keeps its delayed updates.  Pending moves are
 * flushed and a pending proposal dropped.  Once set, proposals go through
 * dsu_propose_ratio_md (the other propose calls return DSU_ESTATE); a
 * dsu_recompute_inverse with a new matrix drops the expansion.  DSU_EINVAL for
 * a non-FP64 walker, m outside [1, 4096], a bad excitation; DSU_ESINGULAR if
 * Psi is zero. */
int dsu_walker_set_multidet(dsu_walker *w, int32_t m, const double *virt_host, int32_t ndet, const int32_t *order,
                            const int32_t *occ, const int32_t *virt, const double *coef);
/* Ratio Psi(new)/Psi(old) for moving `electron` to the point whose occupied
 * orbital values are phi_host (n) and virtual values vphi_host (m); the
 * reference ratio det(A_new)/det(A) goes to ratio_ref_out (may be NULL).
 * The proposal stays pending for dsu_accept / dsu_reject; dsu_accept returns
 * DSU_ESINGULAR if the reference ratio is below 1e-12 in modulus (the
 * single-reference update needs it) or Psi vanishes at the new point.
 * Synchronises. */
int dsu_propose_ratio_md(dsu_walker *w, int32_t electron, const double *phi_host, const double *vphi_host,
                         double *ratio_out, double *ratio_ref_out);
/* log|Psi| and sign(Psi) of the present configuration (running reference
 * log-determinant plus the expansion's ratio to the reference).  DSU_ESTATE
 * without an expansion. */
int dsu_walker_md_value(dsu_walker *w, double *logabs, int32_t *sign);

/* ======================================================================
 * Single walker with complex orbitals (twisted boundary conditions).
 * The same look-ahead (eq. (3)), bordering and en-bloc update (eq. (4)) in
 * FP64 complex arithmetic: the determinant lemma and the Woodbury identity
 * hold over the complex field with plain transposes.  Complex arrays are
 * interleaved (re, im) doubles, row-major, row i = electron i.  The
 * Metropolis weight of a move is |R|^2; the walker tracks log|det A| and
 * arg det A in (-pi, pi].
 * ====================================================================== */
typedef struct dsu_zwalker dsu_zwalker;

/* Create from the complex Slater matrix (2*n*n doubles).  Computes A^{-1},
 * log|det A| and arg det A in FP64 complex on the device (Gauss-Jordan with
 * partial pivoting by modulus).  n in [1, 16384], k_delay in [1, DSU_MAX_K],
 * policy as for dsu_walker_create.  DSU_ESINGULAR if A is singular to working
 * precision (a pivot at or below n * 2^-52 times the largest pivot). */
int dsu_zwalker_create(int32_t n, int32_t k_delay, int32_t policy, const double *slater_host, void *hip_stream,
                       dsu_zwalker **out);
int dsu_zwalker_destroy(dsu_zwalker *w);
/* Complex ratio for replacing row `electron` by phi_host (2*n doubles):
 * eq. (3) look-ahead; ratio_out receives (re, im).  The proposal stays
 * pending until dsu_zaccept / dsu_zreject; an electron holding a pending
 * accepted move flushes the pending moves first.  Synchronises. */
int dsu_zpropose_ratio(dsu_zwalker *w, int32_t electron, const double *phi_host, double *ratio_out);
/* Accept the pending proposal (bordering; flush by the walker's policy).
 * DSU_ESTATE without a pending proposal; DSU_ESINGULAR (walker unchanged) if
 * |R| <= 1e-12 or R is not finite. */
int dsu_zaccept(dsu_zwalker *w);
int dsu_zreject(dsu_zwalker *w);
/* Apply the pending moves now (eq. (4)). */
int dsu_zflush(dsu_zwalker *w);
/* Fresh inverse from the walker's current A (or from slater_host_or_null,
 * which then replaces A); log|det|, arg det and running-minus-fresh log|det|
 * out (each may be NULL).  Clears pending moves. */
int dsu_zrecompute_inverse(dsu_zwalker *w, const double *slater_host_or_null, double *logabs_out, double *phase_out,
                           double *drift_out);
/* A^{-1} (2*n*n doubles, row-major) after flushing pending moves. */
int dsu_zget_inverse(dsu_zwalker *w, double *out_host);
/* Running log|det A| and arg det A (sum of log|R| and arg R of accepted moves
 * since the last fresh inverse). */
int dsu_zget_logdet(dsu_zwalker *w, double *logabs, double *phase);
int dsu_zwalker_pending(dsu_zwalker *w, int32_t *k_out);
/* Flush kernel of the complex walker.  W = (BT U^T - E) C^{-T} is formed row
 * by row on the vector ALUs; the rank-k update BT -= W Vg then runs, with
 * DSU_FLUSH_MFMA, on the FP64 matrix cores through the real embedding of the
 * complex operands (the inverse and W read as real rows of interleaved
 * doubles, Vg expanded to 2k real rows: each complex product as its four real
 * products), tiled over rows and columns, when 2k <= 256; otherwise, and
 * with DSU_FLUSH_VALU, as a complex product on the vector ALUs.  DSU_FLUSH_AUTO (default): the matrix cores for k > 2. */
int dsu_zwalker_set_flush_kernel(dsu_zwalker *w, int32_t mode);

/* ======================================================================
 * Batched form: many walker determinants of one size n, proposals drawn on
 * the device, lock-step windows of K proposals per determinant.
 * ====================================================================== */
typedef struct dsu_batch dsu_batch;

/* Create a batch of `walkers` walkers with `spins` (1 or 2) determinants of
 * size n each.  Per walker: RNG key (seeds[w], walker_ids[w]) -- Philox4x64-10
 * counter = (sweep, spin*n + electron, block, 0) --, Gaussian step sigma[w],
 * and initial positions positions_host[w][spin][n][3] in the periodic cubic
 * box of side box_L (orbitals: plane waves cos/sin(k.r), k = 2 pi n / L, by
 * shells of |n|^2).  Builds each A and inverts it in FP64 on the device.
 * recompute_every: FP64 recompute of every inverse after that many sweeps of
 * a walker (0 = never).  Policy is DSU_FLUSH_K_PROPOSED (lock-step windows). */
int dsu_batch_create(int32_t walkers, int32_t n, int32_t spins, int32_t k_delay, int32_t precision,
                     double box_L, const uint64_t *seeds, const uint64_t *walker_ids, const double *sigma,
                     const double *positions_host, int32_t recompute_every, void *hip_stream, dsu_batch **out);
int dsu_batch_destroy(dsu_batch *b);
/* Run `sweeps` Monte Carlo sweeps on every walker: per sweep and determinant,
 * electrons 0..n-1 in windows of K: propose, look-ahead ratio (eq. (3)),
 * Metropolis decision u < R^2 (or accept all with force_accept, the paper's
 * 100% acceptance test mode), then the en-bloc Woodbury update (eq. (4)).
 * Stream ordered: returns once the work is enqueued; dsu_batch_sync waits. */
int dsu_batch_sweep(dsu_batch *b, int32_t sweeps, int32_t force_accept);
int dsu_batch_sync(dsu_batch *b);
/* FP64 recompute of every inverse now; drift_out (optional, walkers*spins)
 * receives running-minus-fresh log|det| before re-basing. */
int dsu_batch_recompute(dsu_batch *b, double *drift_out);
/* Per determinant d = w*spins + s: running log|det|, sign, accepted moves,
 * completed sweeps.  Any pointer may be NULL.  Synchronises. */
int dsu_batch_stats(dsu_batch *b, double *logdet, int32_t *sign, int64_t *accepted, int64_t *sweeps_done);
/* Resume: set every determinant's completed-sweep count, which keys the
 * random stream of its next sweep (Philox counter word 0).  A checkpoint is
 * {positions (dsu_batch_get_positions), seeds, walker ids, sweeps done}; a
 * batch created from it (fresh FP64 inverses) and set to the same count
 * proposes and draws exactly what the uninterrupted batch would.  Takes
 * effect at the next sweep.  DSU_EINVAL for a negative count. */
int dsu_batch_set_sweep(dsu_batch *b, int64_t sweeps_done);
/* Watchdog (enable = 1): after every sweep, determinants that met a zero or
 * non-finite ratio during it get a fresh FP64 inverse from their positions
 * (dsu_batch_recompute of those members only); the others are untouched.
 * Costs one synchronisation per sweep.  dsu_batch_watchdog_count reports the
 * number of such recomputes so far. */
int dsu_batch_set_watchdog(dsu_batch *b, int32_t enable);
int dsu_batch_watchdog_count(dsu_batch *b, int64_t *recomputes);
/* Sampled residuals of every determinant's device inverse X against its
 * Slater matrix A (Sec. III checks the delayed updates against a direct
 * calculation), A rebuilt in FP64 from the current positions, X converted
 * exactly to FP64, products on FP64 matrix cores.  With S = samples and
 * t = sweeps_done mod (n / S):
 *   right_host[d] = max |(A X - I)[r][j]| over the S rows r = s * (n / S) + t
 *                   (s < S) and every column j;
 *   left_host[d]  = max |(X A - I)[i][j]| over the S consecutive rows
 *                   i = t * S + s (s < S) and every column j;
 * +inf if an entry is not finite.  The rows visited rotate with the completed
 * sweeps, so n / S consecutive sweeps cover every row below S * (n / S).
 * For a proposal close to the present position the ratio error is about the
 * right residual's diagonal entry; the left residual is the norm
 * ||A^{-1} A - I|| of the FP32 form's accuracy statement.  Either output may
 * be NULL (its kernel is skipped), not both.  samples in [1, min(64, n)],
 * else DSU_EINVAL.  Synchronises. */
int dsu_batch_residual(dsu_batch *b, int32_t samples, double *right_host, double *left_host);
/* dsu_batch_residual for callers that cannot allocate device memory (code
 * under HIP graph capture nearby, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, with every device buffer
 * (sample rows, sample indices, result words) carved from one static 32 MiB
 * array per GPU that the library holds until the process ends; nothing is
 * allocated, on the device or the host.  Needed: 16 * ndet and
 * 4 * ndet * S' bytes, each rounded up to 256, plus ndet * S' * np * 8
 * (S' = samples rounded up to 16, 32 or 64; np = n rounded up to 64;
 * ndet = walkers * spins), at most 32 MiB: e.g. 32 determinants of
 * n = 4096 with up to 32 samples; a batch that needs more gets DSU_EINVAL
 * with the figure, and nothing runs.  Call with the batch's device current.  Every call on one GPU
 * shares that GPU's array, whose contents the next call overwrites (the
 * kernels clear what must start at zero): calls that overlap on one GPU, from
 * threads or streams, race.  Synchronises the batch's stream. */
int dsu_batch_residual_noalloc(dsu_batch *b, int32_t samples, double *right_host, double *left_host);
/* Residual watchdog (the adaptive recompute of the FP32 form): after every
 * sweep, the sampled right residual above for every determinant; a
 * determinant whose right residual exceeds `threshold` (or is not finite)
 * gets a fresh FP64 inverse at once, from its positions.  The right residual
 * is the one that bounds the ratios: a proposal phi~ = A[e, :] + delta has
 * R_computed - R = F[e][e] + delta A^{-1} F[:, e] with F = A X - I, so for the
 * small moves of a high-acceptance run the relative ratio error is about
 * F[e][e].  samples = 0 turns it off; otherwise samples as for
 * dsu_batch_residual and threshold > 0, else DSU_EINVAL.  Costs the right
 * residual's kernels (one pass over every inverse) and one synchronisation
 * per sweep. */
int dsu_batch_set_residual_watchdog(dsu_batch *b, int32_t samples, double threshold);
/* Blocking of the FP64 Gauss-Jordan recompute (Sec. III's direct
 * calculation; the paper leaves such parameters to an autotuner, Sec. II):
 * panel = columns factored per pass over the matrix (16, 32, 64, or 128 =
 * two 64-column panels factored one after the other that share one pass;
 * single 64-column panels where fewer than 128 columns remain or the padded
 * n exceeds 4096), chunk = columns of the single-panel trailing update per
 * step (32, or 64 when n rounded up to a multiple of 64 is a multiple of
 * 128; a pair's update takes 32), apply_columns = panel columns one
 * workgroup updates after each group of pivots (1 or 4).  0 keeps the
 * built-in choice for this n.  Results agree to FP64 rounding whatever the
 * choice.  Waits for the batch's stream; DSU_EINVAL for other values. */
int dsu_batch_set_recompute_tiles(dsu_batch *b, int32_t panel, int32_t chunk, int32_t apply_columns);
/* The blocking in use (any output may be NULL). */
int dsu_batch_get_recompute_tiles(dsu_batch *b, int32_t *panel, int32_t *chunk, int32_t *apply_columns);
/* Accuracy record, per determinant d (any pointer may be NULL):
 * residual_out[d] = the sampled right residual after the latest sweep run
 * with the residual watchdog on (before any recompute it triggered; 0 before
 * the first); drift_out[d] = running-minus-fresh log|det| found by the latest
 * FP64 recompute of d (periodic, either watchdog, or dsu_batch_recompute; 0
 * before the first after creation); *residual_recomputes = recomputes the
 * residual watchdog has made. */
int dsu_batch_accuracy(dsu_batch *b, double *residual_out, double *drift_out, int64_t *residual_recomputes);
/* Fault injection for tests of the failure handling: overwrite row `row` of
 * determinant `det`'s device inverse with NaN.  Synchronises. */
int dsu_batch_poison_row(dsu_batch *b, int32_t det, int32_t row);
/* Current positions of determinant d (n*3 FP64). */
int dsu_batch_get_positions(dsu_batch *b, int32_t det, double *out_host);
/* A^{-1} of determinant d, natural layout (n*n FP64, from the device copy). */
int dsu_batch_get_inverse(dsu_batch *b, int32_t det, double *out_host);
/* Record per-move ratios and decisions for the next `sweeps` sweeps
 * (0 disables).  dsu_batch_get_trace copies determinant d's record:
 * ratio[sweeps*n] (FP64) and accepted[sweeps*n]. */
int dsu_batch_set_trace(dsu_batch *b, int32_t sweeps);
int dsu_batch_get_trace(dsu_batch *b, int32_t det, double *ratio_host, uint8_t *accepted_host);
/* Kernel timing: enable = 1 brackets every launch with HIP events on the
 * stream it runs on, 2 only the flush launches (phase 3: fewer events
 * between kernels, so the rest of the sweep runs as untimed), 0 none (and
 * sweeps may replay a captured graph again); any other value is DSU_EINVAL.
 * Each call clears the totals.  dsu_batch_kernel_time returns (count,
 * total ms) for one phase: 0 proposals, 1 look-ahead products, 2 decisions,
 * 3 flush, 4 recompute. */
int dsu_batch_set_timing(dsu_batch *b, int32_t enable);
int dsu_batch_kernel_time(dsu_batch *b, int32_t phase, int64_t *launches, double *total_ms);
/* Capture one sweep into a hipGraph and replay it for dsu_batch_sweep
 * (enable = 1) or launch kernels directly (0). */
int dsu_batch_use_graph(dsu_batch *b, int32_t enable);
/* Change the delay K of a live batch (1 <= k_delay <= the K it was created
 * with; Sec. II: K is the tunable of the method).  Takes effect at the next
 * sweep. */
int dsu_batch_set_delay(dsu_batch *b, int32_t k_delay);

/* ======================================================================
 * Serving: a pool of walkers of mixed n admitted by a device-memory budget,
 * continuously batched (one lock-step batch per n, on its own stream).
 * ====================================================================== */
typedef struct dsu_server dsu_server;

typedef struct {
    uint64_t request_id;
    int32_t n;              /* determinant size per spin                          */
    int32_t spins;          /* 1 or 2 determinants per walker                     */
    uint64_t seed;          /* RNG key word 0 (request seed); word 1 = request_id */
    double sigma;           /* Gaussian step                                      */
    int32_t sweeps;         /* sweeps to run                                      */
    double arrival_s;       /* arrival time, seconds after dsu_server_run starts   */
    const double *positions;/* spins*n*3 FP64 initial positions (host)           */
} dsu_request;

typedef struct {
    uint64_t request_id;
    int32_t status;         /* DSU_OK, or DSU_EBUDGET if it can never fit         */
    int32_t sweeps_done;
    double admit_s;         /* time admitted (s after start)                      */
    double finish_s;        /* time its last sweep completed                      */
    double logdet[2];       /* per spin, running log|det|                         */
    int32_t sign[2];
    int64_t accepted;       /* accepted moves over all spins and sweeps           */
} dsu_result;

/* budget_bytes: device memory the pool may use (one arena, allocated here)
 * for walker state and, for every size n with a resident walker, that size's
 * FP64 recompute workspace (four determinants per pass; released when the
 * size's last walker leaves); requests wait until enough is free.  Beyond the
 * arena the pool holds only descriptor arrays, the orbital table and
 * streams (under 1 MB per size).  recompute_every as in dsu_batch_create. */
/* Bytes of the budget a pool charges for the recompute workspace of size n
 * while walkers of that size are resident (0 on a bad n). */
size_t dsu_server_workspace_bytes(int32_t n);
int dsu_server_create(int32_t k_delay, int32_t precision, double box_L, size_t budget_bytes,
                      int32_t recompute_every, dsu_server **out);
int dsu_server_destroy(dsu_server *s);
/* Manual control.  dsu_server_add admits one walker now (its arrival_s is
 * ignored) and waits for its FP64 inverses: DSU_EBUDGET if it does not fit
 * the free budget, DSU_EINVAL if it never can, DSU_ESINGULAR (not admitted)
 * if a determinant is singular.  dsu_server_step runs one sweep of every
 * resident walker (the sizes concurrently) and waits.  dsu_server_result
 * reads a walker's result (status DSU_ESINGULAR if a periodic recompute found
 * its matrix singular); with remove = 1 it also retires the walker and frees
 * its memory.  dsu_server_usage reports arena bytes in use and resident
 * walkers. */
int dsu_server_add(dsu_server *s, const dsu_request *req, int32_t *slot_out);
int dsu_server_step(dsu_server *s);
int dsu_server_result(dsu_server *s, int32_t slot, dsu_result *out, int32_t remove);
int dsu_server_usage(dsu_server *s, size_t *used_bytes, int32_t *resident_walkers);
/* Serve `count` requests in arrival order (wall clock): admit by budget,
 * sweep all resident walkers (one batch per n, concurrently), retire
 * finished ones.  Fills results[count]; a walker whose matrix is singular
 * at admission or at a recompute ends early with status DSU_ESINGULAR (the
 * inverses are computed on the device ahead of the walker's next sweep, so
 * admission never waits for them).  sweep_latency_ms (optional,
 * capacity latency_cap) receives every per-walker sweep latency: the time
 * between consecutive sweep completions of a walker (the first measured from
 * its admission); *latency_count is the number written. */
int dsu_server_run(dsu_server *s, const dsu_request *reqs, int32_t count, dsu_result *results,
                   double *sweep_latency_ms, int64_t latency_cap, int64_t *latency_count);

#ifdef __cplusplus
}
#endif
#endif /* DSU_H */
