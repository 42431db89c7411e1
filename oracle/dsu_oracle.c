/*
 * dsu_oracle.c -- plain, slow, sequential FP64 CPU oracle for the delayed
 * Slater-determinant update method of McDaniel, D'Azevedo, Li, Wong and Kent,
 * "Delayed Slater determinant update algorithms for high efficiency quantum
 * Monte Carlo" (arXiv:1708.00744).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the HIP implementation.
 *
 * What it computes is the *definition* the delayed scheme must reproduce: the
 * paper states (Sec. II, the paragraph after eq. (4)) that the delayed scheme
 * is exactly equivalent to applying every move one at a time.  So the oracle
 * applies every accepted move immediately with the rank-1 Sherman-Morrison
 * formula, eq. (2), and takes each acceptance ratio from the matrix
 * determinant lemma, eq. (1).  It never delays anything.
 *
 * Convention (transpose of the paper's, Sec. I): A[i][j] = phi_j(r_i), i.e.
 * electron i is ROW i.  Moving electron e replaces row e, so
 *   A_new = A + e_e (phi_new - A[e,:])
 * and eq. (1) with u = row change, v = e_e gives the ratio
 *   R = 1 + (phi_new - A[e,:]) . Ainv[:,e] = phi_new . Ainv[:,e].
 *
 * Parity pins live in tests/test_oracle_*.py (exact rational determinants,
 * numpy LU, numpy Philox, lattice shell counts, orthogonality).
 *
 * Build: gcc -O3 -march=x86-64-v3 -ffp-contract=off -fno-fast-math -fopenmp
 * -shared -fPIC (oracle/build.py).  Without contraction and without
 * reassociation the compiler keeps every sum in its source order, so the
 * optimisation level does not change a single result bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Written from the */
/* published round definition: two 64x64->128 multiplies per round, the     */
/* high halves xor-ed with the other counter words and the key, and a Weyl  */
/* key schedule.  Ten rounds.                                               */
/* ------------------------------------------------------------------------ */
static const uint64_t ORC_PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t ORC_PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t ORC_PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t ORC_PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1  */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += ORC_PHILOX_W0; k1 += ORC_PHILOX_W1; }
        __uint128_t p0 = (__uint128_t)ORC_PHILOX_M0 * x0;
        __uint128_t p1 = (__uint128_t)ORC_PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 53 random bits -> double in [0, 1). */
double orc_uniform53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Box-Muller (1958): two uniforms -> two independent standard normals.
 * 1 - u1 lies in (0, 1], so the logarithm is finite. */
static void orc_box_muller(double u1, double u2, double *z0, double *z1)
{
    double rad = sqrt(-2.0 * log(1.0 - u1));
    double th = 2.0 * ORC_PI * u2;
    *z0 = rad * cos(th);
    *z1 = rad * sin(th);
}

/* The random numbers of one proposed move.  Key = (seed, walker);
 * counter = (sweep, slot, block, 0) with slot = spin * n + electron.
 * Block 0: four words -> two Box-Muller pairs -> (gx, gy) and gz.
 * Block 1: first word -> the Metropolis uniform u. */
void orc_move_randoms(uint64_t seed, uint64_t walker, uint64_t sweep, uint64_t slot,
                      double g[3], double *u)
{
    uint64_t key[2] = {seed, walker};
    uint64_t c0[4] = {sweep, slot, 0, 0}, c1[4] = {sweep, slot, 1, 0};
    uint64_t w[4], v[4];
    orc_philox4x64_10(c0, key, w);
    orc_philox4x64_10(c1, key, v);
    double z0, z1, z2, z3;
    orc_box_muller(orc_uniform53(w[0]), orc_uniform53(w[1]), &z0, &z1);
    orc_box_muller(orc_uniform53(w[2]), orc_uniform53(w[3]), &z2, &z3);
    (void)z3;
    g[0] = z0; g[1] = z1; g[2] = z2;
    *u = orc_uniform53(v[0]);
}

/* ------------------------------------------------------------------------ */
/* Plane-wave orbitals phi_j(r) = 1, cos(k.r), sin(k.r), k = (2 pi / L) n,   */
/* n integer.  The Slater matrix of Sec. I needs N single-particle           */
/* functions; they are taken from the lowest |n|^2 shells.  Order: by |n|^2, */
/* then by (nx, ny, nz) ascending, over representatives whose first nonzero  */
/* component is positive (n and -n give the same cos/sin pair).  n = 0 gives */
/* the constant; each representative gives cos then sin.                    */
/* Output per orbital: {nx, ny, nz, kind} with kind 0 = 1, 1 = cos, 2 = sin. */
/* ------------------------------------------------------------------------ */
typedef struct { int nx, ny, nz, n2; } orc_rep;

static int orc_rep_less(const orc_rep *a, const orc_rep *b)
{
    if (a->n2 != b->n2) return a->n2 < b->n2;
    if (a->nx != b->nx) return a->nx < b->nx;
    if (a->ny != b->ny) return a->ny < b->ny;
    return a->nz < b->nz;
}

static int orc_rep_cmp(const void *pa, const void *pb)
{
    const orc_rep *a = (const orc_rep *)pa, *b = (const orc_rep *)pb;
    if (orc_rep_less(a, b)) return -1;
    if (orc_rep_less(b, a)) return 1;
    return 0;
}

int orc_pw_kvectors(int n, int *out /* n*4 */)
{
    if (n <= 0) return -1;
    /* A cube [-m, m]^3 holds every lattice vector with |n|^2 <= m^2. */
    for (int m = 2;; ++m) {
        int side = 2 * m + 1;
        orc_rep *reps = (orc_rep *)malloc(sizeof(orc_rep) * side * side * side);
        int cnt = 0;
        for (int x = -m; x <= m; ++x)
            for (int y = -m; y <= m; ++y)
                for (int z = -m; z <= m; ++z) {
                    int first = x != 0 ? x : (y != 0 ? y : z);
                    if (first <= 0) continue; /* skips n = 0 and the -n partner */
                    reps[cnt].nx = x; reps[cnt].ny = y; reps[cnt].nz = z;
                    reps[cnt].n2 = x * x + y * y + z * z;
                    ++cnt;
                }
        qsort(reps, cnt, sizeof(orc_rep), orc_rep_cmp);
        int need_reps = n / 2; /* orbitals 1..n-1 come in cos/sin pairs */
        if (need_reps <= cnt && (need_reps == 0 || reps[need_reps - 1].n2 <= m * m)) {
            out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0;
            int j = 1;
            for (int r = 0; r < need_reps && j < n; ++r) {
                for (int kind = 1; kind <= 2 && j < n; ++kind, ++j) {
                    out[4 * j + 0] = reps[r].nx;
                    out[4 * j + 1] = reps[r].ny;
                    out[4 * j + 2] = reps[r].nz;
                    out[4 * j + 3] = kind;
                }
            }
            free(reps);
            return 0;
        }
        free(reps);
    }
}

/* One Slater-matrix row: row[j] = phi_j(r).  Phase = (2 pi / L) * ((nx x + ny y) + nz z). */
void orc_pw_row(int n, const int *kv, double L, const double r[3], double *row)
{
    double twopi_l = 2.0 * ORC_PI / L;
    for (int j = 0; j < n; ++j) {
        int kind = kv[4 * j + 3];
        if (kind == 0) { row[j] = 1.0; continue; }
        double t = ((double)kv[4 * j + 0] * r[0] + (double)kv[4 * j + 1] * r[1]) + (double)kv[4 * j + 2] * r[2];
        double ph = twopi_l * t;
        row[j] = kind == 1 ? cos(ph) : sin(ph);
    }
}

/* Gradient rows of one Slater-matrix row with respect to the electron
 * position: drow[a*n + j] = d phi_j(r) / d r_a (a = x, y, z).  With
 * g = 2 pi / L and phase ph = g (n . r):  d cos(ph) = -g n_a sin(ph),
 * d sin(ph) = g n_a cos(ph), the constant orbital has zero gradient. */
void orc_pw_row_grad(int n, const int *kv, double L, const double r[3], double *drow)
{
    double twopi_l = 2.0 * ORC_PI / L;
    for (int j = 0; j < n; ++j) {
        int kind = kv[4 * j + 3];
        double t = ((double)kv[4 * j + 0] * r[0] + (double)kv[4 * j + 1] * r[1]) + (double)kv[4 * j + 2] * r[2];
        double ph = twopi_l * t;
        for (int a = 0; a < 3; ++a) {
            double ga = twopi_l * (double)kv[4 * j + a];
            double d = 0.0;
            if (kind == 1) d = -ga * sin(ph);
            else if (kind == 2) d = ga * cos(ph);
            drow[(size_t)a * n + j] = d;
        }
    }
}

/* Slater matrix A (n x n, row-major, row i = electron i). */
void orc_pw_matrix(int n, const int *kv, double L, const double *pos, double *a)
{
    for (int i = 0; i < n; ++i) orc_pw_row(n, kv, L, pos + 3 * i, a + (size_t)i * n);
}

/* ------------------------------------------------------------------------ */
/* LU factorisation with partial pivoting (Golub & Van Loan, Alg. 3.4.1):     */
/* the explicit O(N^3) route of Sec. I, used for fresh determinants after a   */
/* sweep (Sec. III) and for the initial inverse.  Pivot = largest |entry| in  */
/* the column, lowest row index on ties.                                      */
/* ------------------------------------------------------------------------ */
int orc_lu(int n, double *a /* in: A, out: L\U */, int *piv, double *logdet, int *sign)
{
    int s = 1;
    double ld = 0.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return -3; /* exactly singular */
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
            s = -s;
        }
        double d = a[(size_t)k * n + k];
        ld += log(fabs(d));
        if (d < 0) s = -s;
        for (int i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / d;
            a[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    if (logdet) *logdet = ld;
    if (sign) *sign = s;
    return 0;
}

/* log|det A| and sign(det A) of an n x n matrix (input untouched). */
int orc_slogdet(int n, const double *a, double *logdet, int *sign)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *piv = (int *)malloc(sizeof(int) * (size_t)n);
    memcpy(w, a, sizeof(double) * (size_t)n * n);
    int rc = orc_lu(n, w, piv, logdet, sign);
    free(w); free(piv);
    return rc;
}

/* A^{-1} by LU: solve A X = I one column at a time. */
int orc_inverse(int n, const double *a, double *ainv, double *logdet, int *sign)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *piv = (int *)malloc(sizeof(int) * (size_t)n);
    double *col = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(w, a, sizeof(double) * (size_t)n * n);
    int rc = orc_lu(n, w, piv, logdet, sign);
    if (rc == 0) {
        for (int c = 0; c < n; ++c) {
            for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < n; ++k) { /* same row swaps as the factorisation */
                double t = col[k]; col[k] = col[piv[k]]; col[piv[k]] = t;
            }
            for (int i = 0; i < n; ++i) /* L y = P e_c, unit lower */
                for (int k = 0; k < i; ++k) col[i] -= w[(size_t)i * n + k] * col[k];
            for (int i = n - 1; i >= 0; --i) { /* U x = y */
                for (int k = i + 1; k < n; ++k) col[i] -= w[(size_t)i * n + k] * col[k];
                col[i] /= w[(size_t)i * n + i];
            }
            for (int i = 0; i < n; ++i) ainv[(size_t)i * n + c] = col[i];
        }
    }
    free(w); free(piv); free(col);
    return rc;
}

/* max_ij |(Ainv A - I)_ij| */
double orc_residual(int n, const double *ainv, const double *a)
{
    double worst = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += ainv[(size_t)i * n + k] * a[(size_t)k * n + j];
            if (i == j) s -= 1.0;
            if (fabs(s) > worst) worst = fabs(s);
        }
    return worst;
}

/* Rows of the right residual A Ainv - I: the largest |sum_k a[r][k] ainv[k][j]
 * - [r == j]| over the listed rows r = rows[0..m) and every column j (the
 * check of an inverse against the matrix itself, Sec. III, restricted to a
 * sample of electrons).  Rows outside [0, n) are skipped. */
double orc_residual_rows(int n, const double *ainv, const double *a, int m, const int *rows)
{
    double worst = 0.0;
    for (int q = 0; q < m; ++q) {
        const int r = rows[q];
        if (r < 0 || r >= n) continue;
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += a[(size_t)r * n + k] * ainv[(size_t)k * n + j];
            if (r == j) s -= 1.0;
            if (fabs(s) > worst) worst = fabs(s);
        }
    }
    return worst;
}

/* Rows of the left residual Ainv A - I: the largest |sum_k ainv[r][k] a[k][j]
 * - [r == j]| over the listed rows r and every column j.  Rows outside
 * [0, n) are skipped. */
double orc_residual_left_rows(int n, const double *ainv, const double *a, int m, const int *rows)
{
    double worst = 0.0;
    for (int q = 0; q < m; ++q) {
        const int r = rows[q];
        if (r < 0 || r >= n) continue;
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += ainv[(size_t)r * n + k] * a[(size_t)k * n + j];
            if (r == j) s -= 1.0;
            if (fabs(s) > worst) worst = fabs(s);
        }
    }
    return worst;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): ratio det(A_new)/det(A) when row e of A becomes phi.             */
/* ------------------------------------------------------------------------ */
double orc_sm_ratio(int n, const double *ainv, int e, const double *phi)
{
    double r = 0.0;
    for (int j = 0; j < n; ++j) r += phi[j] * ainv[(size_t)j * n + e];
    return r;
}

/* Gradient of the eq. (1) ratio with respect to the new position of
 * electron e.  The determinant is linear in row e, so differentiating the
 * new row phi(r') and applying eq. (1) to each derivative row gives
 *   d R / d r'_a = (d phi / d r'_a) . Ainv[:,e],   a = x, y, z.
 * Called with the electron's present row and its gradient rows this is the
 * drift grad_e ln|det A| (R = 1 there).  Returns R, writes grad[3]. */
double orc_sm_ratio_grad(int n, const double *ainv, int e, const double *phi, const double *dphi, double *grad)
{
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += dphi[(size_t)a * n + j] * ainv[(size_t)j * n + e];
        grad[a] = s;
    }
    return orc_sm_ratio(n, ainv, e, phi);
}

/* Eq. (2): rank-1 Sherman-Morrison update of Ainv after row e -> phi with
 * ratio r.  With u = phi - A[e,:] (a row change) and v = e_e:
 *   Ainv_new = Ainv - Ainv[:,e] (u Ainv) / r,   u Ainv = phi Ainv - e_e^T.
 * Also writes the new row into A.  `work` holds 2n doubles. */
void orc_sm_accept(int n, double *ainv, double *a, int e, const double *phi, double r, double *work)
{
    double *w = work, *c = work + n;
    /* w[k] = sum_j phi[j] Ainv[j][k], accumulated row by row of Ainv so the
     * matrix is read in storage order; every w[k] still adds its terms in
     * ascending j from 0.0, exactly as a dot product over j would. */
    for (int k = 0; k < n; ++k) w[k] = 0.0;
    for (int j = 0; j < n; ++j) {
        const double pj = phi[j];
        const double *arow = ainv + (size_t)j * n;
        for (int k = 0; k < n; ++k) w[k] += pj * arow[k];
    }
    w[e] -= 1.0;
    for (int i = 0; i < n; ++i) c[i] = ainv[(size_t)i * n + e];
    for (int i = 0; i < n; ++i) {
        double f = c[i] / r;
        for (int k = 0; k < n; ++k) ainv[(size_t)i * n + k] -= f * w[k];
    }
    if (a) memcpy(a + (size_t)e * n, phi, sizeof(double) * n);
}

/* ------------------------------------------------------------------------ */
/* One walker determinant driven by the counter-based stream: the           */
/* Metropolis single-electron loop of Sec. I/II (move proposed, ratio by    */
/* eq. (1), accepted with probability min(1, R^2), inverse updated by eq.   */
/* (2) at once).  Electrons are visited 0..n-1 every sweep.                 */
/*                                                                          */
/* Inputs: n, L, seed, walker id, spin (counter slot = spin*n + e), sigma,  */
/* first sweep index, number of sweeps, force_accept, positions (n*3).      */
/* Outputs (any may be NULL): per move ratio[], u[], accepted[]; per sweep  */
/* running log|det| / sign (after the sweep), fresh LU log|det| / sign, and */
/* max |Ainv A - I|; final positions and final Ainv (row-major, natural).   */
/* Returns 0, or -3 if A is singular at the start.                          */
/* ------------------------------------------------------------------------ */
int orc_walker_run(int n, double L, uint64_t seed, uint64_t walker, int spin, double sigma,
                   int first_sweep, int sweeps, int force_accept, const double *pos_in,
                   double *ratio, double *uout, uint8_t *accepted,
                   double *logdet_run, int *sign_run, double *logdet_fresh, int *sign_fresh,
                   double *residual, double *pos_out, double *ainv_out, int64_t *n_accepted)
{
    int *kv = (int *)malloc(sizeof(int) * 4 * (size_t)n);
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *ainv = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    double *work = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    int rc = 0;
    int64_t nacc = 0;
    orc_pw_kvectors(n, kv);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    orc_pw_matrix(n, kv, L, pos, a);
    double ld = 0.0;
    int sg = 1;
    if (orc_inverse(n, a, ainv, &ld, &sg) != 0) { rc = -3; goto done; }
    for (int s = 0; s < sweeps; ++s) {
        int sweep = first_sweep + s;
        for (int e = 0; e < n; ++e) {
            double g[3], u;
            orc_move_randoms(seed, walker, (uint64_t)sweep, (uint64_t)spin * (uint64_t)n + (uint64_t)e, g, &u);
            double rt[3] = {pos[3 * e + 0] + sigma * g[0], pos[3 * e + 1] + sigma * g[1], pos[3 * e + 2] + sigma * g[2]};
            orc_pw_row(n, kv, L, rt, phi);
            double r = orc_sm_ratio(n, ainv, e, phi);
            int acc = force_accept ? 1 : (u < r * r);
            size_t m = (size_t)s * n + e;
            if (ratio) ratio[m] = r;
            if (uout) uout[m] = u;
            if (accepted) accepted[m] = (uint8_t)acc;
            if (acc) {
                orc_sm_accept(n, ainv, a, e, phi, r, work);
                pos[3 * e + 0] = rt[0]; pos[3 * e + 1] = rt[1]; pos[3 * e + 2] = rt[2];
                ld += log(fabs(r));
                if (r < 0) sg = -sg;
                ++nacc;
            }
        }
        if (logdet_run) logdet_run[s] = ld;
        if (sign_run) sign_run[s] = sg;
        if (logdet_fresh || sign_fresh) {
            double lf = 0.0; int sf = 0;
            orc_slogdet(n, a, &lf, &sf);
            if (logdet_fresh) logdet_fresh[s] = lf;
            if (sign_fresh) sign_fresh[s] = sf;
        }
        if (residual) residual[s] = orc_residual(n, ainv, a);
    }
    if (pos_out) memcpy(pos_out, pos, sizeof(double) * 3 * (size_t)n);
    if (ainv_out) memcpy(ainv_out, ainv, sizeof(double) * (size_t)n * n);
    if (n_accepted) *n_accepted = nacc;
done:
    free(kv); free(pos); free(a); free(ainv); free(phi); free(work);
    return rc;
}

/* Many independent walker determinants, one per OpenMP thread at a time.
 * Arrays are per-walker blocks: pos_in [w][n*3], seeds/walker ids [w],
 * spins [w]; per-move outputs [w][sweeps*n]; per-sweep outputs [w][sweeps];
 * pos_out [w][n*3].  No residual (it costs an extra N^3 per sweep).
 * Returns the number of threads used. */
int orc_walkers_run(int nw, int n, double L, const uint64_t *seeds, const uint64_t *walker_ids,
                    const int *spins, double sigma, int first_sweep, int sweeps, int force_accept,
                    const double *pos_in, double *ratio, uint8_t *accepted, double *logdet_run,
                    double *pos_out, int64_t *n_accepted, int *status)
{
    int threads = 1;
#ifdef _OPENMP
    threads = omp_get_max_threads();
    if (threads > nw) threads = nw;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
    for (int w = 0; w < nw; ++w) {
        size_t mv = (size_t)w * sweeps * n;
        status[w] = orc_walker_run(n, L, seeds[w], walker_ids[w], spins ? spins[w] : 0, sigma, first_sweep, sweeps,
                                   force_accept, pos_in + (size_t)w * 3 * n, ratio ? ratio + mv : NULL, NULL,
                                   accepted ? accepted + mv : NULL, logdet_run ? logdet_run + (size_t)w * sweeps : NULL,
                                   NULL, NULL, NULL, NULL, pos_out ? pos_out + (size_t)w * 3 * n : NULL, NULL,
                                   n_accepted ? n_accepted + w : NULL);
    }
    return threads;
}

/* ------------------------------------------------------------------------ */
/* A bounded sample of the same Metropolis loop: `nmoves` moves of sweep     */
/* `sweep` starting at electron `e_first`, from a supplied state (positions, */
/* A and Ainv, all updated in place).  Used to time the oracle on a slice of */
/* a large workload whose O(N^3) set-up would dominate a full run.           */
/* Returns the number of accepted moves.                                     */
/* ------------------------------------------------------------------------ */
int64_t orc_walker_moves(int n, double L, uint64_t seed, uint64_t walker, int spin, double sigma, int sweep,
                         int e_first, int nmoves, int force_accept, double *pos, double *a, double *ainv,
                         double *ratio_out)
{
    int *kv = (int *)malloc(sizeof(int) * 4 * (size_t)n);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    double *work = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    int64_t nacc = 0;
    orc_pw_kvectors(n, kv);
    for (int m = 0; m < nmoves; ++m) {
        int e = (e_first + m) % n;
        double g[3], u;
        orc_move_randoms(seed, walker, (uint64_t)sweep, (uint64_t)spin * (uint64_t)n + (uint64_t)e, g, &u);
        double rt[3] = {pos[3 * e + 0] + sigma * g[0], pos[3 * e + 1] + sigma * g[1], pos[3 * e + 2] + sigma * g[2]};
        orc_pw_row(n, kv, L, rt, phi);
        double r = orc_sm_ratio(n, ainv, e, phi);
        if (ratio_out) ratio_out[m] = r;
        if (force_accept || u < r * r) {
            orc_sm_accept(n, ainv, a, e, phi, r, work);
            pos[3 * e + 0] = rt[0]; pos[3 * e + 1] = rt[1]; pos[3 * e + 2] = rt[2];
            ++nacc;
        }
    }
    free(kv); free(phi); free(work);
    return nacc;
}

/* orc_walker_moves for nw walkers at once, one OpenMP thread each; arrays are
 * per-walker blocks (ratios, if not NULL: nmoves per walker).  Returns the
 * number of threads used. */
int orc_walkers_moves(int nw, int n, double L, const uint64_t *seeds, const uint64_t *walker_ids, double sigma,
                      int sweep, int e_first, int nmoves, int force_accept, double *pos, double *a, double *ainv,
                      int64_t *n_accepted, double *ratios)
{
    int threads = 1;
#ifdef _OPENMP
    threads = omp_get_max_threads();
    if (threads > nw) threads = nw;
#pragma omp parallel for schedule(static, 1) num_threads(threads)
#endif
    for (int w = 0; w < nw; ++w)
        n_accepted[w] = orc_walker_moves(n, L, seeds[w], walker_ids[w], 0, sigma, sweep, e_first, nmoves, force_accept,
                                         pos + (size_t)w * 3 * n, a + (size_t)w * n * n, ainv + (size_t)w * n * n,
                                         ratios ? ratios + (size_t)w * nmoves : NULL);
    return threads;
}

/* ======================================================================== */
/* Complex orbitals (twisted boundary conditions).  The same definitions in */
/* complex arithmetic: no conjugation anywhere, transposes are plain.       */
/* Complex arrays are interleaved (re, im), i.e. C99 double complex.        */
/* ======================================================================== */
#include <complex.h>

typedef struct { int nx, ny, nz; double k2; } orc_zrep;

static int orc_zrep_cmp(const void *pa, const void *pb)
{
    const orc_zrep *a = (const orc_zrep *)pa, *b = (const orc_zrep *)pb;
    if (a->k2 != b->k2) return a->k2 < b->k2 ? -1 : 1;
    if (a->nx != b->nx) return a->nx < b->nx ? -1 : 1;
    if (a->ny != b->ny) return a->ny < b->ny ? -1 : 1;
    return a->nz < b->nz ? -1 : (a->nz > b->nz);
}

/* Twisted plane waves phi_j(r) = exp(i (2 pi / L) (n_j + theta) . r): the n
 * integer vectors n_j with the smallest |n + theta|^2, ties in lexicographic
 * order of (nx, ny, nz).  A cube [-m, m]^3 holds every candidate once the n-th
 * value is below (m - 1/2)^2 (a vector outside has some |n_a + theta_a| >= m - 1/2
 * for |theta_a| <= 1/2).  out: n x 3. */
int orc_zpw_kvectors(int n, const double theta[3], int *out)
{
    if (n <= 0) return -1;
    for (int m = 2;; ++m) {
        int side = 2 * m + 1;
        orc_zrep *reps = (orc_zrep *)malloc(sizeof(orc_zrep) * side * side * side);
        int cnt = 0;
        for (int x = -m; x <= m; ++x)
            for (int y = -m; y <= m; ++y)
                for (int z = -m; z <= m; ++z) {
                    double a = x + theta[0], b = y + theta[1], c = z + theta[2];
                    reps[cnt].nx = x; reps[cnt].ny = y; reps[cnt].nz = z;
                    reps[cnt].k2 = a * a + b * b + c * c;
                    ++cnt;
                }
        qsort(reps, cnt, sizeof(orc_zrep), orc_zrep_cmp);
        if (n <= cnt && reps[n - 1].k2 < (m - 0.5) * (m - 0.5)) {
            for (int j = 0; j < n; ++j) { out[3 * j] = reps[j].nx; out[3 * j + 1] = reps[j].ny; out[3 * j + 2] = reps[j].nz; }
            free(reps);
            return 0;
        }
        free(reps);
    }
}

void orc_zpw_row(int n, const int *kv, const double theta[3], double L, const double r[3], double complex *row)
{
    double g = 2.0 * ORC_PI / L;
    for (int j = 0; j < n; ++j) {
        double ph = g * (((kv[3 * j] + theta[0]) * r[0] + (kv[3 * j + 1] + theta[1]) * r[1]) + (kv[3 * j + 2] + theta[2]) * r[2]);
        row[j] = cos(ph) + I * sin(ph);
    }
}

/* LU with partial pivoting by modulus (lowest row on ties), as orc_lu.
 * logabs = log|det|, phase = arg(det) in (-pi, pi]. */
int orc_zlu(int n, double complex *a, int *piv, double *logabs, double *phase)
{
    double la = 0.0, ph = 0.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = cabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return -3;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double complex t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
            ph += ORC_PI;
        }
        double complex d = a[(size_t)k * n + k];
        la += log(cabs(d));
        ph += carg(d);
        for (int i = k + 1; i < n; ++i) {
            double complex l = a[(size_t)i * n + k] / d;
            a[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    ph = fmod(ph, 2.0 * ORC_PI);
    if (ph > ORC_PI) ph -= 2.0 * ORC_PI;
    if (ph <= -ORC_PI) ph += 2.0 * ORC_PI;
    if (logabs) *logabs = la;
    if (phase) *phase = ph;
    return 0;
}

int orc_zinverse(int n, const double complex *a, double complex *ainv, double *logabs, double *phase)
{
    double complex *w = (double complex *)malloc(sizeof(double complex) * (size_t)n * n);
    double complex *col = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    int *piv = (int *)malloc(sizeof(int) * (size_t)n);
    memcpy(w, a, sizeof(double complex) * (size_t)n * n);
    int rc = orc_zlu(n, w, piv, logabs, phase);
    if (rc == 0 && ainv) {
        for (int c = 0; c < n; ++c) {
            for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < n; ++k) { double complex t = col[k]; col[k] = col[piv[k]]; col[piv[k]] = t; }
            for (int i = 0; i < n; ++i)
                for (int k = 0; k < i; ++k) col[i] -= w[(size_t)i * n + k] * col[k];
            for (int i = n - 1; i >= 0; --i) {
                for (int k = i + 1; k < n; ++k) col[i] -= w[(size_t)i * n + k] * col[k];
                col[i] /= w[(size_t)i * n + i];
            }
            for (int i = 0; i < n; ++i) ainv[(size_t)i * n + c] = col[i];
        }
    }
    free(w); free(col); free(piv);
    return rc;
}

/* Eq. (1) in complex arithmetic: R = phi . Ainv[:, e]. */
double complex orc_zsm_ratio(int n, const double complex *ainv, int e, const double complex *phi)
{
    double complex r = 0.0;
    for (int j = 0; j < n; ++j) r += phi[j] * ainv[(size_t)j * n + e];
    return r;
}

/* Eq. (2) in complex arithmetic (as orc_sm_accept); work holds 2n values. */
void orc_zsm_accept(int n, double complex *ainv, double complex *a, int e, const double complex *phi, double complex r,
                    double complex *work)
{
    double complex *w = work, *c = work + n;
    for (int k = 0; k < n; ++k) {
        double complex s = 0.0;
        for (int j = 0; j < n; ++j) s += phi[j] * ainv[(size_t)j * n + k];
        w[k] = s;
    }
    w[e] -= 1.0;
    for (int i = 0; i < n; ++i) c[i] = ainv[(size_t)i * n + e];
    for (int i = 0; i < n; ++i) {
        double complex f = c[i] / r;
        for (int k = 0; k < n; ++k) ainv[(size_t)i * n + k] -= f * w[k];
    }
    if (a) memcpy(a + (size_t)e * n, phi, sizeof(double complex) * (size_t)n);
}

/* ctypes cannot return a C complex: ratio through an out-parameter. */
void orc_zsm_ratio_out(int n, const double complex *ainv, int e, const double complex *phi, double complex *out)
{
    *out = orc_zsm_ratio(n, ainv, e, phi);
}

void orc_zsm_accept_r(int n, double complex *ainv, double complex *a, int e, const double complex *phi,
                      const double complex *r, double complex *work)
{
    orc_zsm_accept(n, ainv, a, e, phi, *r, work);
}

/* ======================================================================== */
/* Multideterminant wave functions on a single reference.  Psi = sum_I c_I  */
/* det(A_I), where A_I is the reference Slater matrix A (row i = electron   */
/* i, column j = occupied orbital j) with the columns occ[I][a] replaced by */
/* the virtual-orbital columns V[:, virt[I][a]], a < order[I] (order 0 is   */
/* the reference itself).  Evaluated by definition: one LU per term.        */
/* Returns log|Psi| and sign(Psi) (0 if Psi = 0).                           */
/* ======================================================================== */
int orc_md_psi(int n, int m, const double *a, const double *v, int ndet, const int *order, const int *occ,
               const int *virt, const double *coef, double *logabs, int *sign)
{
    for (int d = 0; d < ndet; ++d) {
        if (order[d] < 0 || order[d] > 4) return -1;
        for (int q = 0; q < order[d]; ++q)
            if (occ[4 * d + q] < 0 || occ[4 * d + q] >= n || virt[4 * d + q] < 0 || virt[4 * d + q] >= m) return -1;
    }
    double *w = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *piv = (int *)malloc(sizeof(int) * (size_t)n);
    double *ld = (double *)malloc(sizeof(double) * (size_t)ndet);
    int *sg = (int *)malloc(sizeof(int) * (size_t)ndet);
    double lmax = -INFINITY;
    for (int d = 0; d < ndet; ++d) {
        memcpy(w, a, sizeof(double) * (size_t)n * n);
        for (int q = 0; q < order[d]; ++q) {
            int j = occ[4 * d + q], vv = virt[4 * d + q];
            for (int i = 0; i < n; ++i) w[(size_t)i * n + j] = v[(size_t)i * m + vv];
        }
        if (orc_lu(n, w, piv, &ld[d], &sg[d]) != 0) { sg[d] = 0; ld[d] = -INFINITY; }
        if (sg[d] != 0 && coef[d] != 0.0 && ld[d] > lmax) lmax = ld[d];
    }
    double s = 0.0;
    for (int d = 0; d < ndet; ++d)
        if (sg[d] != 0) s += coef[d] * sg[d] * exp(ld[d] - lmax);
    free(w); free(piv); free(ld); free(sg);
    if (s == 0.0 || !isfinite(lmax)) { *logabs = -INFINITY; *sign = 0; return 0; }
    *logabs = lmax + log(fabs(s));
    *sign = s > 0 ? 1 : -1;
    return 0;
}
