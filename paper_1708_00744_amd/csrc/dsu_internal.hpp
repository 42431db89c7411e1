// dsu_internal.hpp -- shared declarations of libdsu's HIP kernels and host code.
//
// Layout conventions (all device buffers of one determinant):
//   np  = n rounded up to a multiple of 64; every n x n array is stored np x np,
//         row-major, zero padded (the padded rows/columns of BT stay zero through
//         every update, see the flush kernel).
//   kp  = delay K rounded up to a multiple of 16 (one MFMA tile).
//   BT  = (A^{-1})^T, np x np, precision T (double or float).
//   U   = the window's proposed orbital rows, kp x np, T.
//   Vg  = stale BT rows of the window's electrons, kp x np, T.
//   Cfl = zero-embedded inverse of the window's C matrix (eq. (3)), kp x kp, FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsu {

constexpr int kRowBlock = 64;    // rows of BT per flush workgroup
constexpr int kThreads = 256;    // 4 wave64 per workgroup

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ----------------------------------------------------------------- MFMA
// Result row of accumulator element i in lane `lane` of a 16x16 tile:
//     Mma<T>::row0(lane) + i * Mma<T>::row_step,   column lane % 16.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
    typedef f32x4 acc_t;
    // v_mfma_f32_16x16x4_f32: D(16x16) += A(16x4) B(4x16); lane l supplies
    // A[l%16][l/16] and B[l/16][l%16]; D[4*(l/16)+i][l%16] lands in acc[i].
    static __device__ __forceinline__ int row0(int lane) { return 4 * (lane >> 4); }
    static constexpr int row_step = 1;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mma<double> {
    typedef f64x4 acc_t;
    // v_mfma_f64_16x16x4_f64: same A and B layout as above, but the result
    // rows interleave: D[(l/16) + 4*i][l%16] lands in acc[i].
    static __device__ __forceinline__ int row0(int lane) { return lane >> 4; }
    static constexpr int row_step = 4;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Position of C^{-1}[l][j] (window tile KP) in the FP32 copy the streaming
// flush reads as the B operand of W = Y' C^{-T} on 16x16x4 matrix cores: tile
// t = l / 16, step s = j / 4; lane (l % 16) + 16 (j % 4) reads steps 4q..4q+3
// of tile t as one 16-byte vector.
template <int KP> __host__ __device__ __forceinline__ int cfl32_index(int l, int j) {
    const int t = l >> 4, s = j >> 2, lane = (l & 15) + 16 * (j & 3);
    return ((t * (KP / 16) + (s >> 2)) * 64 + lane) * 4 + (s & 3);
}

// --------------------------------------------------- descriptors (device)
// One rank-k update target: BT <- BT - ((BT U^T - E) C^T) Vg   (eq. (4),
// transposed and row-local).  idx[j] = electron of slot j (-1 = unused).
template <typename T> struct FlushDesc {
    T *bt;
    const T *u;
    const T *vg;
    const double *cinv;
    const int *idx;
    int ldc;
};

// Per-determinant running state of the batched form (device memory).
struct DetState {
    double logdet;
    int sign;
    int bad;              // count of zero / non-finite ratios met
    long long accepted;
    long long sweep;      // completed sweeps (RNG counter word 0)
    long long trace_pos;  // next trace slot
};

// One determinant of the batched form.
template <typename T> struct DetDesc {
    T *bt;           // np x np
    T *u;            // kp x np
    T *vg;           // kp x np
    double *cfl;     // kp x kp
    float *cfl32;    // FP32 batched form, window tiles of 32..128: C^{-1} in FP32, laid out as the
                     // W product's B operand (cfl32_index), written by the decisions
    double *cwork;   // kp x (kp+1) when the bordered inverse does not fit LDS
    double *gwork;   // kp x (kp+1) when G does not fit LDS
    double *prop;    // kp x 4 : proposed position (x, y, z) and Metropolis uniform
    double *pos;     // n x 3
    int *idx;        // kp
    DetState *st;
    double *trace_r; // optional per-move ratio record
    uint8_t *trace_a;
    long long trace_cap;
    uint64_t seed, wid;
    double sigma;
    int spin;
    // streaming path: second U/Vg buffers (windows alternate) and the
    // look-ahead products of the next window for every row, y[i][a] = BT[i].U[a]
    T *u2;           // kp x np
    T *vg2;          // kp x np
    T *y;            // np x kp
    double *prop2;   // kp x 4: proposals of the odd windows (the next window's are drawn
                     // while the current window is decided)
};

// ------------------------------------------------------- launchers (host)
// All launchers return hipSuccess or the launch error.

// Flush (eq. (4)) of `ndesc` determinants with `kslots` delayed slots
// (<= kp of the descriptors' buffers); mode 0 = MFMA fused, 1 = VALU.
// ld: row length of BT, U and Vg (0 = np; MFMA mode only otherwise).
template <typename T>
hipError_t launch_flush(const FlushDesc<T> *descs_dev, int ndesc, int n, int np, int kslots, int mode,
                        hipStream_t s, int ld = 0);

// C[0:nrows, 0:ncols] -= W[:, 0:kslots] V[0:kslots, :] (FP64, matrix cores;
// V rows kslots .. padded width zero; nrows and ncols multiples of 64).
hipError_t launch_gemm_sub(const double *W, int ldw, int kslots, const double *V, int ldv, double *C, int ldc,
                           int nrows, int ncols, hipStream_t s);

// FP64 inversion by blocked Gauss-Jordan with partial pivoting.
struct GjDesc {
    double *m;        // np x np work (in: A^T padded with identity; out: inverse scrambled)
    double *m2;       // np x np: the other buffer of the ping-pong trailing update
    double *panel;    // np x nb: the panel's columns, column-major (factored in place)
    double *w;        // np x nb: a column group's update (E - S), column-major
    int *piv;         // n pivots
    int *perm;        // np final column permutation
    int *rowsrc;      // np: the panel's row interchanges, composed (row i <- row rowsrc[i])
    double *logdet;   // out
    int *sign;        // out
    int *status;      // out: 0 or -3 singular
    double *pmax;     // largest pivot magnitude so far (singularity threshold)
    // fused panel pairs (two 64-column panels, one rank-128 trailing update)
    double *panel_b;  // np x 64: the pair's first factored panel, column-major
    double *q2;       // 64 x np: the second panel's pivot rows after the first panel's update
    int *rowsrc_b;    // np: the second panel's own row interchanges, composed
    int *qrow;        // 64: rows of M that hold the first panel's pivot rows
};

// A ratio whose magnitude is at or below this cannot be accepted: the
// updated matrix would be numerically singular (and Metropolis would accept
// it with probability R^2 <= 1e-24 resp. 1e-12).
template <typename T> struct RatioFloor;
template <> struct RatioFloor<double> { static constexpr double value = 1e-12; };
template <> struct RatioFloor<float> { static constexpr double value = 1e-6; };
// Blocking of the Gauss-Jordan inversion: panel width nb (16, 32, 64, or 128
// = 64-column panels factored in pairs that share one rank-128 trailing
// update), the single-panel update's column chunk cw (32, or 64 when np is a
// multiple of 128) and the panel columns one apply workgroup takes, cpb (1 or 4).
struct GjTiles {
    int nb = 64, cw = 32, cpb = 1;
};
GjTiles gj_tiles_default(int n, int np);
// Two descriptor sets of the same matrices with m and m2 exchanged: panel p
// reads set (p mod 2)'s m and writes its m2.  *final_set receives the set
// whose m holds the result (for launch_cast_perm).  The panel buffers hold
// 64 columns (a pair uses panel and panel_b).
hipError_t launch_gj_invert(const GjDesc *set_a, const GjDesc *set_b, int ndesc, int n, int np, const GjTiles &tiles,
                            hipStream_t s, const GjDesc **final_set);
// BT[i][j] = T(M[i][perm[j]]) for i, j < n, zero padding elsewhere.
template <typename T>
hipError_t launch_cast_perm(const GjDesc *gj_dev, T *const *bt_dev, int ndesc, int n, int np, hipStream_t s);
// M = A^T (A row-major n x n, padded with identity to np).
hipError_t launch_load_transpose(const double *const *a_dev, double *const *m_dev, int ndesc, int n, int np,
                                 int lda, hipStream_t s);
// M = A^T with A built from plane waves at the positions.
hipError_t launch_build_pw_transpose(const double *const *pos_dev, double *const *m_dev, int ndesc, int n,
                                     int np, const int4 *kvec, double twopi_over_l, hipStream_t s);
// out[i][j] = BT[j][i] (natural A^{-1}, FP64, n x n).
template <typename T>
hipError_t launch_untranspose(const T *bt, double *out, int n, int np, hipStream_t s);

// Largest delay a kernel stages per-slot values for in LDS.
#define DSU_KMAX_LDS 256

// Batched window kernels.  ktile = padded delay of the launch (template tile
// count, 16..256), kp = padded delay the buffers were allocated for (stride),
// nmax = largest |component| of the plane-wave integer vectors.
// Decisions of one window: the look-ahead products G come from y (formed by
// the previous pass over BT), proposals from prop (pbuf 0) or prop2 (1).
template <typename T>
hipError_t launch_window_decide(const DetDesc<T> *d, int ndesc, int ktile, int kp, int e0, int kw, int force_accept,
                                int last_window, int pbuf, hipStream_t s);

// Streaming path (one pass over BT per window):
//   props : proposals and orbital rows of a window into U buffer `buf`
//           (and, with copy_vg, the window's current BT rows into Vg `buf`)
//   prime : y = BT U[buf]^T for every row (start of a sweep)
//   flush : BT -= W Vg[cur] with W = (y - E) C^{-T}; while each chunk of BT is
//           on chip, y = BT_new U[nxt]^T for the next window and the next
//           window's BT rows into Vg[nxt]
template <typename T>
hipError_t launch_window_props(const DetDesc<T> *d, int ndesc, int n, int np, int ktile, int e0, int kw,
                               const int4 *kvec, double twopi_over_l, int buf, int copy_vg, int nmax, hipStream_t s);
template <typename T>
hipError_t launch_window_prime(const DetDesc<T> *d, int ndesc, int np, int ktile, int kp, int buf, hipStream_t s);
template <typename T>
hipError_t launch_flush_stream(const DetDesc<T> *d, int ndesc, int np, int ktile, int kp, int kslots, int cur,
                               int has_next, int e0n, int kwn, hipStream_t s);
template <typename T>
hipError_t launch_reset_state(const DetDesc<T> *d, const GjDesc *gj, double *drift, int ndesc, hipStream_t s);

// Sampled residual of the inverse: out_bits[d] = bit pattern of
// max_{s, j} |phi(r_{e_s}) . BT[j, :] - delta(j, e_s)| over `samples` (1..64,
// <= n) electrons e_s = s * (n / samples) + (sweep mod (n / samples)).
// Scratch: rows (ndesc x 64 x np FP64), eidx (ndesc x 64).
template <typename T>
hipError_t launch_resid(const DetDesc<T> *d, int ndesc, int n, int np, int samples, const int4 *kvec,
                        double twopi_over_l, double *rows, int *eidx, unsigned long long *out_bits, hipStream_t s);

// Left residual: out_bits[d] = bit pattern of max_{i, j} |(A^{-1} A - I)[i0 + i][j]|
// over i < samples (1..64, <= n), i0 = (sweep mod (n / samples)) * samples,
// with A rebuilt from the positions (no scratch); nmax = largest |component|
// of the plane-wave integer vectors.
template <typename T>
hipError_t launch_resid_left(const DetDesc<T> *d, int ndesc, int n, int np, int samples, const int4 *kvec,
                             double twopi_over_l, int nmax, unsigned long long *out_bits, hipStream_t s);

// rows[c][j] = phi_j(pos_c): plane-wave orbital rows at `count` positions.
hipError_t launch_pw_rows(const double *pos_dev, double *rows_dev, int n, int count, const int4 *kvec,
                          double twopi_over_l, hipStream_t s);

// Host-side plane-wave table: orbitals by shells of |n|^2 (see kvec.cpp).
int build_kvectors(int n, int4 *out /* n entries: nx, ny, nz, kind */);

}  // namespace dsu
