// k_linalg.hip -- matrix kernels of libdsu for gfx950.
//
//  * k_flush_mfma: the en-bloc update of the inverse, Sherman-Morrison-Woodbury,
//    eq. (4) of arXiv:1708.00744, written for the transposed inverse BT:
//        Y  = BT U^T            (np x k)   U   = accepted new orbital rows
//        Y' = Y - E             E[idx_j][j] = 1
//        W  = Y' C^{-T}         C^{-1}     = inverse of I_k + V'A^{-1}U (eq. (3))
//        BT = BT - W Vg         Vg         = stale BT rows of the moved electrons
//    Row i of the new BT needs only row i of the old one, so each workgroup
//    owns 64 rows and does the three products back to back on matrix cores
//    (v_mfma_*_16x16x4), reading its rows of BT twice and writing them once.
//  * k_flush_valu: the same update with vector ALUs, one wave per row (small k).
//  * k_gj_update: the trailing update of the Gauss-Jordan inversion,
//    M' = (row-interchanged M) - W Q, on matrix cores.
//  * Gauss-Jordan inversion with partial pivoting in FP64, blocked by panels of
//    nb columns: the O(N^3) explicit route the paper uses for direct checks.
#include "dsu_internal.hpp"
#include "tiles.hpp"

namespace dsu {

template <typename T, int KP> struct FlushLds {
    static constexpr int LDY = KP + 16 / (int)sizeof(T);
    static constexpr int p1 = KP * (128 / (int)sizeof(T) + 16 / (int)sizeof(T));
    static constexpr int p2 = 64 * LDY + WCfg<T, KP>::elems;  // Y' block + staged C chunk
    static constexpr int p3 = KP * Phase3Cfg<T, KP>::LDV;
    static constexpr int m12 = p1 > p2 ? p1 : p2;
    static constexpr int elems = m12 > p3 ? m12 : p3;
};

// ---------------------------------------------------------------------------
// Fused Woodbury flush, one 64-row block of one determinant per workgroup.
// ---------------------------------------------------------------------------
// Rows of BT, U and Vg are `ld` elements long (ld = np for a real inverse;
// the complex walker passes its interleaved complex inverse as real rows of
// 2 np, with U, Vg and C^{-1} in their real embedding).
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_flush_mfma(const FlushDesc<T> *__restrict__ descs, int ld,
                                                         int nblk, int kslots) {
    __shared__ __attribute__((aligned(16))) T lds[FlushLds<T, KP>::elems];
    constexpr int LDY = FlushLds<T, KP>::LDY;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * kRowBlock;
    const FlushDesc<T> fd = descs[d];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    typename Mma<T>::acc_t acc[KP / 16];
    rowblock_times_ut<T, KP>(fd.bt + (size_t)r0 * ld, ld, kRowBlock, fd.u, ld, 0, ld, lds, acc);

    // Y block -> LDS, subtract E, then W = Y' C^{-T} on matrix cores.
#pragma unroll
    for (int t = 0; t < KP / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) lds[(16 * wave + Mma<T>::row0(lane) + i * Mma<T>::row_step) * LDY + 16 * t + (lane & 15)] = acc[t][i];
    __syncthreads();
    for (int j = tid; j < kslots; j += kThreads) {
        const int e = fd.idx[j];
        if (e >= r0 && e < r0 + kRowBlock) lds[(e - r0) * LDY + j] -= T(1);
    }
    __syncthreads();
    typename Mma<T>::acc_t wacc[KP / 16];
    w_from_y<T, KP>(lds, LDY, fd.cinv, fd.ldc, kslots, lds + 64 * LDY, wacc);
#pragma unroll
    for (int t = 0; t < KP / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) lds[(16 * wave + Mma<T>::row0(lane) + i * Mma<T>::row_step) * LDY + 16 * t + (lane & 15)] = wacc[t][i];
    __syncthreads();
    T wa[KP / 4];
#pragma unroll
    for (int s = 0; s < KP / 4; ++s) wa[s] = -lds[(16 * wave + (lane & 15)) * LDY + 4 * s + (lane >> 4)];
    __syncthreads();
    rowblock_plus_wv<T, KP>(fd.bt + (size_t)r0 * ld, ld, ld, fd.vg, ld, wa, lds);
}

// ---------------------------------------------------------------------------
// C[0:nrows, 0:ncols] -= W[:, 0:kslots] V[0:kslots, :] in FP64 on matrix cores,
// tiled over rows and columns (64 x 64 per workgroup) so that one matrix
// fills the GPU.  W fragments beyond kslots are taken as zero; V rows beyond
// kslots (up to KP) must be zero.  nrows and ncols multiples of 64.
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(kThreads) void k_gemm_sub(const double *__restrict__ W, int ldw, int kslots,
                                                       const double *__restrict__ V, int ldv, double *C, int ldc,
                                                       int ncb) {
    __shared__ __attribute__((aligned(16))) double lds[KP * Phase3Cfg<double, KP>::LDV];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int r0 = (b / ncb) * kRowBlock, c0 = (b % ncb) * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double wa[KP / 4];
    const double *wr = W + (size_t)(r0 + 16 * wave + (lane & 15)) * ldw + (lane >> 4);
#pragma unroll
    for (int s = 0; s < KP / 4; ++s) wa[s] = 4 * s + (lane >> 4) < kslots ? -wr[4 * s] : 0.0;
    rowblock_plus_wv<double, KP>(C + (size_t)r0 * ldc + c0, ldc, 64, V + c0, ldv, wa, lds);
}

hipError_t launch_gemm_sub(const double *W, int ldw, int kslots, const double *V, int ldv, double *C, int ldc,
                           int nrows, int ncols, hipStream_t s) {
    if (nrows % kRowBlock || ncols % 64 || kslots < 1) return hipErrorInvalidValue;
    const int ncb = ncols / 64;
    const dim3 grid((nrows / kRowBlock) * ncb);
#define DSU_GS(KPV)                                                                                              \
    if (kslots <= KPV) {                                                                                         \
        hipLaunchKernelGGL((k_gemm_sub<KPV>), grid, dim3(kThreads), 0, s, W, ldw, kslots, V, ldv, C, ldc, ncb);  \
        return hipGetLastError();                                                                                \
    }
    DSU_GS(16) DSU_GS(32) DSU_GS(64) DSU_GS(128) DSU_GS(256)
#undef DSU_GS
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// VALU flush: one wave per row of BT, k <= KMAX slots in registers.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, int KMAX>
__global__ __launch_bounds__(kThreads) void k_flush_valu(const FlushDesc<T> *__restrict__ descs, int np, int kslots) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rows_per_det = np;
    const int g = blockIdx.x * 4 + wave;
    const int d = g / rows_per_det, row = g % rows_per_det;
    const FlushDesc<T> fd = descs[d];
    T *bt = fd.bt + (size_t)row * np;
    T y[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) y[j] = T(0);
    for (int c = lane; c < np; c += 64) {
        const T x = bt[c];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < kslots) y[j] += x * fd.u[(size_t)j * np + c];
    }
    T w[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        y[j] = wave_sum(y[j]);
        if (j < kslots && fd.idx[j] == row) y[j] -= T(1);
    }
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (l < kslots && j < kslots) s += T(fd.cinv[(size_t)l * fd.ldc + j]) * y[j];
        w[l] = s;
    }
    for (int c = lane; c < np; c += 64) {
        T x = bt[c];
#pragma unroll
        for (int l = 0; l < KMAX; ++l)
            if (l < kslots) x -= w[l] * fd.vg[(size_t)l * np + c];
        bt[c] = x;
    }
}

template <typename T>
hipError_t launch_flush(const FlushDesc<T> *descs_dev, int ndesc, int n, int np, int kslots, int mode,
                        hipStream_t s, int ld) {
    (void)n;
    if (ld == 0) ld = np;
    if (mode == 1 && ld != np) return hipErrorInvalidValue;
    if (ndesc <= 0 || kslots <= 0) return hipSuccess;
    if (mode == 1) {
        const int blocks = ndesc * np / 4;
#define DSU_VALU(KM)                                                                             \
    if (kslots <= KM) {                                                                          \
        hipLaunchKernelGGL((k_flush_valu<T, KM>), dim3(blocks), dim3(kThreads), 0, s, descs_dev, np, kslots); \
        return hipGetLastError();                                                                \
    }
        DSU_VALU(1) DSU_VALU(2) DSU_VALU(4) DSU_VALU(8) DSU_VALU(16) DSU_VALU(32) DSU_VALU(64)
#undef DSU_VALU
        return hipErrorInvalidValue;
    }
    const int nblk = np / kRowBlock;
    const dim3 grid(ndesc * nblk);
#define DSU_MFMA(KPV)                                                                            \
    if (kslots <= KPV) {                                                                         \
        hipLaunchKernelGGL((k_flush_mfma<T, KPV>), grid, dim3(kThreads), 0, s, descs_dev, ld, nblk, kslots); \
        return hipGetLastError();                                                                \
    }
    DSU_MFMA(16) DSU_MFMA(32) DSU_MFMA(64) DSU_MFMA(128) DSU_MFMA(256)
#undef DSU_MFMA
    return hipErrorInvalidValue;
}
template hipError_t launch_flush<float>(const FlushDesc<float> *, int, int, int, int, int, hipStream_t, int);
template hipError_t launch_flush<double>(const FlushDesc<double> *, int, int, int, int, int, hipStream_t, int);

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion (FP64, in place, partial pivoting).
// For a panel of columns R = [k0, k1): factor the panel with the unblocked
// in-place Gauss-Jordan step (pivot = largest |entry| among rows >= k, lowest
// index on ties), recording the row swaps.  The panel then holds the columns
// R of the accumulated elimination matrix T.  The other columns follow from
// the swapped pivot rows Q = M[R, :] as  M <- M - (E_R - T) Q.
// After the last panel, column swaps in reverse pivot order unscramble the
// inverse.  logdet = sum ln|pivot|, sign = swap parity * prod sign(pivot).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void argmax_combine(double &v, int &i, double v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// One workgroup per determinant.  The panel P is column-major (P[j*np + i]).
__global__ __launch_bounds__(kThreads) void k_gj_panel(const GjDesc *__restrict__ descs, int n, int np, int nb, int k0,
                                                       int k1) {
    __shared__ double s_v[kThreads / 64];
    __shared__ int s_i[kThreads / 64];
    __shared__ double s_row[64];
    __shared__ int s_p;
    const GjDesc g = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int w = k1 - k0;
    double *P = g.panel;
    for (int v = tid; v < np * w; v += kThreads) {
        const int j = v / np, i = v % np;
        P[(size_t)j * np + i] = g.m[(size_t)i * np + k0 + j];
    }
    if (k0 == 0 && tid == 0) { *g.logdet = 0.0; *g.sign = 1; *g.status = 0; *g.pmax = 0.0; }
    __syncthreads();
    for (int kk = 0; kk < w; ++kk) {
        const int k = k0 + kk;
        const double *pc = P + (size_t)kk * np;
        double best = -1.0;
        int bi = n;
        for (int i = k + tid; i < n; i += kThreads) argmax_combine(best, bi, fabs(pc[i]), i);
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(best, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            argmax_combine(best, bi, v2, i2);
        }
        if (lane == 0) { s_v[wave] = best; s_i[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            double bv = s_v[0];
            int bidx = s_i[0];
            for (int q = 1; q < kThreads / 64; ++q) argmax_combine(bv, bidx, s_v[q], s_i[q]);
            // singular when the best pivot is at rounding level of the largest one
            const double pm = fmax(*g.pmax, bv);
            *g.pmax = pm;
            if (!(bv > (double)n * 2.220446049250313e-16 * pm)) { *g.status = -3; bidx = k; }
            s_p = bidx;
            g.piv[k] = bidx;
        }
        __syncthreads();
        const int p = s_p;
        if (p != k && tid < w) {
            double *col = P + (size_t)tid * np;
            const double t = col[k];
            col[k] = col[p];
            col[p] = t;
        }
        __syncthreads();
        const double d = P[(size_t)kk * np + k];
        if (tid == 0) {
            if (d != 0.0) *g.logdet += log(fabs(d));
            int sg = *g.sign;
            if (p != k) sg = -sg;
            if (d < 0.0) sg = -sg;
            *g.sign = sg;
        }
        const double dinv = d != 0.0 ? 1.0 / d : 0.0;
        if (tid < w) s_row[tid] = tid == kk ? dinv : P[(size_t)tid * np + k] * dinv;
        __syncthreads();
        // each thread owns whole rows: read the multiplier first, then update
        for (int i = tid; i < np; i += kThreads) {
            if (i == k) {
                for (int j = 0; j < w; ++j) P[(size_t)j * np + i] = s_row[j];
                continue;
            }
            const double f = P[(size_t)kk * np + i];
            for (int j = 0; j < w; ++j) {
                if (j == kk) P[(size_t)j * np + i] = -f * dinv;
                else P[(size_t)j * np + i] -= f * s_row[j];
            }
        }
        __syncthreads();
    }
}

// The panel's row interchanges, composed: rowsrc[i] = the row of M whose
// contents row i holds after the swaps k <-> piv[k], k = k0 .. k1-1, in order
// (one workgroup per determinant; rows outside the panel's reach stay i).
// The map is built in LDS (np ints, dynamic shared memory) when it fits,
// else in place in global memory.
__global__ __launch_bounds__(kThreads) void k_gj_rowsrc(const GjDesc *__restrict__ descs, int np, int k0, int k1,
                                                        int in_lds) {
    extern __shared__ int s_rs[];
    __shared__ int s_piv[64];
    const GjDesc g = descs[blockIdx.x];
    const int w = k1 - k0;
    int *rs = in_lds ? s_rs : g.rowsrc;
    if (threadIdx.x < w) s_piv[threadIdx.x] = g.piv[k0 + threadIdx.x];
    for (int i = threadIdx.x; i < np; i += kThreads) rs[i] = i;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int kk = 0; kk < w; ++kk) {
            const int k = k0 + kk, p = s_piv[kk];
            if (p != k) {
                const int t = rs[k];
                rs[k] = rs[p];
                rs[p] = t;
            }
        }
    }
    __syncthreads();
    if (in_lds)
        for (int i = threadIdx.x; i < np; i += kThreads) g.rowsrc[i] = s_rs[i];
}

// Trailing update with the row interchanges folded in, into the other buffer:
//     m2[i][c] = m[rowsrc[i]][c] - sum_j W[i][j] Q[j][c]     (c outside the panel)
//     m2[i][c] = T[i][c - k0]                                 (the panel's columns)
// One workgroup per 64 RT rows (wave w: RT row tiles of 16 rows, their W
// fragments in registers), FP64 16x16x4 matrix cores, the columns in chunks
// of CW = 32 or 64 (two or four 16-wide tiles):
//  * Q chunks go global -> LDS directly (no registers), double-buffered in two
//    arrays the compiler can tell apart, so the next chunk's copy stays in
//    flight while the current chunk's products read the other array; each B
//    operand read from LDS serves the wave's RT row tiles;
//  * two accumulator sets serve even and odd chunks: while one set runs a
//    chunk's products, the other is stored (the previous chunk's results) and
//    reloaded with the next chunk's source rows, so every global access has a
//    chunk of products to complete in before the barrier that waits for it.
// PAIR: two 64-column panels R1 = [k0, k0 + 64) and R2 = [k0 + 64, k0 + 128)
// in one pass (KP = 128).  With P1, P2 the panels' interchanges, T1, T2 their
// factored columns and Q1 = (P1 M)[R1], Q2 = (P2 M1)[R2] the pivot rows
// before each panel's update (M1 = M after the first panel):
//     m2 = P2 P1 M + P2 (T1 - E1) Q1 + (T2 - E2) Q2
// outside R1 and R2; rowsrc holds P2 P1, rowsrc_b P2, qrow the rows of M
// that are Q1, q2 the rows Q2.  R2's columns are T2 (the tail below), R1's
// are written afterwards by k_gj_pair_fix.
template <int KP, int RT, int CW, bool PAIR = false>
__global__ __launch_bounds__(kThreads, 2) void k_gj_update(const GjDesc *__restrict__ descs, int np, int nblk, int k0,
                                                        int w) {
    constexpr int NT = CW / 16, RB = 64 * RT;
    constexpr int PIECES = KP * CW / 2;         // 16-byte pieces of one Q chunk
    constexpr int IPW = PIECES / kThreads;      // direct copies per wave per chunk (64 pieces each)
    static_assert(IPW >= 1 && IPW * kThreads == PIECES, "copy split");
    static_assert(!PAIR || KP == 128, "a pair is two 64-column panels");
    __shared__ __attribute__((aligned(16))) double q_even[KP * CW];
    __shared__ __attribute__((aligned(16))) double q_odd[KP * CW];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * RB;
    const GjDesc g = descs[d];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    DSU_GLOBAL const double *msrc = gmem(g.m);
    DSU_GLOBAL double *mdst = gmem(g.m2);
    // -W = T - E_R from the factored panel T (column-major), zero beyond its width
    double wa[RT][KP / 4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int ra = r0 + 16 * (RT * wave + rt) + lr;
        DSU_GLOBAL const double *tp = gmem(g.panel) + ra;
        if constexpr (PAIR) {
            // steps s < 16 are the first panel's columns j < 64 (row P2[ra] of T1 - E1),
            // the rest the second panel's (row ra of T2 - E2)
            const int rb = g.rowsrc_b[ra];
            DSU_GLOBAL const double *tb = gmem(g.panel_b) + rb;
#pragma unroll
            for (int s = 0; s < KP / 4; ++s) {
                const int j = 4 * s + lk;
                wa[rt][s] = s < KP / 8 ? tb[(size_t)j * np] - (rb == k0 + j ? 1.0 : 0.0)
                                       : tp[(size_t)(j - KP / 2) * np] - (ra == k0 + j ? 1.0 : 0.0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KP / 4; ++s) {
                const int j = 4 * s + lk;
                wa[rt][s] = j < w ? tp[(size_t)j * np] - (ra == k0 + j ? 1.0 : 0.0) : 0.0;
            }
        }
    }
    // Q row j = row k0 + j after the interchanges = M[rowsrc[k0 + j]] (rows
    // j >= w meet zero columns of W; the panel's own columns of the result
    // are replaced below).  This lane's copy pieces: piece p = (wave * IPW +
    // i) * 64 + lane lands at LDS byte 16 p, i.e. Q row p / (CW / 2), columns
    // 2 (p % (CW / 2)) + {0, 1} of the chunk
    // (a pair's Q rows 64.. are the rows of q2)
    size_t qoff[IPW];
    DSU_GLOBAL const double *qbase[IPW];
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
        const int p = (wave * IPW + i) * 64 + lane, qr = p / (CW / 2);
        if constexpr (PAIR) {
            qbase[i] = qr < KP / 2 ? msrc : gmem<const double>(g.q2);
            qoff[i] = (size_t)(qr < KP / 2 ? g.qrow[qr] : qr - KP / 2) * np + 2 * (p % (CW / 2));
        } else {
            qbase[i] = msrc;
            qoff[i] = (size_t)g.rowsrc[k0 + qr] * np + 2 * (p % (CW / 2));
        }
    }
    auto copy_q = [&](int c0, double *dstl) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < IPW; ++i)
            __builtin_amdgcn_global_load_lds((const DSU_GLOBAL void *)(qbase[i] + qoff[i] + c0),
                                             (__attribute__((address_space(3))) void *)(dstl + (wave * IPW + i) * 128),
                                             16, 0, 0);
    };
    // result rows of this lane (FP64 tile layout: row (lane / 16) + 4 i), column lr of each tile
    int row[RT][4];
    DSU_GLOBAL const double *src[RT][4];
    DSU_GLOBAL double *dst[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            row[rt][i] = r0 + 16 * (RT * wave + rt) + Mma<double>::row0(lane) + i * Mma<double>::row_step;
            src[rt][i] = msrc + (size_t)g.rowsrc[row[rt][i]] * np + lr;
            dst[rt][i] = mdst + (size_t)row[rt][i] * np + lr;
        }
    typedef Mma<double>::acc_t acc_set[RT][NT];
    acc_set acc_e, acc_o;
    copy_q(0, q_even);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc_e[rt][t][i] = src[rt][i][16 * t];
    // chunk c0 runs its products on `cur` (loaded with its source rows) and Q
    // in q_cur; `oth` holds chunk c0 - CW's results (c0 > 0), is stored, and
    // takes chunk c0 + CW's source rows (the last chunk re-reads its own rows,
    // so the load is unconditional)
    auto chunk = [&](int c0, const double *q_cur, double *q_nxt, acc_set &cur, acc_set &oth)
        __attribute__((always_inline)) {
        // chunk c0's Q is in q_cur (the barrier waits for this wave's copies,
        // and with them for everything issued before); every wave is done
        // reading q_nxt
        __syncthreads();
        if (c0 > 0)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) dst[rt][i][c0 - CW + 16 * t] = oth[rt][t][i];
        const int c1 = c0 + CW;
        if (c1 < np) copy_q(c1, q_nxt);
        const int cl = c1 < np ? c1 : c0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) oth[rt][t][i] = src[rt][i][cl + 16 * t];
        __builtin_amdgcn_sched_barrier(0);  // stores and next loads issued before the products
        const double *qb = q_cur + lk * CW + lr;
#pragma unroll
        for (int s = 0; s < KP / 4; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double bq = qb[4 * s * CW + 16 * t];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) cur[rt][t] = Mma<double>::mma(wa[rt][s], bq, cur[rt][t]);
            }
    };
    // np is a multiple of 2 CW (the launcher's choice of CW): chunks come in
    // pairs, and the loop body is straight-line code over fixed register sets
    for (int c0 = 0; c0 < np; c0 += 2 * CW) {
        chunk(c0, q_even, q_odd, acc_e, acc_o);
        chunk(c0 + CW, q_odd, q_even, acc_o, acc_e);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[rt][i][np - CW + 16 * t] = acc_o[rt][t][i];
    // The panel's columns (a pair's second panel): the lane that stored each of
    // them overwrites it with the factored panel (same thread, same address:
    // program order holds).
    const int tk0 = PAIR ? k0 + KP / 2 : k0, tw = PAIR ? KP / 2 : w;
    for (int c0 = tk0 - tk0 % CW; c0 < tk0 + tw; c0 += CW)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = c0 + 16 * t + lr;
            if (c >= tk0 && c < tk0 + tw)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        dst[rt][i][c - lr] = g.panel[(size_t)(c - tk0) * np + row[rt][i]];
        }
}

// ---------------------------------------------------------------------------
// Two-level panel factorisation (same algebra one level down).  One panel
// pass of the single-workgroup step above moves the whole N x nb panel for
// every column; here the panel's columns are factored WS at a time inside LDS
// by one workgroup per determinant (k_gj_sub), and each group's row swaps and
// rank-WS update  P_c <- P_c - (E - S) P_c[pivot rows]  reach the panel's
// other columns through k_gj_sub_apply, spread over many workgroups.
// ---------------------------------------------------------------------------
constexpr int kGjThreads = 1024;

// P[j][i] = M[i][k0 + j] for the panel's w columns (64-row tiles through LDS).
__global__ __launch_bounds__(kThreads) void k_gj_gather(const GjDesc *__restrict__ descs, int np, int k0, int w) {
    __shared__ double t[64][65];
    const GjDesc g = descs[blockIdx.y];
    const int r0 = blockIdx.x * 64, tid = threadIdx.x;
    for (int v = tid; v < 64 * w; v += kThreads) {
        const int i = v / w, j = v % w;
        t[i][j] = g.m[(size_t)(r0 + i) * np + k0 + j];
    }
    __syncthreads();
    for (int v = tid; v < 64 * w; v += kThreads) {
        const int j = v / 64, i = v % 64;
        g.panel[(size_t)j * np + r0 + i] = t[i][j];
    }
}

template <int WS, int NPMAX>
__global__ __launch_bounds__(kGjThreads) void k_gj_sub(const GjDesc *__restrict__ descs, int n, int np, int k0, int j0,
                                                       int ws) {
    __shared__ double S[WS * NPMAX];  // the group's columns, S[j * np + i]
    __shared__ double s_v[kGjThreads / 64];
    __shared__ int s_i[kGjThreads / 64];
    const GjDesc g = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *P = g.panel + (size_t)j0 * np;
    for (int v = tid; v < ws * np; v += kGjThreads) S[v] = P[v];
    // running log|det|, sign and status: thread 0's registers for the whole
    // group, read once and written once; the largest pivot so far (the
    // singularity threshold): every thread's register
    double logdet = 0.0, pmax = 0.0;
    int sign = 1, status = 0;
    if (!(k0 == 0 && j0 == 0)) {
        pmax = *g.pmax;
        if (tid == 0) {
            logdet = *g.logdet;
            sign = *g.sign;
            status = *g.status;
        }
    }
    __syncthreads();
    for (int kk = 0; kk < ws; ++kk) {
        const int k = k0 + j0 + kk;
        const double *sc = S + kk * np;
        double best = -1.0;
        int bi = n;
        for (int i = k + tid; i < n; i += kGjThreads) argmax_combine(best, bi, fabs(sc[i]), i);
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(best, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            argmax_combine(best, bi, v2, i2);
        }
        if (lane == 0) { s_v[wave] = best; s_i[wave] = bi; }
        __syncthreads();
        // every thread combines the waves' candidates (same order, same result)
        double bv = s_v[0];
        int p = s_i[0];
#pragma unroll
        for (int q = 1; q < kGjThreads / 64; ++q) argmax_combine(bv, p, s_v[q], s_i[q]);
        pmax = fmax(pmax, bv);
        // singular when the best pivot is at rounding level of the largest one:
        // flagged, and no interchange
        if (!(bv > (double)n * 2.220446049250313e-16 * pmax)) {
            status = -3;
            p = k;
        }
        // the pivot row (old row p) in registers before anything is written
        const double d = S[kk * np + p];
        const double dinv = d != 0.0 ? 1.0 / d : 0.0;
        double rp[WS];
#pragma unroll
        for (int j = 0; j < WS; ++j) rp[j] = j < ws ? (j == kk ? dinv : S[j * np + p] * dinv) : 0.0;
        if (tid == 0) {
            g.piv[k] = p;
            if (d != 0.0) logdet += log(fabs(d));
            if (p != k) sign = -sign;
            if (d < 0.0) sign = -sign;
        }
        __syncthreads();
        // rows after the interchange: row k = the scaled pivot row, row p =
        // old row k eliminated, every other row eliminated in place; the owner
        // of row k writes rows k and p
        for (int i = tid; i < np; i += kGjThreads) {
            if (i == p && p != k) continue;
            if (i == k) {
                const double f = S[kk * np + k];
#pragma unroll
                for (int j = 0; j < WS; ++j) {
                    if (j >= ws) continue;
                    const double ok = S[j * np + k];
                    S[j * np + k] = rp[j];
                    if (p != k) S[j * np + p] = j == kk ? -f * dinv : ok - f * rp[j];
                }
                continue;
            }
            const double f = S[kk * np + i];
#pragma unroll
            for (int j = 0; j < WS; ++j) {
                if (j >= ws) continue;
                S[j * np + i] = j == kk ? -f * dinv : S[j * np + i] - f * rp[j];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        *g.logdet = logdet;
        *g.pmax = pmax;
        *g.sign = sign;
        *g.status = status;
    }
    // the factored columns, and the group's update (E - S) column-major in w
    for (int v = tid; v < ws * np; v += kGjThreads) {
        const int j = v / np, i = v % np;
        P[v] = S[v];
        g.w[v] = (i == k0 + j0 + j ? 1.0 : 0.0) - S[v];
    }
}

// Register-resident form of the group step above: thread t owns rows
// t + 1024 r (r < RPT) of the group's WS columns in registers, so a group can
// be WS = 32 / RPT columns wide where the LDS form holds 4 (np = 4096).  Per
// column two barriers: one for the waves' pivot candidates, one for the
// pivot row and the old row k, which their owners publish in LDS.  Every
// element gets the same operations as in k_gj_sub.
template <int WS, int RPT>
__global__ __launch_bounds__(kGjThreads) void k_gj_subr(const GjDesc *__restrict__ descs, int n, int np, int k0,
                                                        int j0, int ws) {
    __shared__ double s_v[kGjThreads / 64];
    __shared__ int s_i[kGjThreads / 64];
    __shared__ double s_prow[WS], s_krow[WS];
    const GjDesc g = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    DSU_GLOBAL double *P = gmem(g.panel) + (size_t)j0 * np;
    DSU_GLOBAL double *Wg = gmem(g.w);
    double sv[RPT][WS];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = tid + kGjThreads * r;
#pragma unroll
        for (int j = 0; j < WS; ++j) sv[r][j] = 0.0;
        if (i < np) {
            if (ws == WS) {
#pragma unroll
                for (int j = 0; j < WS; ++j) sv[r][j] = P[(size_t)j * np + i];
            } else {
#pragma unroll
                for (int j = 0; j < WS; ++j)
                    if (j < ws) sv[r][j] = P[(size_t)j * np + i];
            }
        }
    }
    double logdet = 0.0, pmax = 0.0;
    int sign = 1, status = 0;
    if (!(k0 == 0 && j0 == 0)) {
        pmax = *g.pmax;
        if (tid == 0) {
            logdet = *g.logdet;
            sign = *g.sign;
            status = *g.status;
        }
    }
    // fully unrolled (every register index fixed); columns past ws skipped
    auto step = [&](auto kk_c) __attribute__((always_inline)) {
        constexpr int kk = decltype(kk_c)::value;
        if (kk >= ws) return;  // uniform
        const int k = k0 + j0 + kk;
        double best = -1.0;
        int bi = n;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + kGjThreads * r;
            if (i >= k && i < n) argmax_combine(best, bi, fabs(sv[r][kk]), i);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(best, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            argmax_combine(best, bi, v2, i2);
        }
        if (lane == 0) { s_v[wave] = best; s_i[wave] = bi; }
        __syncthreads();
        double bv = s_v[0];
        int p = s_i[0];
#pragma unroll
        for (int q = 1; q < kGjThreads / 64; ++q) argmax_combine(bv, p, s_v[q], s_i[q]);
        pmax = fmax(pmax, bv);
        if (!(bv > (double)n * 2.220446049250313e-16 * pmax)) {
            status = -3;
            p = k;
        }
        // the owners publish the pivot row (old row p) and the old row k
        // (rows p and k have one owner each: rare, divergent branches)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + kGjThreads * r;
            if (i == p)
#pragma unroll
                for (int j = 0; j < WS; ++j) s_prow[j] = sv[r][j];
            if (i == k)
#pragma unroll
                for (int j = 0; j < WS; ++j) s_krow[j] = sv[r][j];
        }
        __syncthreads();
        const double d = s_prow[kk];
        const double dinv = d != 0.0 ? 1.0 / d : 0.0;
        if (tid == 0) {
            g.piv[k] = p;
            if (d != 0.0) logdet += log(fabs(d));
            if (p != k) sign = -sign;
            if (d < 0.0) sign = -sign;
        }
        if constexpr (RPT >= 4) {
            // narrow groups: the scaled pivot row (its own column becomes 1/d)
            // in registers; every row eliminated in place, then the owners of
            // rows k and p overwrite theirs: row k = the scaled pivot row, row
            // p = old row k eliminated
            double rp[WS];
#pragma unroll
            for (int j = 0; j < WS; ++j) rp[j] = j == kk ? dinv : s_prow[j] * dinv;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + kGjThreads * r;
                const double f = sv[r][kk];
#pragma unroll
                for (int j = 0; j < WS; ++j) sv[r][j] = j == kk ? -f * dinv : sv[r][j] - f * rp[j];
                if (i == k) {
#pragma unroll
                    for (int j = 0; j < WS; ++j) sv[r][j] = rp[j];
                } else if (i == p) {
                    const double fk = s_krow[kk];
#pragma unroll
                    for (int j = 0; j < WS; ++j) sv[r][j] = j == kk ? -fk * dinv : s_krow[j] - fk * rp[j];
                }
            }
        } else {
            // wide groups (registers are short): the same values by selects,
            // the pivot row read from LDS where it is used
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + kGjThreads * r;
                if (i >= np) continue;
                const bool is_k = i == k, is_p = i == p && p != k;
                const double f = is_p ? s_krow[kk] : sv[r][kk];
#pragma unroll
                for (int j = 0; j < WS; ++j) {
                    const double rpj = j == kk ? dinv : s_prow[j] * dinv;
                    const double cur = is_p ? s_krow[j] : sv[r][j];
                    sv[r][j] = is_k ? rpj : (j == kk ? -f * dinv : cur - f * rpj);
                }
            }
        }
    };
    static_for(std::make_integer_sequence<int, WS>{}, step);
    if (tid == 0) {
        *g.logdet = logdet;
        *g.pmax = pmax;
        *g.sign = sign;
        *g.status = status;
    }
    // the factored columns, and the group's update (E - S) column-major in w
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = tid + kGjThreads * r;
        if (i >= np) continue;
#pragma unroll
        for (int j = 0; j < WS; ++j) {
            if (j >= ws) continue;
            P[(size_t)j * np + i] = sv[r][j];
            Wg[(size_t)j * np + i] = (i == k0 + j0 + j ? 1.0 : 0.0) - sv[r][j];
        }
    }
}

// The group's swaps, then P_c -= (E - S) Q_c, for every other panel column c.
// The swaps k <-> piv[k] (k = k0 + j0 .. + ws - 1, in order) compose into a
// permutation of at most 2 ws rows: row r ends up holding the old row
// s_0(s_1(...s_{ws-1}(r))), traced by one thread per involved row, so the
// values move in one parallel round of loads and stores.  A workgroup takes
// CPB columns, so each element of (E - S) it reads serves CPB of them.
template <int CPB, int RB>
__global__ __launch_bounds__(kThreads) void k_gj_sub_apply(const GjDesc *__restrict__ descs, int np, int k0, int j0,
                                                           int ws, int w) {
    __shared__ int s_k[64], s_p[64], s_src[128];
    __shared__ double s_val[CPB][128];
    const int c0 = blockIdx.x * CPB, tid = threadIdx.x;
    bool on[CPB], any = false;  // columns of this block that take the update: in the panel, outside the group
#pragma unroll
    for (int q = 0; q < CPB; ++q) {
        on[q] = c0 + q < w && !(c0 + q >= j0 && c0 + q < j0 + ws);
        any = any || on[q];
    }
    if (!any) return;  // uniform
    const GjDesc g = descs[blockIdx.y];
    DSU_GLOBAL double *P = gmem(g.panel);
    DSU_GLOBAL const double *Wg = gmem(g.w);
    if (tid < ws) {
        s_k[tid] = k0 + j0 + tid;
        s_p[tid] = g.piv[k0 + j0 + tid];
    }
    __syncthreads();
    if (tid < 2 * ws) {
        int x = tid < ws ? s_k[tid] : s_p[tid - ws];
        for (int kk = ws - 1; kk >= 0; --kk) x = x == s_k[kk] ? s_p[kk] : (x == s_p[kk] ? s_k[kk] : x);
        s_src[tid] = x;
    }
    __syncthreads();
    for (int v = tid; v < CPB * 2 * ws; v += kThreads) {
        const int q = v / (2 * ws), t = v % (2 * ws);
        if (on[q]) s_val[q][t] = P[(size_t)(c0 + q) * np + s_src[t]];
    }
    __syncthreads();
    for (int v = tid; v < CPB * 2 * ws; v += kThreads) {
        const int q = v / (2 * ws), t = v % (2 * ws);
        const int r = t < ws ? s_k[t] : s_p[t - ws];
        if (on[q]) P[(size_t)(c0 + q) * np + r] = s_val[q][t];  // rows named twice receive the same value
    }
    __syncthreads();
    // q[kk] = the value at row k0 + j0 + kk after the swaps = s_val[.][kk].
    // RB rows a thread per pass, their loads all issued before the pass's
    // stores (which may alias them for all the compiler knows): one memory
    // latency per RB rows.  RB = 4 where the blocks are few (np >= 2048: 2 ms
    // less per recompute of 32 x 4096); where they are many, the registers it
    // takes cost more occupancy than it saves (RB = 1).
    for (int i0 = tid; i0 < np; i0 += RB * kThreads) {
        double a[RB][CPB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = i0 + r * kThreads;
#pragma unroll
            for (int q = 0; q < CPB; ++q) a[r][q] = on[q] && i < np ? P[(size_t)(c0 + q) * np + i] : 0.0;
        }
#pragma unroll 8
        for (int kk = 0; kk < ws; ++kk) {
            double e[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = i0 + r * kThreads;
                e[r] = i < np ? Wg[(size_t)kk * np + i] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int q = 0; q < CPB; ++q) a[r][q] -= e[r] * s_val[q][kk];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = i0 + r * kThreads;
#pragma unroll
            for (int q = 0; q < CPB; ++q)
                if (on[q] && i < np) P[(size_t)(c0 + q) * np + i] = a[r][q];
        }
    }
}

// ---------------------------------------------------------------------------
// Panel pairs: the pieces of the fused two-panel step around k_gj_update's
// PAIR form (same notation: R1, R2, P1, P2, T1, T2, Q1, Q2, M1).
// ---------------------------------------------------------------------------

// After the first panel: R2's columns of M1 = P1 M + (T1 - E1) Q1 become the
// second panel, and T1 moves to panel_b.  Rows are independent, so each block
// rewrites the rows it read.  One block per 64 rows.  In the three pair
// kernels every global load of a thread is issued before its first store (the
// stores may alias the loads for all the compiler knows, which would otherwise
// serialise them), and the 64-term products run in two halves of 32 through
// 32 KB of LDS (three blocks a compute unit instead of two).
constexpr int kPairLoads = 64 * 64 / kThreads;  // elements of a 64 x 64 tile per thread
constexpr int kPairHalf = kPairLoads / 2;       // element q holds index grp + 4 q: q < 8 is the first half

__global__ __launch_bounds__(kThreads) void k_gj_pair_slab(const GjDesc *__restrict__ descs, int np, int k0) {
    __shared__ double s_t[32][64];  // (T1 - E1)[r0 + i][l] at s_t[l - 32 h][i], half h of l at a time
    __shared__ double s_q[32][64];  // Q1[l][R2 column j] at s_q[l - 32 h][j]
    const GjDesc g = descs[blockIdx.y];
    const int r0 = blockIdx.x * 64, tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    DSU_GLOBAL const double *m = gmem<const double>(g.m);
    DSU_GLOBAL double *pb = gmem(g.panel_b), *pa = gmem(g.panel);
    // element q of this thread: column / row a = grp + 4 q, the other index lane
    double tv[kPairLoads], qv[kPairLoads], acc[16];
    int qr[kPairLoads];
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) qr[q] = g.rowsrc[k0 + grp + 4 * q];
    // lane = row, 16 columns a thread (one 128-byte line of its row of P1 M)
    DSU_GLOBAL const double *mr = m + (size_t)g.rowsrc[r0 + lane] * np + k0 + 64 + 16 * grp;
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) {
        tv[q] = pa[(size_t)(grp + 4 * q) * np + r0 + lane];
        qv[q] = m[(size_t)qr[q] * np + k0 + 64 + lane];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = mr[q];
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) pb[(size_t)(grp + 4 * q) * np + r0 + lane] = tv[q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();  // the first half read by every wave
#pragma unroll
        for (int q = kPairHalf * h; q < kPairHalf * (h + 1); ++q) {
            const int a = grp + 4 * q;
            s_t[a - 32 * h][lane] = tv[q] - (r0 + lane == k0 + a ? 1.0 : 0.0);
            s_q[a - 32 * h][lane] = qv[q];
        }
        __syncthreads();
        for (int l = 0; l < 32; ++l) {
            const double t = s_t[l][lane];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = __builtin_fma(t, s_q[l][16 * grp + q], acc[q]);
        }
    }
    // column-major stores, coalesced
#pragma unroll
    for (int q = 0; q < 16; ++q) pa[(size_t)(16 * grp + q) * np + r0 + lane] = acc[q];
}

// After the second panel: rowsrc_b = P2 (its own swaps), rowsrc = P2 P1 (row
// i of the result <- row rowsrc[i] of M), qrow[l] = P1's source of row k0 + l.
// One workgroup per determinant; both maps in dynamic LDS (8 np bytes).
__global__ __launch_bounds__(kThreads) void k_gj_pair_rowsrc(const GjDesc *__restrict__ descs, int np, int k0) {
    extern __shared__ int s_rr[];
    __shared__ int s_piv[64];
    const GjDesc g = descs[blockIdx.x];
    int *r1 = s_rr, *r2 = s_rr + np;
    if (threadIdx.x < 64) s_piv[threadIdx.x] = g.piv[k0 + 64 + threadIdx.x];
    for (int i = threadIdx.x; i < np; i += kThreads) {
        r1[i] = g.rowsrc[i];
        r2[i] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int kk = 0; kk < 64; ++kk) {
            const int k = k0 + 64 + kk, p = s_piv[kk];
            if (p != k) {
                const int t = r2[k];
                r2[k] = r2[p];
                r2[p] = t;
            }
        }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += kThreads) {
        g.rowsrc_b[i] = r2[i];
        g.rowsrc[i] = r1[r2[i]];
    }
    if (threadIdx.x < 64) g.qrow[threadIdx.x] = r1[k0 + threadIdx.x];
}

// Q2[j] = M1[P2 row k0 + 64 + j] = M[rowsrc[k0 + 64 + j]] + (T1 - E1)[r_j] Q1,
// r_j = rowsrc_b[k0 + 64 + j], for all columns (R1's and R2's are not used).
// One block per 64 columns; loads first and halves of 32, as above.
__global__ __launch_bounds__(kThreads) void k_gj_pair_q2(const GjDesc *__restrict__ descs, int np, int k0) {
    __shared__ double s_w[32][64];  // (T1 - E1)[r_j][l] at s_w[l - 32 h][j]
    __shared__ double s_q[32][64];  // Q1[l][c0 + c] at s_q[l - 32 h][c]
    const GjDesc g = descs[blockIdx.y];
    const int c0 = blockIdx.x * 64, tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    DSU_GLOBAL const double *m = gmem<const double>(g.m), *pb = gmem<const double>(g.panel_b);
    double wv[kPairLoads], qv[kPairLoads], acc[16];
    int qr[kPairLoads], sr[16];
    const int r = g.rowsrc_b[k0 + 64 + lane];  // r_j of j = lane
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) qr[q] = g.qrow[grp + 4 * q];
#pragma unroll
    for (int q = 0; q < 16; ++q) sr[q] = g.rowsrc[k0 + 64 + 16 * grp + q];
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) {
        qv[q] = m[(size_t)qr[q] * np + c0 + lane];
        wv[q] = pb[(size_t)(grp + 4 * q) * np + r];
    }
    // lane = column, 16 rows of Q2 a thread
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = m[(size_t)sr[q] * np + c0 + lane];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();
#pragma unroll
        for (int q = kPairHalf * h; q < kPairHalf * (h + 1); ++q) {
            const int a = grp + 4 * q;
            s_q[a - 32 * h][lane] = qv[q];
            s_w[a - 32 * h][lane] = wv[q] - (r == k0 + a ? 1.0 : 0.0);
        }
        __syncthreads();
        for (int l = 0; l < 32; ++l) {
            const double qq = s_q[l][lane];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = __builtin_fma(s_w[l][16 * grp + q], qq, acc[q]);
        }
    }
    // row-major stores, coalesced
#pragma unroll
    for (int q = 0; q < 16; ++q) g.q2[(size_t)(16 * grp + q) * np + c0 + lane] = acc[q];
}

// R1's columns of the pair's result: m2[i][k0 + j] = (P2 T1)[i][j] +
// (T2 - E2)[i] (P2 T1)[R2][j] (T1 is M1's R1 block, Q2's R1 columns are its
// rows at P2's pivots).  Runs after the update, which leaves those columns
// to it.  One block per 64 rows; loads first, as above.  The 32 KB of LDS
// first hold (P2 T1) of the block's rows at [i][j ^ i] (an XOR swizzle: the
// row-wise stores and column-wise reads both spread over the LDS banks), then
// per half h of l: (T2 - E2)[r0 + i][l] at [l - 32 h][i] in the first 16 KB
// and (P2 T1)[R2 row l][j] at [l - 32 h][j ^ l] in the second.
__global__ __launch_bounds__(kThreads) void k_gj_pair_fix(const GjDesc *__restrict__ descs, int np, int k0) {
    __shared__ double s_buf[64 * 64];
    const GjDesc g = descs[blockIdx.y];
    const int r0 = blockIdx.x * 64, tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    DSU_GLOBAL const double *pa = gmem<const double>(g.panel), *pb = gmem<const double>(g.panel_b);
    double av[kPairLoads], x1[kPairLoads], x2[kPairLoads], acc[16];
    const int rb = g.rowsrc_b[r0 + lane], rz = g.rowsrc_b[k0 + 64 + lane];
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) {
        const int a = grp + 4 * q;
        av[q] = pa[(size_t)a * np + r0 + lane];
        x1[q] = pb[(size_t)a * np + rb];
        x2[q] = pb[(size_t)a * np + rz];
    }
#pragma unroll
    for (int q = 0; q < kPairLoads; ++q) {
        const int a = grp + 4 * q;
        s_buf[lane * 64 + (a ^ lane)] = x1[q];
    }
    __syncthreads();
    // lane = column, 16 rows a thread
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = 16 * grp + q;
        acc[q] = s_buf[i * 64 + (lane ^ i)];
    }
    double *s_a = s_buf, *s_z = s_buf + 32 * 64;
    // half h of l (a compile-time constant, so every register index is fixed)
    auto half = [&](auto h_c) __attribute__((always_inline)) {
        constexpr int h = decltype(h_c)::value;
        __syncthreads();  // every wave done with the previous contents
#pragma unroll
        for (int q = kPairHalf * h; q < kPairHalf * (h + 1); ++q) {
            const int a = grp + 4 * q;
            s_a[(a - 32 * h) * 64 + lane] = av[q] - (r0 + lane == k0 + 64 + a ? 1.0 : 0.0);
        }
        if ((lane >> 5) == h)
#pragma unroll
            for (int q = 0; q < kPairLoads; ++q) {
                const int a = grp + 4 * q;
                s_z[(lane - 32 * h) * 64 + (a ^ lane)] = x2[q];
            }
        __syncthreads();
#pragma unroll 4
        for (int l = 0; l < 32; ++l) {
            const int la = 32 * h + l;
            const double z = s_z[l * 64 + (lane ^ la)];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = __builtin_fma(s_a[l * 64 + 16 * grp + q], z, acc[q]);
        }
    };
    half(std::integral_constant<int, 0>{});
    half(std::integral_constant<int, 1>{});
    // row-major stores, coalesced
#pragma unroll
    for (int q = 0; q < 16; ++q) g.m2[(size_t)(r0 + 16 * grp + q) * np + k0 + lane] = acc[q];
}

template <int RT, int CW>
static void launch_gj_update(const GjDesc *descs_dev, int ndesc, int np, int nb, int k0, int w, hipStream_t s) {
    const int nblk = np / (64 * RT);
    const dim3 grid(ndesc * nblk);
    if (nb == 16) hipLaunchKernelGGL((k_gj_update<16, RT, CW>), grid, dim3(kThreads), 0, s, descs_dev, np, nblk, k0, w);
    else if (nb == 32) hipLaunchKernelGGL((k_gj_update<32, RT, CW>), grid, dim3(kThreads), 0, s, descs_dev, np, nblk, k0, w);
    else hipLaunchKernelGGL((k_gj_update<64, RT, CW>), grid, dim3(kThreads), 0, s, descs_dev, np, nblk, k0, w);
}

// gather = 0: the panel buffer already holds the panel's columns (a pair's second panel)
template <int WS, int NPMAX, bool REG = false>
static void launch_gj_panel2(const GjDesc *descs_dev, int ndesc, int n, int np, int nb, int k0, int w, int cpb,
                             hipStream_t s, bool gather = true) {
    if (gather) hipLaunchKernelGGL(k_gj_gather, dim3(np / 64, ndesc), dim3(kThreads), 0, s, descs_dev, np, k0, w);
    for (int j0 = 0; j0 < w; j0 += WS) {
        const int ws = j0 + WS <= w ? WS : w - j0;
        if constexpr (REG)
            hipLaunchKernelGGL((k_gj_subr<WS, NPMAX / kGjThreads>), dim3(ndesc), dim3(kGjThreads), 0, s, descs_dev, n,
                               np, k0, j0, ws);
        else
            hipLaunchKernelGGL((k_gj_sub<WS, NPMAX>), dim3(ndesc), dim3(kGjThreads), 0, s, descs_dev, n, np, k0, j0,
                               ws);
        if (w > ws && cpb == 4 && np >= 2048)
            hipLaunchKernelGGL((k_gj_sub_apply<4, 4>), dim3((w + 3) / 4, ndesc), dim3(kThreads), 0, s, descs_dev, np,
                               k0, j0, ws, w);
        else if (w > ws && cpb == 4)
            hipLaunchKernelGGL((k_gj_sub_apply<4, 1>), dim3((w + 3) / 4, ndesc), dim3(kThreads), 0, s, descs_dev, np,
                               k0, j0, ws, w);
        else if (w > ws)
            hipLaunchKernelGGL((k_gj_sub_apply<1, 1>), dim3(w, ndesc), dim3(kThreads), 0, s, descs_dev, np, k0, j0, ws,
                               w);
    }
}

// Final column permutation: idx = identity, then for k = n-1..0 swap idx[k],
// idx[piv[k]].  The swaps are a serial chain on one thread; it runs over LDS
// copies of the pivots and the permutation (dynamic LDS: 8 np bytes) when
// they fit, which the workgroup loads and stores in parallel, else in place.
__global__ __launch_bounds__(kThreads) void k_gj_perm(const GjDesc *__restrict__ descs, int n, int np, int in_lds) {
    extern __shared__ int s_pp[];
    const GjDesc g = descs[blockIdx.x];
    int *perm = in_lds ? s_pp : g.perm;
    const int *piv = in_lds ? s_pp + np : g.piv;
    for (int j = threadIdx.x; j < np; j += kThreads) {
        perm[j] = j;
        if (in_lds) s_pp[np + j] = j < n ? g.piv[j] : j;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = n - 1; k >= 0; --k) {
            const int p = piv[k];
            const int t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
    __syncthreads();
    if (in_lds)
        for (int j = threadIdx.x; j < np; j += kThreads) g.perm[j] = s_pp[j];
}

GjTiles gj_tiles_default(int n, int np) {
    // measured on MI355X: 64-column panels from N = 512, in pairs from 1024
    // (4096: 146 ms against 162 for 32 inverses, 2048: 45 against 47 ms for
    // 64, 1024: 26.2 against 26.8 ms for 256; at 512 single panels are
    // faster); 64-column update chunks where np pairs them up (3 % faster
    // than 32 at N = 4096); four apply columns a workgroup from N = 2048 (one
    // below: enough workgroups)
    GjTiles t;
    t.nb = n >= 1024 && np <= 4096 ? 128 : (n >= 512 ? 64 : (n >= 64 ? 32 : 16));
    t.cw = np % 128 == 0 ? 64 : 32;
    t.cpb = np >= 2048 ? 4 : 1;
    return t;
}

hipError_t launch_gj_invert(const GjDesc *set_a, const GjDesc *set_b, int ndesc, int n, int np, const GjTiles &tiles,
                            hipStream_t s, const GjDesc **final_set) {
    const int nb = tiles.nb, cw = tiles.cw, cpb = tiles.cpb;
    if (nb != 16 && nb != 32 && nb != 64 && nb != 128) return hipErrorInvalidValue;
    if (np % 64) return hipErrorInvalidValue;  // the trailing update takes column chunks in pairs
    if (!(cw == 32 || (cw == 64 && np % 128 == 0)) || (cpb != 1 && cpb != 4)) return hipErrorInvalidValue;
    const int pw = nb == 128 ? 64 : nb;  // columns factored at a time
    const int in_lds = np <= 8192;       // row map in dynamic LDS (32 KB at most)
    // factor the panel [k0, k0 + w): groups of 32 / 16 / 8 columns in registers up to np = 4096 (32 doubles a
    // thread), then 2 columns in LDS up to 8192, else one column at a time
    auto factor = [&](const GjDesc *d, int k0, int w, bool gather) {
        if (np <= 1024) launch_gj_panel2<32, 1024, true>(d, ndesc, n, np, pw, k0, w, cpb, s, gather);
        else if (np <= 2048) launch_gj_panel2<16, 2048, true>(d, ndesc, n, np, pw, k0, w, cpb, s, gather);
        else if (np <= 4096) launch_gj_panel2<8, 4096, true>(d, ndesc, n, np, pw, k0, w, cpb, s, gather);
        else if (np <= 8192) launch_gj_panel2<2, 8192>(d, ndesc, n, np, pw, k0, w, cpb, s, gather);
        else hipLaunchKernelGGL(k_gj_panel, dim3(ndesc), dim3(kThreads), 0, s, d, n, np, pw, k0, k0 + w);
    };
    const GjDesc *cur = set_a, *nxt = set_b;
    for (int k0 = 0; k0 < n;) {
        const int k1 = k0 + pw < n ? k0 + pw : n;
        // two whole 64-column panels share one trailing update (both row maps
        // in LDS: np <= 4096); otherwise one panel at a time
        const bool pair = nb == 128 && k0 + 128 <= n && np <= 4096;
        factor(cur, k0, k1 - k0, true);
        // row interchanges, then the trailing update into the other buffer
        hipLaunchKernelGGL(k_gj_rowsrc, dim3(ndesc), dim3(kThreads), in_lds ? np * sizeof(int) : 0, s, cur, np, k0,
                           k1, in_lds);
        if (pair) {
            hipLaunchKernelGGL(k_gj_pair_slab, dim3(np / 64, ndesc), dim3(kThreads), 0, s, cur, np, k0);
            factor(cur, k0 + 64, 64, false);
            hipLaunchKernelGGL(k_gj_pair_rowsrc, dim3(ndesc), dim3(kThreads), (size_t)np * 2 * sizeof(int), s, cur, np,
                               k0);
            hipLaunchKernelGGL(k_gj_pair_q2, dim3(np / 64, ndesc), dim3(kThreads), 0, s, cur, np, k0);
            hipLaunchKernelGGL((k_gj_update<128, 1, 32, true>), dim3(ndesc * (np / 64)), dim3(kThreads), 0, s, cur, np,
                               np / 64, k0, 64);
            hipLaunchKernelGGL(k_gj_pair_fix, dim3(np / 64, ndesc), dim3(kThreads), 0, s, cur, np, k0);
            k0 += 128;
        } else {
            // (128-row workgroups, RT = 2, measured no faster than 64-row ones)
            if (cw == 64)
                launch_gj_update<1, 64>(cur, ndesc, np, pw, k0, k1 - k0, s);
            else
                launch_gj_update<1, 32>(cur, ndesc, np, pw, k0, k1 - k0, s);
            k0 = k1;
        }
        const GjDesc *t = cur;
        cur = nxt;
        nxt = t;
    }
    const int perm_lds = np <= 8192;  // 64 KB of dynamic LDS at most
    hipLaunchKernelGGL(k_gj_perm, dim3(ndesc), dim3(kThreads), perm_lds ? (size_t)np * 2 * sizeof(int) : 0, s, cur, n,
                       np, perm_lds);
    if (final_set) *final_set = cur;
    return hipGetLastError();
}

// BT[i][j] = T(M[i][perm[j]]) inside n x n, zero padding.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cast_perm(const GjDesc *__restrict__ gj, T *const *__restrict__ bt, int n,
                                                        int np) {
    const int d = blockIdx.z;
    const GjDesc g = gj[d];
    T *out = bt[d];
    const int j = blockIdx.x * kThreads + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= np) return;
    out[(size_t)i * np + j] = (i < n && j < n) ? T(g.m[(size_t)i * np + g.perm[j]]) : T(0);
}

// The same with the row staged in LDS first (one row per workgroup, dynamic
// LDS of np doubles): the permuted gather then reads LDS instead of scattered
// global lines; the row comes in with 16-byte loads and leaves four columns a
// thread (np is a multiple of 64).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cast_perm_row(const GjDesc *__restrict__ gj, T *const *__restrict__ bt,
                                                            int n, int np) {
    extern __shared__ double s_row[];
    typedef double d2 __attribute__((ext_vector_type(2)));
    const GjDesc g = gj[blockIdx.y];
    T *out = bt[blockIdx.y] + (size_t)blockIdx.x * np;
    const int i = blockIdx.x;
    const d2 *src = reinterpret_cast<const d2 *>(g.m + (size_t)i * np);
    for (int j = threadIdx.x; j < np / 2; j += kThreads) reinterpret_cast<d2 *>(s_row)[j] = src[j];
    __syncthreads();
    for (int j4 = threadIdx.x; j4 < np / 4; j4 += kThreads) {
        const int j = 4 * j4;
        const int4 pv = reinterpret_cast<const int4 *>(g.perm)[j4];
        const int pj[4] = {pv.x, pv.y, pv.z, pv.w};
        T v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (i < n && j + e < n) ? T(s_row[pj[e]]) : T(0);
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4 *>(out + j) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            reinterpret_cast<d2 *>(out + j)[0] = d2{(double)v[0], (double)v[1]};
            reinterpret_cast<d2 *>(out + j)[1] = d2{(double)v[2], (double)v[3]};
        }
    }
}

template <typename T>
hipError_t launch_cast_perm(const GjDesc *gj_dev, T *const *bt_dev, int ndesc, int n, int np, hipStream_t s) {
    if (np <= 8192)
        hipLaunchKernelGGL((k_cast_perm_row<T>), dim3(np, ndesc), dim3(kThreads), (size_t)np * sizeof(double), s,
                           gj_dev, bt_dev, n, np);
    else
        hipLaunchKernelGGL((k_cast_perm<T>), dim3((np + kThreads - 1) / kThreads, np, ndesc), dim3(kThreads), 0, s,
                           gj_dev, bt_dev, n, np);
    return hipGetLastError();
}
template hipError_t launch_cast_perm<float>(const GjDesc *, float *const *, int, int, int, hipStream_t);
template hipError_t launch_cast_perm<double>(const GjDesc *, double *const *, int, int, int, hipStream_t);

// M = A^T padded with the identity (32 x 32 tiles through LDS).
__global__ __launch_bounds__(kThreads) void k_load_transpose(const double *const *__restrict__ a_all,
                                                             double *const *__restrict__ m_all, int n, int np, int lda) {
    __shared__ double tile[32][33];
    const double *a = a_all[blockIdx.z];
    double *m = m_all[blockIdx.z];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;  // read A[i][j]
        tile[r][tx] = (i < n && j < n) ? a[(size_t)i * lda + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;  // write M[j][i] = A[i][j]
        if (j < np && i < np) m[(size_t)j * np + i] = tile[tx][r];
    }
}

hipError_t launch_load_transpose(const double *const *a_dev, double *const *m_dev, int ndesc, int n, int np, int lda,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_load_transpose, dim3(np / 32, np / 32, ndesc), dim3(kThreads), 0, s, a_dev, m_dev, n, np, lda);
    return hipGetLastError();
}

// out[i][j] = BT[j][i], n x n FP64.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_untranspose(const T *__restrict__ bt, double *__restrict__ out, int n,
                                                          int np) {
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        tile[r][tx] = (i < n && j < n) ? double(bt[(size_t)i * np + j]) : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (j < n && i < n) out[(size_t)j * n + i] = tile[tx][r];
    }
}

template <typename T>
hipError_t launch_untranspose(const T *bt, double *out, int n, int np, hipStream_t s) {
    hipLaunchKernelGGL((k_untranspose<T>), dim3(np / 32, np / 32), dim3(kThreads), 0, s, bt, out, n, np);
    return hipGetLastError();
}
template hipError_t launch_untranspose<float>(const float *, double *, int, int, hipStream_t);
template hipError_t launch_untranspose<double>(const double *, double *, int, int, hipStream_t);

}  // namespace dsu
