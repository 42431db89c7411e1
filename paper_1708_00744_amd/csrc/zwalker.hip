// zwalker.hip -- the host-driven single walker with complex orbitals
// (twisted boundary conditions), FP64 complex arithmetic throughout.
//
// The method carries over unchanged: the determinant lemma and the Woodbury
// identity hold over the complex field with plain (not conjugate) transposes,
// so the look-ahead ratio of Sec. II, eq. (3), is R = r0 - p^T C_k^{-1} q,
// C_k^{-1} is bordered on each acceptance, and the flush is eq. (4):
// Y = BT U^T, Y[e_j][j] -= 1, W = Y C^{-T}, BT -= W Vg.  BT = (A^{-1})^T.
// The Metropolis weight is |R|^2; the walker tracks log|det A| and arg det A.
// Complex values are stored interleaved (re, im) as double2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_common.hpp"

namespace dsu {

typedef double2 zc;

__device__ __forceinline__ zc zmul(zc a, zc b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ zc zfma(zc a, zc b, zc c) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ zc zsub(zc a, zc b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ zc zinv(zc a) {
    const double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
}

struct ZWalkerDev {
    zc *bt;            // np x np
    zc *u;             // kp x np: new rows of the pending moves
    zc *vg;            // kp x np: stale BT rows of the pending electrons
    zc *a;             // np x np: Slater matrix
    zc *phi;           // np: pending proposal row
    zc *cinv;          // kp x (kp + 1): C_k^{-1} in pending order
    zc *dots;          // 1 + 2 kp: r0, p[0..k), q[0..k)
    zc *t;             // kp: C_k^{-1} q
    zc *ratio;         // device copy of R
    double *ratio_host;// mapped pinned: R (re, im), then the call's completion tag
    int *idx;          // kp pending electrons
    unsigned *counter; // blocks finished (last-block reduction)
    zc *w;             // np x (kp + 1): flush scratch W
    zc *fcol;          // np: Gauss-Jordan multipliers
    int *piv;          // np: Gauss-Jordan row interchanges
    double *stat;      // log|det|, arg det, largest pivot modulus
    int *status;       // 1 if a pivot is singular to working precision
    int ldc;           // kp + 1
};

__device__ __forceinline__ zc block_zsum(zc v, zc *sbuf) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[wave] = v;
    __syncthreads();
    zc s = make_double2(0.0, 0.0);
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s = make_double2(s.x + sbuf[q].x, s.y + sbuf[q].y);
    return s;
}

// Look-ahead ratio: 2k+1 blocks (r0, p, q dot products); the last block to
// finish forms t = C_k^{-1} q and R = r0 - p.t.
__global__ __launch_bounds__(kThreads) void k_zpropose(ZWalkerDev w, int np, int k, int e, unsigned tag) {
    __shared__ zc sbuf[kThreads / 64];
    __shared__ int is_last;
    __shared__ zc s_t[DSU_KMAX_LDS];
    const int b = blockIdx.x, tid = threadIdx.x;
    const zc *x, *yv;
    if (b == 0) { x = w.phi; yv = w.bt + (size_t)e * np; }
    else if (b <= k) { x = w.phi; yv = w.vg + (size_t)(b - 1) * np; }
    else { x = w.u + (size_t)(b - 1 - k) * np; yv = w.bt + (size_t)e * np; }
    zc acc = make_double2(0.0, 0.0);
    for (int c = tid; c < np; c += kThreads) acc = zfma(x[c], yv[c], acc);
    acc = block_zsum(acc, sbuf);
    if (tid == 0) {
        w.dots[b] = acc;
        __threadfence();
        is_last = atomicAdd(w.counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    for (int i = tid; i < k; i += kThreads) {
        zc s = make_double2(0.0, 0.0);
        for (int j = 0; j < k; ++j) s = zfma(w.cinv[(size_t)i * w.ldc + j], w.dots[1 + k + j], s);
        s_t[i] = s;
        w.t[i] = s;
    }
    __syncthreads();
    zc part = make_double2(0.0, 0.0);
    for (int i = tid; i < k; i += kThreads) part = zfma(w.dots[1 + i], s_t[i], part);
    part = block_zsum(part, sbuf);
    if (tid == 0) {
        const zc r = zsub(w.dots[0], part);
        w.ratio[0] = r;
        w.ratio_host[0] = r.x;
        w.ratio_host[1] = r.y;
        *w.counter = 0u;
        __threadfence_system();  // the ratio reaches host memory before the tag
        w.ratio_host[2] = (double)tag;
    }
}

// Bordering on acceptance (one block):
//   C_{k+1}^{-1} = [[C^{-1} + t b^T / R, -t / R], [-b^T / R, 1 / R]],
//   t = C^{-1} q, b^T = p^T C^{-1}; then append U, Vg, A rows and the electron.
__global__ __launch_bounds__(kThreads) void k_zaccept(ZWalkerDev w, int np, int k, int e) {
    __shared__ zc s_b[DSU_KMAX_LDS];
    __shared__ zc s_t[DSU_KMAX_LDS];
    const int tid = threadIdx.x;
    const zc rinv = zinv(w.ratio[0]);
    for (int j = tid; j < k; j += kThreads) {
        zc s = make_double2(0.0, 0.0);
        for (int i = 0; i < k; ++i) s = zfma(w.dots[1 + i], w.cinv[(size_t)i * w.ldc + j], s);
        s_b[j] = zmul(s, rinv);
        s_t[j] = w.t[j];
    }
    __syncthreads();
    const int k1 = k + 1;
    for (int v = tid; v < k1 * k1; v += kThreads) {
        const int i = v / k1, j = v % k1;
        zc *c = w.cinv + (size_t)i * w.ldc + j;
        if (i < k && j < k) *c = zfma(s_t[i], s_b[j], *c);
        else if (i < k) {
            const zc v = zmul(s_t[i], rinv);
            *c = make_double2(-v.x, -v.y);
        }
        else if (j < k) *c = make_double2(-s_b[j].x, -s_b[j].y);
        else *c = rinv;
    }
    for (int c = tid; c < np; c += kThreads) {
        w.u[(size_t)k * np + c] = w.phi[c];
        w.vg[(size_t)k * np + c] = w.bt[(size_t)e * np + c];
        w.a[(size_t)e * np + c] = w.phi[c];
    }
    if (tid == 0) w.idx[k] = e;
}

// C[M x N] = (or -=) A[M x Kd] op(B); op(B) = B^T with B stored N x Kd when
// TRANSB, else B stored Kd x N.  64 x 64 tile per workgroup, 4 x 4 per thread.
template <bool TRANSB, bool SUB>
__global__ __launch_bounds__(kThreads) void k_zgemm(const zc *__restrict__ A, int lda, const zc *__restrict__ B, int ldb,
                                                    zc *C, int ldc, int M, int N, int Kd) {
    constexpr int TM = 64, TN = 64, TK = 8;
    __shared__ zc sa[TK][TM + 1], sb[TK][TN + 1];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    zc acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < Kd; k0 += TK) {
        for (int v = tid; v < TM * TK; v += kThreads) {
            const int i = v / TK, kk = v % TK, m = m0 + i, kx = k0 + kk;
            sa[kk][i] = (m < M && kx < Kd) ? A[(size_t)m * lda + kx] : make_double2(0.0, 0.0);
        }
        for (int v = tid; v < TN * TK; v += kThreads) {
            if (TRANSB) {
                const int j = v / TK, kk = v % TK, n = n0 + j, kx = k0 + kk;
                sb[kk][j] = (n < N && kx < Kd) ? B[(size_t)n * ldb + kx] : make_double2(0.0, 0.0);
            } else {
                const int kk = v / TN, j = v % TN, n = n0 + j, kx = k0 + kk;
                sb[kk][j] = (n < N && kx < Kd) ? B[(size_t)kx * ldb + n] : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            zc a[4], bb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = sa[kk][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bb[c] = sb[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = zfma(a[r], bb[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = m0 + ty + 16 * r, n = n0 + tx + 16 * c;
            if (m < M && n < N) {
                zc *p = C + (size_t)m * ldc + n;
                *p = SUB ? zsub(*p, acc[r][c]) : acc[r][c];
            }
        }
}

template <bool TRANSB, bool SUB>
static hipError_t zgemm(const zc *A, int lda, const zc *B, int ldb, zc *C, int ldc, int M, int N, int Kd, hipStream_t s) {
    const dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_zgemm<TRANSB, SUB>), grid, dim3(kThreads), 0, s, A, lda, B, ldb, C, ldc, M, N, Kd);
    return hipGetLastError();
}

// Flush, first half, one wave per row of BT (4 rows per workgroup): the
// row's look-ahead products y_j = BT[i] . U[j] (16 slots at a time, lanes
// striding the columns, then a wave reduction), y_j -= 1 where e_j = i, and
// the row of W = (Y - E) C^{-T}: w_j = sum_l y_l Cinv[j][l].
__global__ __launch_bounds__(kThreads) void k_zflush_w(ZWalkerDev w, int np, int k) {
    __shared__ zc s_y[4][DSU_KMAX_LDS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + wave;  // np is a multiple of 64: every wave has a row
    const zc *bt = w.bt + (size_t)i * np;
    for (int j0 = 0; j0 < k; j0 += 16) {
        const int nj = k - j0 < 16 ? k - j0 : 16;
        zc acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = make_double2(0.0, 0.0);
        for (int c = lane; c < np; c += 64) {
            const zc b = bt[c];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < nj) acc[j] = zfma(b, w.u[(size_t)(j0 + j) * np + c], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            zc v = acc[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                v.x += __shfl_xor(v.x, o, 64);
                v.y += __shfl_xor(v.y, o, 64);
            }
            if (lane == 0 && j < nj) s_y[wave][j0 + j] = make_double2(v.x - (w.idx[j0 + j] == i ? 1.0 : 0.0), v.y);
        }
    }
    __syncthreads();
    for (int j = lane; j < k; j += 64) {
        zc s = make_double2(0.0, 0.0);
        for (int l = 0; l < k; ++l) s = zfma(s_y[wave][l], w.cinv[(size_t)j * w.ldc + l], s);
        w.w[(size_t)i * w.ldc + j] = s;
    }
}

// Real embedding of the rank-k update BT -= W Vg for the FP64 matrix cores.
// Read as real matrices (each complex entry two adjacent doubles), BT is
// np x 2np and W np x 2k; with Vg[j][c] = x + i y,
//   Vh[2j][2c] = x,  Vh[2j][2c+1] = y,  Vh[2j+1][2c] = -y,  Vh[2j+1][2c+1] = x
// the real product W Vh is W Vg: each complex product as its four real
// products.  Rows 2k .. kp2-1 of Vh are zero.
__global__ void k_zembed_v(ZWalkerDev w, double *vh, int np, int k) {
    const int r = blockIdx.y;  // embedded slot row
    const int j = r >> 1, odd = r & 1;
    const bool live = j < k;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < np; c += gridDim.x * blockDim.x) {
        const zc v = live ? w.vg[(size_t)j * np + c] : make_double2(0.0, 0.0);
        double *vr = vh + (size_t)r * 2 * np + 2 * c;
        vr[0] = odd ? -v.y : v.x;
        vr[1] = odd ? v.x : v.y;
    }
}

// BT[i][j] = A[j][i] for i, j < n (zero elsewhere up to np).
__global__ void k_zload_t(const zc *a, zc *bt, int n, int np) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= np) return;
    bt[(size_t)i * np + j] = (i < n && j < n) ? a[(size_t)j * np + i] : make_double2(0.0, 0.0);
}

// One Gauss-Jordan step on column kk (one workgroup): partial pivoting by
// modulus (lowest row on ties), row interchange, pivot row scaled by 1/p with
// 1/p left in the pivot position, multipliers of the other rows saved and
// their column-kk entries cleared; log|p|, arg p (+ pi per interchange) and
// the largest pivot modulus accumulated; a pivot at or below n 2^-52 times the
// largest so far marks the matrix singular.
__global__ __launch_bounds__(1024) void k_zgj_pivot(ZWalkerDev w, int ld, int n, int kk) {
    __shared__ double s_v[1024];
    __shared__ int s_i[1024];
    const int tid = threadIdx.x;
    zc *m = w.bt;
    // a row index in [kk, n) is always chosen (NaN moduli lose every
    // comparison, so a column of NaN keeps row kk and is flagged below)
    double best = -1.0;
    int bi = kk;
    for (int i = kk + tid; i < n; i += 1024) {
        const zc v = m[(size_t)i * ld + kk];
        const double a = hypot(v.x, v.y);
        if (a > best) { best = a; bi = i; }
    }
    s_v[tid] = best;
    s_i[tid] = bi;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o) {
            const double a = s_v[tid + o];
            const int ia = s_i[tid + o];
            if (a > s_v[tid] || (a == s_v[tid] && ia < s_i[tid])) {
                s_v[tid] = a;
                s_i[tid] = ia;
            }
        }
        __syncthreads();
    }
    const int p = s_i[0];
    const double pabs = s_v[0];
    if (p != kk)
        for (int j = tid; j < n; j += 1024) {
            const zc t = m[(size_t)kk * ld + j];
            m[(size_t)kk * ld + j] = m[(size_t)p * ld + j];
            m[(size_t)p * ld + j] = t;
        }
    __syncthreads();
    const zc pv = m[(size_t)kk * ld + kk];
    if (tid == 0) {
        w.piv[kk] = p;
        const double mx = fmax(w.stat[2], pabs);
        if (!(pabs > (double)n * 0x1p-52 * mx)) *w.status = 1;
        w.stat[0] += log(pabs);
        w.stat[1] += atan2(pv.y, pv.x) + (p != kk ? M_PI : 0.0);
        w.stat[2] = mx;
    }
    __syncthreads();
    const zc inv = zinv(pv);
    for (int j = tid; j < n; j += 1024) {
        zc *q = m + (size_t)kk * ld + j;
        *q = j == kk ? inv : zmul(*q, inv);
    }
    for (int i = tid; i < n; i += 1024) {
        if (i == kk) {
            w.fcol[i] = make_double2(0.0, 0.0);
        } else {
            w.fcol[i] = m[(size_t)i * ld + kk];
            m[(size_t)i * ld + kk] = make_double2(0.0, 0.0);
        }
    }
}

// Rows i != kk: row_i -= f_i row_kk.
__global__ void k_zgj_elim(ZWalkerDev w, int ld, int n, int kk) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= n || i == kk) return;
    const zc f = w.fcol[i];
    zc *q = w.bt + (size_t)i * ld + j;
    *q = zsub(*q, zmul(f, w.bt[(size_t)kk * ld + j]));
}

// Undo the row interchanges on the inverse's columns, last interchange first.
__global__ void k_zgj_unperm(ZWalkerDev w, int ld, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    zc *r = w.bt + (size_t)i * ld;
    for (int kk = n - 1; kk >= 0; --kk) {
        const int p = w.piv[kk];
        if (p != kk) {
            const zc t = r[kk];
            r[kk] = r[p];
            r[p] = t;
        }
    }
}

// The proposal row from mapped pinned host memory (read once over the host link).
__global__ void k_zrow_from_host(const double *src, zc *phi, int np) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < np) phi[c] = make_double2(src[2 * c], src[2 * c + 1]);
}

// out[i][j] = BT[j][i] (A^{-1}, n x n).
__global__ void k_zuntranspose(const zc *bt, zc *out, int n, int np) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j < n) out[(size_t)i * n + j] = bt[(size_t)j * np + i];
}

}  // namespace dsu

using namespace dsu;

struct dsu_zwalker {
    int n = 0, np = 0, K = 0, kp = 0, policy = 0;
    // real embedding of the stale rows for the matrix-core rank-k update
    // (k_zembed_v), for delays whose embedded width 2k is at most 256
    double *vh = nullptr;
    int kp2 = 0;
    int flush_mode = DSU_FLUSH_AUTO;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ZWalkerDev wd{};
    double *ratio_h = nullptr;
    double *row_stage = nullptr;            // mapped pinned host staging of a proposal row
    const double *row_stage_dev = nullptr;  // its device address
    zc *inv_tmp = nullptr;
    int k = 0, slots = 0;
    unsigned tag = 0;  // completion tag of the last look-ahead call
    std::vector<int> idx;
    bool has_prop = false;
    int prop_e = -1;
    double prop_re = 0.0, prop_im = 0.0;
    double logabs = 0.0, phase = 0.0;
};

static double wrap_phase(double p) {
    p = std::fmod(p, 2.0 * M_PI);
    if (p > M_PI) p -= 2.0 * M_PI;
    if (p <= -M_PI) p += 2.0 * M_PI;
    return p;
}

static void zwalker_free(dsu_zwalker *w) {
    for (void *p : {(void *)w->wd.bt, (void *)w->wd.u, (void *)w->wd.vg, (void *)w->wd.a, (void *)w->wd.phi,
                    (void *)w->wd.cinv, (void *)w->wd.dots, (void *)w->wd.t, (void *)w->wd.ratio, (void *)w->wd.idx,
                    (void *)w->wd.counter, (void *)w->wd.w, (void *)w->wd.fcol, (void *)w->wd.piv,
                    (void *)w->wd.stat, (void *)w->wd.status, (void *)w->inv_tmp, (void *)w->vh})
        dfree(p);
    if (w->ratio_h) (void)hipHostFree(w->ratio_h);
    if (w->row_stage) (void)hipHostFree(w->row_stage);
    if (w->own_stream && w->stream) (void)hipStreamDestroy(w->stream);
}

// Fresh inverse from A: BT = (A^T)^{-1} by in-place Gauss-Jordan on A^T.
static int zwalker_recompute(dsu_zwalker *w, double *logabs, double *phase) {
    const int n = w->n, np = w->np;
    hipLaunchKernelGGL(k_zload_t, dim3((np + 255) / 256, np), dim3(256), 0, w->stream, (const zc *)w->wd.a, w->wd.bt,
                       n, np);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(w->wd.stat, 0, 3 * sizeof(double), w->stream));
    HIPCHK(hipMemsetAsync(w->wd.status, 0, sizeof(int), w->stream));
    for (int kk = 0; kk < n; ++kk) {
        hipLaunchKernelGGL(k_zgj_pivot, dim3(1), dim3(1024), 0, w->stream, w->wd, np, n, kk);
        hipLaunchKernelGGL(k_zgj_elim, dim3((n + 255) / 256, n), dim3(256), 0, w->stream, w->wd, np, n, kk);
    }
    hipLaunchKernelGGL(k_zgj_unperm, dim3((n + 255) / 256), dim3(256), 0, w->stream, w->wd, np, n);
    HIPCHK(hipGetLastError());
    double st[3];
    int bad = 0;
    HIPCHK(hipMemcpyAsync(st, w->wd.stat, sizeof(st), hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(&bad, w->wd.status, sizeof(int), hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    if (bad) return fail(DSU_ESINGULAR, "Slater matrix is singular");
    *logabs = st[0];
    *phase = wrap_phase(st[1]);
    return DSU_OK;
}

static int zwalker_flush(dsu_zwalker *w) {
    const int k = w->k, np = w->np, kp = w->kp;
    if (k > 0) {
        // W = (BT U^T - E) C^{-T}, row by row (vector ALUs); then BT -= W Vg:
        // on the matrix cores through the real embedding when its width fits
        // (2k <= 256), else as a complex product on the vector ALUs
        hipLaunchKernelGGL(k_zflush_w, dim3(np / 4), dim3(kThreads), 0, w->stream, w->wd, np, k);
        HIPCHK(hipGetLastError());
        const bool mfma = w->vh && 2 * k <= w->kp2 &&
                          (w->flush_mode == DSU_FLUSH_MFMA || (w->flush_mode == DSU_FLUSH_AUTO && k > 2));
        if (mfma) {
            const int bx = np >= 256 ? np / 256 : 1;
            hipLaunchKernelGGL(k_zembed_v, dim3(bx, kpad(2 * k)), dim3(256), 0, w->stream, w->wd, w->vh, np, k);
            HIPCHK(hipGetLastError());
            HIPCHK(launch_gemm_sub(reinterpret_cast<const double *>(w->wd.w), 2 * w->wd.ldc, 2 * k, w->vh, 2 * np,
                                   reinterpret_cast<double *>(w->wd.bt), 2 * np, np, 2 * np, w->stream));
        } else {
            HIPCHK((zgemm<false, true>(w->wd.w, w->wd.ldc, w->wd.vg, np, w->wd.bt, np, np, np, k, w->stream)));
        }
    }
    w->k = 0;
    w->slots = 0;
    std::fill(w->idx.begin(), w->idx.end(), -1);
    return DSU_OK;
}

extern "C" int dsu_zwalker_set_flush_kernel(dsu_zwalker *w, int32_t mode) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (mode != DSU_FLUSH_AUTO && mode != DSU_FLUSH_VALU && mode != DSU_FLUSH_MFMA)
        return fail(DSU_EINVAL, "bad flush kernel %d", mode);
    w->flush_mode = mode;
    return DSU_OK;
}

extern "C" int dsu_zwalker_create(int32_t n, int32_t k_delay, int32_t policy, const double *slater_host,
                                  void *hip_stream, dsu_zwalker **out) {
    if (!out) return fail(DSU_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 16384) return fail(DSU_EINVAL, "n = %d out of range [1, 16384]", n);
    if (k_delay < 1 || k_delay > DSU_MAX_K) return fail(DSU_EINVAL, "k_delay = %d out of range [1, %d]", k_delay, DSU_MAX_K);
    if (policy != DSU_FLUSH_K_ACCEPTED && policy != DSU_FLUSH_K_PROPOSED) return fail(DSU_EINVAL, "bad policy %d", policy);
    if (!slater_host) return fail(DSU_EINVAL, "slater matrix is NULL");
    dsu_zwalker *w = new dsu_zwalker();
    w->n = n;
    w->np = round_up(n, 64);
    w->K = k_delay;
    w->kp = kpad(k_delay);
    w->policy = policy;
    const size_t np = w->np, kp = w->kp;
    int rc = DSU_OK;
#define TRY(x)              \
    do {                    \
        rc = (x);           \
        if (rc != DSU_OK) { \
            zwalker_free(w); \
            delete w;       \
            return rc;      \
        }                   \
    } while (0)
    TRY(make_stream(hip_stream, &w->stream, &w->own_stream));
    TRY(dalloc(&w->wd.bt, np * np));
    TRY(dalloc(&w->wd.u, kp * np));
    TRY(dalloc(&w->wd.vg, kp * np));
    TRY(dalloc(&w->wd.a, np * np));
    TRY(dalloc(&w->wd.phi, np));
    TRY(dalloc(&w->wd.cinv, kp * (kp + 1)));
    TRY(dalloc(&w->wd.dots, 1 + 2 * kp));
    TRY(dalloc(&w->wd.t, kp));
    TRY(dalloc(&w->wd.ratio, 1));
    TRY(dalloc(&w->wd.idx, kp));
    TRY(dalloc(&w->wd.counter, 1));
    TRY(dalloc(&w->wd.w, np * (kp + 1)));
    TRY(dalloc(&w->wd.fcol, np));
    TRY(dalloc(&w->wd.piv, np));
    TRY(dalloc(&w->wd.stat, 3));
    TRY(dalloc(&w->wd.status, 1));
    // embedded stale rows: 2 kp slots (capped at 256, the widest matrix-core update)
    w->kp2 = std::min<int>(256, kpad(std::min<int>(2 * (int)kp, 256)));
    TRY(dalloc(&w->vh, (size_t)w->kp2 * 2 * np));
    w->wd.ldc = (int)kp + 1;
    // coherent: the host watches the completion tag while the kernel runs
    if (hipHostMalloc((void **)&w->ratio_h, 3 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        TRY(fail(DSU_ENOMEM, "hipHostMalloc failed"));
    std::memset(w->ratio_h, 0, 3 * sizeof(double));
    if (hipHostMalloc((void **)&w->row_stage, 2 * np * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
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
    if (hipMemcpy2D(w->wd.a, np * sizeof(zc), slater_host, n * sizeof(zc), n * sizeof(zc), n, hipMemcpyHostToDevice) !=
        hipSuccess)
        TRY(fail(DSU_EDEVICE, "matrix upload failed"));
    TRY(zwalker_recompute(w, &w->logabs, &w->phase));
    w->idx.assign(w->kp, -1);
#undef TRY
    *out = w;
    return DSU_OK;
}

extern "C" int dsu_zwalker_destroy(dsu_zwalker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    (void)hipStreamSynchronize(w->stream);
    zwalker_free(w);
    delete w;
    return DSU_OK;
}

extern "C" int dsu_zpropose_ratio(dsu_zwalker *w, int32_t electron, const double *phi_host, double *ratio_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (electron < 0 || electron >= w->n) return fail(DSU_EINVAL, "electron %d out of range", electron);
    if (!phi_host) return fail(DSU_EINVAL, "row is NULL");
    // an electron may hold at most one pending move: apply the window first
    for (int j = 0; j < w->k; ++j)
        if (w->idx[j] == electron) {
            CHK(zwalker_flush(w));
            break;
        }
    // every earlier copy out of the staging buffer was followed on the stream by
    // a look-ahead kernel the host waited for, so the buffer is free
    std::memcpy(w->row_stage, phi_host, sizeof(double) * 2 * w->n);
    std::memset(w->row_stage + 2 * w->n, 0, sizeof(double) * 2 * (w->np - w->n));
    hipLaunchKernelGGL(k_zrow_from_host, dim3((w->np + 255) / 256), dim3(256), 0, w->stream, w->row_stage_dev, w->wd.phi,
                       w->np);
    HIPCHK(hipGetLastError());
    const unsigned tag = ++w->tag;
    hipLaunchKernelGGL(k_zpropose, dim3(2 * w->k + 1), dim3(kThreads), 0, w->stream, w->wd, w->np, w->k, electron,
                       tag);
    HIPCHK(hipGetLastError());
    // the kernel writes the tag to mapped memory after the ratio; after 2 s
    // without it the stream is synchronised instead (reports a failed kernel)
    const volatile double *h = w->ratio_h;
    {
        const auto t0 = std::chrono::steady_clock::now();
        bool seen = false;
        for (unsigned spin = 0; !seen; ++spin) {
            if (h[2] == (double)tag) seen = true;
            else if ((spin & 4095u) == 4095u && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) break;
        }
        if (!seen) {
            HIPCHK(hipStreamSynchronize(w->stream));
            if (h[2] != (double)tag) return fail(DSU_EDEVICE, "look-ahead kernel did not report");
        }
    }
    w->prop_re = h[0];
    w->prop_im = h[1];
    w->has_prop = true;
    w->prop_e = electron;
    if (ratio_out) {
        ratio_out[0] = w->prop_re;
        ratio_out[1] = w->prop_im;
    }
    return DSU_OK;
}

static int zwalker_slot_used(dsu_zwalker *w) {
    ++w->slots;
    const bool full = w->policy == DSU_FLUSH_K_ACCEPTED ? (w->k >= w->K) : (w->slots >= w->K);
    if (full) return zwalker_flush(w);
    return DSU_OK;
}

extern "C" int dsu_zaccept(dsu_zwalker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->has_prop) return fail(DSU_ESTATE, "no pending proposal");
    const double mod = std::hypot(w->prop_re, w->prop_im);
    if (!(mod > RatioFloor<double>::value) || !std::isfinite(mod))
        return fail(DSU_ESINGULAR, "ratio (%g, %g) cannot be accepted", w->prop_re, w->prop_im);
    hipLaunchKernelGGL(k_zaccept, dim3(1), dim3(kThreads), 0, w->stream, w->wd, w->np, w->k, w->prop_e);
    HIPCHK(hipGetLastError());
    w->idx[w->k] = w->prop_e;
    ++w->k;
    w->logabs += std::log(mod);
    w->phase = wrap_phase(w->phase + std::atan2(w->prop_im, w->prop_re));
    w->has_prop = false;
    return zwalker_slot_used(w);
}

extern "C" int dsu_zreject(dsu_zwalker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (!w->has_prop) return fail(DSU_ESTATE, "no pending proposal");
    w->has_prop = false;
    if (w->policy == DSU_FLUSH_K_PROPOSED) return zwalker_slot_used(w);
    return DSU_OK;
}

extern "C" int dsu_zflush(dsu_zwalker *w) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    return zwalker_flush(w);
}

extern "C" int dsu_zrecompute_inverse(dsu_zwalker *w, const double *slater_host_or_null, double *logabs_out,
                                      double *phase_out, double *drift_out) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (slater_host_or_null)
        HIPCHK(hipMemcpy2DAsync(w->wd.a, w->np * sizeof(zc), slater_host_or_null, w->n * sizeof(zc), w->n * sizeof(zc),
                                w->n, hipMemcpyHostToDevice, w->stream));
    double la, ph;
    CHK(zwalker_recompute(w, &la, &ph));
    if (drift_out) *drift_out = w->logabs - la;
    w->logabs = la;
    w->phase = ph;
    w->k = 0;
    w->slots = 0;
    w->has_prop = false;
    std::fill(w->idx.begin(), w->idx.end(), -1);
    if (logabs_out) *logabs_out = la;
    if (phase_out) *phase_out = ph;
    return DSU_OK;
}

extern "C" int dsu_zget_inverse(dsu_zwalker *w, double *out_host) {
    if (!w || !out_host) return fail(DSU_EINVAL, "NULL argument");
    CHK(zwalker_flush(w));
    if (!w->inv_tmp) CHK(dalloc(&w->inv_tmp, (size_t)w->n * w->n));
    hipLaunchKernelGGL(k_zuntranspose, dim3((w->n + 255) / 256, w->n), dim3(256), 0, w->stream, (const zc *)w->wd.bt,
                       w->inv_tmp, w->n, w->np);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out_host, w->inv_tmp, sizeof(zc) * w->n * w->n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    return DSU_OK;
}

extern "C" int dsu_zget_logdet(dsu_zwalker *w, double *logabs, double *phase) {
    if (!w) return fail(DSU_EINVAL, "walker is NULL");
    if (logabs) *logabs = w->logabs;
    if (phase) *phase = w->phase;
    return DSU_OK;
}

extern "C" int dsu_zwalker_pending(dsu_zwalker *w, int32_t *k_out) {
    if (!w || !k_out) return fail(DSU_EINVAL, "NULL argument");
    *k_out = w->k;
    return DSU_OK;
}
