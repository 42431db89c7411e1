// k_walker.hip -- kernels of the host-driven single-walker form.
//
// With k accepted moves pending (electrons e_1..e_k, new rows U, stale BT rows
// Vg) the ratio for moving electron e to the row phi is the look-ahead of
// Sec. II: by the generalised determinant lemma, eq. (3),
//     det(A_{k+1}) / det(A_k) = det(C_{k+1}) / det(C_k),
//     C_{k+1} = [[C_k, q], [p^T, r0]],  r0 = phi.BT[e],  p_j = phi.Vg[j],
//     q_j = U[j].BT[e],
// and the Schur complement gives R = r0 - p^T C_k^{-1} q.  C_k^{-1} is kept up
// to date by bordering when a move is accepted, so the look-ahead costs
// (2k+1) dot products of length n plus O(k^2) -- no explicit k x k
// determinants.
#include "walker.hpp"

namespace dsu {


// Sum NV values over the block; every thread gets the totals.
template <typename T, int NV>
__device__ __forceinline__ void block_sum_n(T (&v)[NV], T (*sbuf)[kThreads / 64]) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sbuf[i][wave] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        T s = T(0);
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sbuf[i][q];
        v[i] = s;
    }
}

// Look-ahead products of a set of x rows against one electron (Sec. II,
// eq. (3)).  R(x) = x.BT[e] - sum_j (x.Vg[j]) t_j with t = C_k^{-1} q is
// linear in x, so the ratio (x = phi) and its gradient with respect to the
// new position (x = d phi / d r_a, a = x, y, z) share q and t; so does the
// drift grad_e ln|det A| at the present position (x = gradient rows of the
// present row, whose own ratio is 1).
//   GR = 0: x = {phi};  GR = 1: x = {phi, dphi_x, dphi_y, dphi_z};
//   GR = 2: x = {dphi_x, dphi_y, dphi_z}, the present position's gradient:
//           results go to gdots and ratio_host[1..3] and leave the pending
//           proposal (dots, t, ratio) untouched.  If e itself holds pending
//           slot m, row e of the delayed matrix is U[m], and the lemma's
//           right-hand side becomes q - 1_m.
// Grid of 2k+1 blocks: block 0 -> x.BT[e], 1..k -> x.Vg[j], k+1..2k -> q.
// The last block to finish forms t and the results.
template <typename T, int GR>
__global__ __launch_bounds__(kThreads) void k_walker_propose(WalkerDev w, int np, int k, int e, int m, unsigned tag) {
    constexpr int NX = GR == 0 ? 1 : (GR == 1 ? 4 : 3);
    constexpr int X0 = GR == 1 ? 1 : 0;  // first gradient row
    __shared__ T sbuf[NX][kThreads / 64];
    __shared__ double dbuf[4][kThreads / 64];
    __shared__ int is_last;
    __shared__ double s_t[DSU_KMAX_LDS];
    const int b = blockIdx.x, tid = threadIdx.x;
    const T *bt = static_cast<const T *>(w.bt), *u = static_cast<const T *>(w.u), *vg = static_cast<const T *>(w.vg);
    const T *phi = static_cast<const T *>(w.phi), *dphi = static_cast<const T *>(w.dphi);
    const int ld = k + 1;
    if (b <= k) {
        const T *x[NX];
        if (GR != 2) x[0] = phi;
        if (GR != 0)
#pragma unroll
            for (int a = 0; a < 3; ++a) x[X0 + a] = dphi + (size_t)a * np;
        const T *y = b == 0 ? bt + (size_t)e * np : vg + (size_t)(b - 1) * np;
        T acc[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) acc[i] = T(0);
        for (int c = tid; c < np; c += kThreads) {
            const T yc = y[c];
#pragma unroll
            for (int i = 0; i < NX; ++i) acc[i] += x[i][c] * yc;
        }
        block_sum_n<T, NX>(acc, sbuf);
        if (tid == 0) {
            if (GR != 2) w.dots[b] = double(acc[0]);
            if (GR != 0)
#pragma unroll
                for (int a = 0; a < 3; ++a) w.gdots[a * ld + b] = double(acc[X0 + a]);
        }
    } else {
        const T *x = u + (size_t)(b - 1 - k) * np, *y = bt + (size_t)e * np;
        T acc[1] = {T(0)};
        for (int c = tid; c < np; c += kThreads) acc[0] += x[c] * y[c];
        block_sum_n<T, 1>(acc, sbuf);
        if (tid == 0) (GR == 2 ? w.gdots + 3 * ld : w.dots + 1 + k)[b - 1 - k] = double(acc[0]);
    }
    if (tid == 0) {
        __threadfence();
        is_last = atomicAdd(w.counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const double *q = GR == 2 ? w.gdots + 3 * ld : w.dots + 1 + k;
    for (int i = tid; i < k; i += kThreads) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += w.cinv[(size_t)i * w.ldc + j] * (q[j] - (j == m ? 1.0 : 0.0));
        s_t[i] = s;
        if (GR != 2) w.t[i] = s;
    }
    __syncthreads();
    constexpr int NO = GR == 0 ? 1 : (GR == 1 ? 4 : 3);  // ratio and / or three gradient components
    double part[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) part[o] = 0.0;
    for (int i = tid; i < k; i += kThreads) {
        if (GR != 2) part[0] += w.dots[1 + i] * s_t[i];
        if (GR != 0)
#pragma unroll
            for (int a = 0; a < 3; ++a) part[X0 + a] += w.gdots[a * ld + 1 + i] * s_t[i];
    }
    block_sum_n<double, NO>(part, dbuf);
    if (tid == 0) {
        if (GR != 2) {
            const double r = w.dots[0] - part[0];
            w.ratio[0] = r;
            w.ratio_host[0] = r;
        }
        if (GR != 0)
#pragma unroll
            for (int a = 0; a < 3; ++a) w.ratio_host[1 + a] = w.gdots[a * ld] - part[X0 + a];
        *w.counter = 0u;
        __threadfence_system();  // results reach host memory before the tag
        w.ratio_host[4] = (double)tag;
    }
}

// One block: border C_k^{-1} to C_{k+1}^{-1} with the accepted proposal and
// append it to the delayed buffer (U row, stale BT row, A row, electron).
//   t = C^{-1} q,  b^T = p^T C^{-1},  R = r0 - p.t
//   C_{k+1}^{-1} = [[C^{-1} + t b^T / R, -t / R], [-b^T / R, 1 / R]]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_walker_accept(WalkerDev w, int np, int k, int e) {
    __shared__ double s_b[DSU_KMAX_LDS];
    __shared__ double s_t[DSU_KMAX_LDS];
    const int tid = threadIdx.x;
    const double r = w.ratio[0];
    const double rinv = 1.0 / r;
    for (int j = tid; j < k; j += kThreads) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += w.dots[1 + i] * w.cinv[(size_t)i * w.ldc + j];
        s_b[j] = s;
        s_t[j] = w.t[j];
    }
    __syncthreads();
    const int k1 = k + 1;
    for (int v = tid; v < k1 * k1; v += kThreads) {
        const int i = v / k1, j = v % k1;
        double *c = w.cinv + (size_t)i * w.ldc + j;
        if (i < k && j < k) *c += s_t[i] * s_b[j] * rinv;
        else if (i < k) *c = -s_t[i] * rinv;
        else if (j < k) *c = -s_b[j] * rinv;
        else *c = rinv;
    }
    T *u = static_cast<T *>(w.u), *vg = static_cast<T *>(w.vg);
    const T *bt = static_cast<const T *>(w.bt), *phi = static_cast<const T *>(w.phi);
    for (int c = tid; c < np; c += kThreads) {
        u[(size_t)k * np + c] = phi[c];
        vg[(size_t)k * np + c] = bt[(size_t)e * np + c];
        w.a[(size_t)e * np + c] = w.phi64[c];
    }
    if (tid == 0) w.idx[k] = e;
}

template <typename T>
hipError_t launch_walker_propose(WalkerDev *wd, int n, int np, int k, int e, int grad_mode, int m, unsigned tag,
                                 hipStream_t s) {
    (void)n;
    const dim3 g(2 * k + 1), b(kThreads);
    if (grad_mode == 0) hipLaunchKernelGGL((k_walker_propose<T, 0>), g, b, 0, s, *wd, np, k, e, -1, tag);
    else if (grad_mode == 1) hipLaunchKernelGGL((k_walker_propose<T, 1>), g, b, 0, s, *wd, np, k, e, -1, tag);
    else hipLaunchKernelGGL((k_walker_propose<T, 2>), g, b, 0, s, *wd, np, k, e, m, tag);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_walker_accept(WalkerDev *wd, int n, int np, int k, int kp, int e, hipStream_t s) {
    (void)n;
    (void)kp;
    hipLaunchKernelGGL((k_walker_accept<T>), dim3(1), dim3(kThreads), 0, s, *wd, np, k, e);
    return hipGetLastError();
}
template hipError_t launch_walker_propose<float>(WalkerDev *, int, int, int, int, int, int, unsigned, hipStream_t);
template hipError_t launch_walker_propose<double>(WalkerDev *, int, int, int, int, int, int, unsigned, hipStream_t);
template hipError_t launch_walker_accept<float>(WalkerDev *, int, int, int, int, int, hipStream_t);
template hipError_t launch_walker_accept<double>(WalkerDev *, int, int, int, int, int, hipStream_t);

// ------------------------------------------------------------------------
// Multideterminant expansion on a single reference (FP64 walker).
// Psi = sum_I c_I det(A_I): A_I is A with occupied columns J_I replaced by
// virtual columns V_I, and det(A_I) / det(A) = det S_I, S_I = T[J_I][V_I]
// with the table T = A^{-1} V.  Moving electron e (rows phi, vphi) changes T
// by a rank-1 term: T' = T + c x^T, c = A^{-1}[:, e] (the delayed inverse's
// column, i.e. BT[e] corrected by the pending moves as in the look-ahead),
// x = (vphi - phi T) / R with R the reference ratio.
// ------------------------------------------------------------------------

// T[j][v] = sum_i BT[i][j] V[i][v], j < n (rows past n stay zero).
__global__ void k_md_table(const double *bt, MdDev md, int n, int np) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += bt[(size_t)i * np + j] * md.v[(size_t)i * md.m + v];
    md.t[(size_t)j * md.m + v] = s;
}

// c[j] = BT[e][j] - sum_l t_l Vg[l][j]  (t from the look-ahead kernel).
__global__ void k_md_c(WalkerDev w, MdDev md, int np, int k, int e) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const double *bt = static_cast<const double *>(w.bt), *vg = static_cast<const double *>(w.vg);
    double s = bt[(size_t)e * np + j];
    for (int l = 0; l < k; ++l) s -= w.t[l] * vg[(size_t)l * np + j];
    md.c[j] = s;
}

// x[v] = (vphi[v] - sum_j phi_j T[j][v]) / R, one workgroup per v.
__global__ __launch_bounds__(kThreads) void k_md_x(WalkerDev w, MdDev md, int n) {
    __shared__ double sbuf[1][kThreads / 64];
    const int v = blockIdx.x;
    double acc[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += kThreads) acc[0] += w.phi64[j] * md.t[(size_t)j * md.m + v];
    block_sum_n<double, 1>(acc, sbuf);
    if (threadIdx.x == 0) md.x[v] = (md.vphi[v] - acc[0]) / w.ratio[0];
}

// det of the order x order matrix S[a][b] = T[J_a][V_b] + (with_x ? c[J_a] x[V_b] : 0),
// Gaussian elimination with partial pivoting.
__device__ double md_det(const MdDev &md, int d, bool with_x) {
    const int o = md.order[d];
    double s[4][4];
    for (int a = 0; a < o; ++a)
        for (int b = 0; b < o; ++b) {
            const int j = md.occ[4 * d + a], v = md.virt[4 * d + b];
            s[a][b] = md.t[(size_t)j * md.m + v] + (with_x ? md.c[j] * md.x[v] : 0.0);
        }
    double det = 1.0;
    for (int p = 0; p < o; ++p) {
        int r = p;
        for (int a = p + 1; a < o; ++a)
            if (fabs(s[a][p]) > fabs(s[r][p])) r = a;
        if (s[r][p] == 0.0) return 0.0;
        if (r != p) {
            for (int b = 0; b < o; ++b) {
                const double tmp = s[p][b];
                s[p][b] = s[r][b];
                s[r][b] = tmp;
            }
            det = -det;
        }
        det *= s[p][p];
        for (int a = p + 1; a < o; ++a) {
            const double f = s[a][p] / s[p][p];
            for (int b = p + 1; b < o; ++b) s[a][b] -= f * s[p][b];
        }
    }
    return det;
}

// One workgroup: Q = sum_I c_I det S_I (mode 0: the proposal, with the
// rank-1 term; mode 1: the present table).
__global__ __launch_bounds__(kThreads) void k_md_sum(WalkerDev w, MdDev md, int mode, unsigned tag) {
    __shared__ double sbuf[1][kThreads / 64];
    double acc[1] = {0.0};
    for (int d = threadIdx.x; d < md.ndet; d += kThreads) acc[0] += md.coef[d] * md_det(md, d, mode == 0);
    block_sum_n<double, 1>(acc, sbuf);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            const double r = w.ratio[0];
            md.q[0] = acc[0];
            w.ratio_host[0] = r * acc[0] / md.q[1];
            w.ratio_host[1] = r;
        } else {
            md.q[1] = acc[0];
        }
        w.ratio_host[2] = acc[0];
        __threadfence_system();
        w.ratio_host[4] = (double)tag;
    }
}

// T += c x^T; V[e] = vphi; Q = Q'.
__global__ void k_md_accept(MdDev md, int n, int e) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
    if (j < n) md.t[(size_t)j * md.m + v] += md.c[j] * md.x[v];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        md.v[(size_t)e * md.m + v] = md.vphi[v];
        if (v == 0) md.q[1] = md.q[0];
    }
}

hipError_t launch_md_table(const WalkerDev *wd, const MdDev *md, int n, int np, hipStream_t s) {
    hipLaunchKernelGGL(k_md_table, dim3((n + 255) / 256, md->m), dim3(256), 0, s, (const double *)wd->bt, *md, n, np);
    return hipGetLastError();
}

hipError_t launch_md_propose(const WalkerDev *wd, const MdDev *md, int n, int np, int k, int e, unsigned tag,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_md_c, dim3((np + 255) / 256), dim3(256), 0, s, *wd, *md, np, k, e);
    hipLaunchKernelGGL(k_md_x, dim3(md->m), dim3(kThreads), 0, s, *wd, *md, n);
    hipLaunchKernelGGL(k_md_sum, dim3(1), dim3(kThreads), 0, s, *wd, *md, 0, tag);
    return hipGetLastError();
}

hipError_t launch_md_init(const WalkerDev *wd, const MdDev *md, unsigned tag, hipStream_t s) {
    hipLaunchKernelGGL(k_md_sum, dim3(1), dim3(kThreads), 0, s, *wd, *md, 1, tag);
    return hipGetLastError();
}

hipError_t launch_md_accept(const MdDev *md, int n, int np, int e, hipStream_t s) {
    (void)np;
    hipLaunchKernelGGL(k_md_accept, dim3((n + 255) / 256, md->m), dim3(256), 0, s, *md, n, e);
    return hipGetLastError();
}

// Row conversion: FP64 -> T (is_float = 1: float, else copy) into dst,
// zero padded to np; or, with is_float = 2, float src -> FP64 dst.
__global__ void k_row_convert(const void *src, void *dst, int mode, int n, int np) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    if (mode == 1) static_cast<float *>(dst)[c] = c < n ? float(static_cast<const double *>(src)[c]) : 0.0f;
    else if (mode == 2) static_cast<double *>(dst)[c] = c < n ? double(static_cast<const float *>(src)[c]) : 0.0;
    else static_cast<double *>(dst)[c] = c < n ? static_cast<const double *>(src)[c] : 0.0;
}

// Rows staged by the host in mapped pinned memory, read once over the host
// link: dst64[c] = src[c] and, when dst32 is given, dst32[c] = float(src[c]),
// for c < count (padding already zero in the staging rows).
__global__ void k_rows_from_host(const double *src, double *dst64, float *dst32, int count) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    const double v = src[c];
    dst64[c] = v;
    if (dst32) dst32[c] = float(v);
}

hipError_t launch_rows_from_host(const double *src_mapped, double *dst64, float *dst32, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_from_host, dim3((count + 255) / 256), dim3(256), 0, s, src_mapped, dst64, dst32, count);
    return hipGetLastError();
}

hipError_t launch_row_to(const double *src, void *dst, int mode, int n, int np, hipStream_t s) {
    hipLaunchKernelGGL(k_row_convert, dim3((np + 255) / 256), dim3(256), 0, s, (const void *)src, dst, mode, n, np);
    return hipGetLastError();
}

}  // namespace dsu
