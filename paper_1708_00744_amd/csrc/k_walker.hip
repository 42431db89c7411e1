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
#include "dsu_internal.hpp"

namespace dsu {


template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sbuf) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[wave] = v;
    __syncthreads();
    T s = T(0);
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sbuf[q];
    return s;
}

// Grid of 2k+1 blocks: block 0 -> r0, 1..k -> p, k+1..2k -> q.  The last
// block to finish forms t = C_k^{-1} q and R = r0 - p.t.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_walker_propose(WalkerDev w, int np, int k, int e) {
    __shared__ T sbuf[kThreads / 64];
    __shared__ double dbuf[kThreads / 64];
    __shared__ int is_last;
    __shared__ double s_t[DSU_KMAX_LDS];
    const int b = blockIdx.x, tid = threadIdx.x;
    const T *bt = static_cast<const T *>(w.bt), *u = static_cast<const T *>(w.u), *vg = static_cast<const T *>(w.vg);
    const T *phi = static_cast<const T *>(w.phi);
    const T *x, *y;
    if (b == 0) { x = phi; y = bt + (size_t)e * np; }
    else if (b <= k) { x = phi; y = vg + (size_t)(b - 1) * np; }
    else { x = u + (size_t)(b - 1 - k) * np; y = bt + (size_t)e * np; }
    T acc = T(0);
    for (int c = tid; c < np; c += kThreads) acc += x[c] * y[c];
    acc = block_sum(acc, sbuf);
    if (tid == 0) {
        w.dots[b] = double(acc);
        __threadfence();
        is_last = atomicAdd(w.counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    for (int i = tid; i < k; i += kThreads) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += w.cinv[(size_t)i * w.ldc + j] * w.dots[1 + k + j];
        s_t[i] = s;
        w.t[i] = s;
    }
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < k; i += kThreads) part += w.dots[1 + i] * s_t[i];
    part = block_sum(part, dbuf);
    if (tid == 0) {
        const double r = w.dots[0] - part;
        w.ratio[0] = r;
        *w.ratio_host = r;
        *w.counter = 0u;
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
hipError_t launch_walker_propose(WalkerDev *wd, int n, int np, int k, int e, hipStream_t s) {
    (void)n;
    hipLaunchKernelGGL((k_walker_propose<T>), dim3(2 * k + 1), dim3(kThreads), 0, s, *wd, np, k, e);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_walker_accept(WalkerDev *wd, int n, int np, int k, int kp, int e, hipStream_t s) {
    (void)n;
    (void)kp;
    hipLaunchKernelGGL((k_walker_accept<T>), dim3(1), dim3(kThreads), 0, s, *wd, np, k, e);
    return hipGetLastError();
}
template hipError_t launch_walker_propose<float>(WalkerDev *, int, int, int, int, hipStream_t);
template hipError_t launch_walker_propose<double>(WalkerDev *, int, int, int, int, hipStream_t);
template hipError_t launch_walker_accept<float>(WalkerDev *, int, int, int, int, int, hipStream_t);
template hipError_t launch_walker_accept<double>(WalkerDev *, int, int, int, int, int, hipStream_t);

// Row conversion: FP64 -> T (is_float = 1: float, else copy) into dst,
// zero padded to np; or, with is_float = 2, float src -> FP64 dst.
__global__ void k_row_convert(const void *src, void *dst, int mode, int n, int np) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    if (mode == 1) static_cast<float *>(dst)[c] = c < n ? float(static_cast<const double *>(src)[c]) : 0.0f;
    else if (mode == 2) static_cast<double *>(dst)[c] = c < n ? double(static_cast<const float *>(src)[c]) : 0.0;
    else static_cast<double *>(dst)[c] = c < n ? static_cast<const double *>(src)[c] : 0.0;
}

hipError_t launch_row_to(const double *src, void *dst, int mode, int n, int np, hipStream_t s) {
    hipLaunchKernelGGL(k_row_convert, dim3((np + 255) / 256), dim3(256), 0, s, (const void *)src, dst, mode, n, np);
    return hipGetLastError();
}

}  // namespace dsu
