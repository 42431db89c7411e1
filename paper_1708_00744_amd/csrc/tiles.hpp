// tiles.hpp -- matrix-core (MFMA 16x16x4) building blocks shared by the
// flush, the Gauss-Jordan trailing update and the window look-ahead product.
// A workgroup is 4 waves; wave w owns rows 16w..16w+15 of a 64-row block.
#pragma once
#include "dsu_internal.hpp"

#include <type_traits>
#include <utility>

namespace dsu {

// Calls f(integral_constant<int, I>) for I = 0, 1, ... in order (compile-time
// unrolling that keeps register-array indices fixed).
template <int... I, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F &&f) {
    (f(std::integral_constant<int, I>{}), ...);
}

template <typename T> struct alignas(16) V16 { T v[16 / sizeof(T)]; };

// 16-byte vector registers, and global-memory pointers: pointers read from a
// descriptor are generic (flat) to the compiler; flat accesses also count
// against the LDS wait counter, which would serialise prefetches with LDS use.
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
#define DSU_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ DSU_GLOBAL T *gmem(T *p) { return (DSU_GLOBAL T *)p; }

// The hardware hands consecutive workgroups to the 8 XCDs in turn; renumber
// them so that each XCD (own L2) works on a contiguous range of logical blocks,
// i.e. on the same determinant's U and Vg.
__device__ __forceinline__ int xcd_remap(int b, int g) {
    const int full = g & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Phase 1: acc = rows[0:64, c_begin:c_end] * U[0:KP, c_begin:c_end]^T
// Wave w owns output rows 16w..16w+15, all KP columns (KP/16 tiles).
// rows beyond rows_valid read as zero.  U chunks are staged in LDS.
// ---------------------------------------------------------------------------
template <typename T, int KP>
__device__ __forceinline__ void rowblock_times_ut(const T *__restrict__ rows, int ld, int rows_valid,
                                                  const T *__restrict__ U, int ldu, int c_begin, int c_end,
                                                  T *lds, typename Mma<T>::acc_t (&acc)[KP / 16]) {
    constexpr int CW = 128 / sizeof(T);      // chunk: 128 bytes of every row
    constexpr int E = CW / 4;                // elements per lane per row
    constexpr int VEC = 16 / sizeof(T);
    constexpr int LDU = CW + VEC;            // +16 B row pad (bank spread)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int arow = wave * 16 + (lane & 15);
    const bool avalid = arow < rows_valid;
    const T *ap = rows + (size_t)(avalid ? arow : 0) * ld + E * (lane >> 4);
    for (int t = 0; t < KP / 16; ++t) acc[t] = typename Mma<T>::acc_t{0, 0, 0, 0};

    for (int c0 = c_begin; c0 < c_end; c0 += CW) {
        for (int v = tid; v < KP * (CW / VEC); v += kThreads) {
            const int r = v / (CW / VEC), cc = (v % (CW / VEC)) * VEC;
            *reinterpret_cast<V16<T> *>(lds + r * LDU + cc) =
                *reinterpret_cast<const V16<T> *>(U + (size_t)r * ldu + c0 + cc);
        }
        T a[E];
        if (avalid) {
#pragma unroll
            for (int h = 0; h < E / VEC; ++h) {
                V16<T> x = *reinterpret_cast<const V16<T> *>(ap + c0 + h * VEC);
#pragma unroll
                for (int q = 0; q < VEC; ++q) a[h * VEC + q] = x.v[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) a[q] = T(0);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < KP / 16; ++t) {
            const T *bp = lds + (16 * t + (lane & 15)) * LDU + E * (lane >> 4);
            T b[E];
#pragma unroll
            for (int h = 0; h < E / VEC; ++h) {
                V16<T> x = *reinterpret_cast<const V16<T> *>(bp + h * VEC);
#pragma unroll
                for (int q = 0; q < VEC; ++q) b[h * VEC + q] = x.v[q];
            }
#pragma unroll
            for (int s = 0; s < E; ++s) acc[t] = Mma<T>::mma(a[s], b[s], acc[t]);
        }
        __syncthreads();
    }
}

// Column chunk of phase 3: keep the staged V chunk at <= 32 KB.
template <typename T, int KP> struct Phase3Cfg {
    static constexpr int bytes_row = 32768 / KP;               // per V row
    static constexpr int raw = bytes_row / (int)sizeof(T);
    static constexpr int CW = raw >= 64 ? 64 : (raw >= 32 ? 32 : 16);
    static constexpr int LDV = CW + 64 / (int)sizeof(T);        // +64 B pad
};

// ---------------------------------------------------------------------------
// Phase 3: rows[0:64, 0:ncols] += Wneg[0:64, 0:KP] * V[0:KP, 0:ncols]
// wa[s] holds this lane's A fragments of Wneg: Wneg[16w + lane%16][4s + lane/16].
// ---------------------------------------------------------------------------
template <typename T, int KP>
__device__ __forceinline__ void rowblock_plus_wv(T *__restrict__ rows, int ld, int ncols, const T *__restrict__ V,
                                                 int ldv, const T (&wa)[KP / 4], T *lds) {
    typedef Phase3Cfg<T, KP> C;
    constexpr int CW = C::CW, LDV = C::LDV, VEC = 16 / sizeof(T);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int RS = Mma<T>::row_step;
    T *rp = rows + (size_t)(wave * 16 + Mma<T>::row0(lane)) * ld + (lane & 15);
    for (int c0 = 0; c0 < ncols; c0 += CW) {
        for (int v = tid; v < KP * (CW / VEC); v += kThreads) {
            const int r = v / (CW / VEC), cc = (v % (CW / VEC)) * VEC;
            *reinterpret_cast<V16<T> *>(lds + r * LDV + cc) =
                *reinterpret_cast<const V16<T> *>(V + (size_t)r * ldv + c0 + cc);
        }
        typename Mma<T>::acc_t acc[CW / 16];
#pragma unroll
        for (int t = 0; t < CW / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[t][i] = rp[(size_t)(i * RS) * ld + c0 + 16 * t];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < KP / 4; ++s) {
            const T *bp = lds + (4 * s + (lane >> 4)) * LDV + (lane & 15);
#pragma unroll
            for (int t = 0; t < CW / 16; ++t) acc[t] = Mma<T>::mma(wa[s], bp[16 * t], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < CW / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) rp[(size_t)(i * RS) * ld + c0 + 16 * t] = acc[t][i];
        __syncthreads();
    }
}


// W = Y' C^T for the block's 64 rows: Y' (64 x KP) in LDS with pitch ldy,
// C = inverse of eq. (3)'s C matrix, FP64 in global memory (pitch ldc), taken
// as zero beyond kslots.  C is staged in LDS chunk by chunk (converted to T
// and zero padded), so the product is a branch-free loop over LDS operands.
template <typename T, int KP> struct WCfg {
    // chunk budget: 32 KB, or 16 KB when the Y' block itself is large (FP64, K = 256)
    static constexpr int budget = KP * (int)sizeof(T) >= 2048 ? 16384 : 32768;
    static constexpr int JC = (KP * 64 * (int)sizeof(T) <= budget) ? 64
                              : (KP * 32 * (int)sizeof(T) <= budget ? 32 : (KP * 16 * (int)sizeof(T) <= budget ? 16 : 8));
    static constexpr int JCE = JC < KP ? JC : KP;
    static constexpr int LDC = JCE + 16 / (int)sizeof(T);
    static constexpr int elems = KP * LDC;
};

template <typename T, int KP>
__device__ __forceinline__ void w_from_y(const T *ylds, int ldy, const double *__restrict__ cinv, int ldc, int kslots,
                                         T *cbuf, typename Mma<T>::acc_t (&wacc)[KP / 16]) {
    typedef WCfg<T, KP> C;
    constexpr int JC = C::JCE, LDC = C::LDC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int t = 0; t < KP / 16; ++t) wacc[t] = typename Mma<T>::acc_t{0, 0, 0, 0};
    // loads issued in batches of up to 8 before their stores (not one wait per element)
    constexpr int NL = (KP * JC + kThreads - 1) / kThreads;
    constexpr int NB = NL < 8 ? NL : 8;
    DSU_GLOBAL const double *cg = (DSU_GLOBAL const double *)cinv;
    for (int j0 = 0; j0 < KP; j0 += JC) {
#pragma unroll
        for (int q0 = 0; q0 < NL; q0 += NB) {
            double cv[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int v = tid + (q0 + q) * kThreads, l = v / JC, jj = v % JC, j = j0 + jj;
                const bool in = v < KP * JC && l < kslots && j < kslots;
                cv[q] = cg[in ? (size_t)l * ldc + j : 0];
                if (!in) cv[q] = 0.0;
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int v = tid + (q0 + q) * kThreads, l = v / JC, jj = v % JC;
                if (v < KP * JC) cbuf[l * LDC + jj] = T(cv[q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < JC / 4; ++s) {
            const T a = ylds[(16 * wave + (lane & 15)) * ldy + j0 + 4 * s + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < KP / 16; ++t)
                wacc[t] = Mma<T>::mma(a, cbuf[(16 * t + (lane & 15)) * LDC + 4 * s + (lane >> 4)], wacc[t]);
        }
        __syncthreads();
    }
}

}  // namespace dsu
