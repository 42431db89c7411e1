// k_stream.hip -- the streaming Woodbury flush of the batched form (eq. (4)),
// fused with the next window's look-ahead products (eq. (3)).
#include "dsu_internal.hpp"
#include "tiles.hpp"

namespace dsu {

// One pass over BT per window.  Per 64-row block:
//   W    = (y - E) C^{-T}          (from this block's rows of y, on matrix cores)
//   for each column chunk of BT (on chip once):
//     BT  -= W Vg[cur]              (eq. (4), row-local)
//     y   += BT_new U[nxt]^T        (look-ahead products of the next window)
//     rows of the next window -> Vg[nxt]
// In the streaming pass the BT tile is kept transposed in the matrix cores:
// D' = V^T (-W)^T, so that a lane's four results are one BT row's four
// consecutive columns 16t + 4*(lane/16) + i (one vector load and store), and
// the same registers are directly the A operand of the next window's product
// BT_new U_next^T (its contraction order is free).  For the FP64 result layout
// (rows lane/16 + 4i) the V operand of tile row m is taken from column
// tcol(m) to give the same column set.
template <typename T> __device__ __forceinline__ int tcol(int m) {
    return Mma<T>::row_step == 1 ? m : 4 * (m & 3) + (m >> 2);
}

template <typename T, int KP> struct StreamCfg {
    static constexpr int CW = Phase3Cfg<T, KP>::CW;
    static constexpr int VEC = 16 / (int)sizeof(T);
    static constexpr int LDVT = KP + VEC;  // V chunk stored transposed: [column][slot]
    static constexpr int LDU = CW + VEC;
    static constexpr int LDY = KP + VEC;
    static constexpr int NV = KP * (CW / VEC) / kThreads;  // staged vectors per thread and operand
    static constexpr int buf = CW * LDVT + KP * LDU;  // one chunk's V^T and U
    static constexpr int chunk = 2 * buf;                // double-buffered
    static constexpr int wpart = 64 * LDY + WCfg<T, KP>::elems;
    static constexpr int elems = chunk > wpart ? chunk : wpart;
    static_assert(NV >= 1 && NV * kThreads == KP * (CW / VEC), "staging split");
};

template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_flush_stream(const DetDesc<T> *__restrict__ descs, int np, int nblk,
                                                           int kp, int kslots, int cur, int has_next, int e0n,
                                                           int kwn) {
    typedef StreamCfg<T, KP> C;
    typedef typename Mma<T>::acc_t acc_t;
    typedef typename Vec16<T>::type vec_t;
    constexpr int CW = C::CW, LDVT = C::LDVT, LDU = C::LDU, LDY = C::LDY, VEC = C::VEC, NV = C::NV, NT = CW / 16;
    constexpr int RS = Mma<T>::row_step, HV = 4 / VEC;  // 16-byte vectors per 4-element tile column group
    constexpr int KQ = KP / 4;                          // slots per lane group in the V^T W^T product
    __shared__ __attribute__((aligned(16))) T lds[C::elems];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * kRowBlock;
    const DetDesc<T> dd = descs[d];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    DSU_GLOBAL const T *vcur = gmem<const T>(cur ? dd.vg2 : dd.vg);
    DSU_GLOBAL const T *unext = gmem<const T>(cur ? dd.u : dd.u2);
    DSU_GLOBAL T *y = gmem(dd.y);

    // W = (y - E) C^{-T} for this block's 64 rows
    {
        // loads in batches of 8 before their stores
        constexpr int NYL = 64 * KP / kThreads, NB = NYL < 8 ? NYL : 8;
#pragma unroll
        for (int q0 = 0; q0 < NYL; q0 += NB) {
            T yv[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int v = tid + (q0 + q) * kThreads, i = v / KP, j = v % KP;
                yv[q] = y[(size_t)(r0 + i) * kp + j];
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int v = tid + (q0 + q) * kThreads, i = v / KP, j = v % KP;
                lds[i * LDY + j] = yv[q];
            }
        }
    }
    __syncthreads();
    for (int j = tid; j < kslots; j += kThreads) {
        const int e = dd.idx[j];
        if (e >= r0 && e < r0 + kRowBlock) lds[(e - r0) * LDY + j] -= T(1);
    }
    __syncthreads();
    T wa[KP / 4];
    {
        acc_t wacc[KP / 16];
        w_from_y<T, KP>(lds, LDY, dd.cfl, kp, kslots, lds + 64 * LDY, wacc);
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lds[(16 * wave + Mma<T>::row0(lane) + i * RS) * LDY + 16 * t + (lane & 15)] = wacc[t][i];
        __syncthreads();
        // B operand of the V^T W^T product; its contraction runs over slot
        // (lane/16)*KQ + s so that a lane's V operands are contiguous in Vt
#pragma unroll
        for (int s = 0; s < KQ; ++s) wa[s] = -lds[(16 * wave + (lane & 15)) * LDY + (lane >> 4) * KQ + s];
        __syncthreads();
    }

    // this lane's BT row, and its first column in each 16-column tile
    const int lrow = 16 * wave + (lane & 15);
    DSU_GLOBAL T *rp = gmem(dd.bt) + (size_t)(r0 + lrow) * np + 4 * (lane >> 4);
    const int g = r0 + lrow - e0n;
    const bool wv = has_next && g >= 0 && g < kwn;
    DSU_GLOBAL T *vp = gmem(cur ? dd.vg : dd.vg2) + (size_t)(wv ? g : 0) * np + 4 * (lane >> 4);
    // staging of V and U: this thread's 16-byte pieces (row r, column cc of a chunk)
    int goff[NV], voff[NV], uoff[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int v = tid + q * kThreads, r = v / (CW / VEC), cc = (v % (CW / VEC)) * VEC;
        goff[q] = r * np + cc;
        voff[q] = cc * LDVT + r;
        uoff[q] = r * LDU + cc;
    }
    // chunk c's V^T and U sit in LDS buffer c & 1; chunk c+1's are loaded into
    // registers while chunk c's products run, then written to the other buffer:
    // one barrier per chunk
    vec_t sv[NV], su[NV], nx[NT * HV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        sv[q] = *(DSU_GLOBAL const vec_t *)(vcur + goff[q]);
        if (has_next) su[q] = *(DSU_GLOBAL const vec_t *)(unext + goff[q]);
    }
#pragma unroll
    for (int h = 0; h < NT * HV; ++h) nx[h] = *(DSU_GLOBAL const vec_t *)(rp + (h / HV) * 16 + (h % HV) * VEC);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[voff[q] + e * LDVT] = sv[q][e];
        if (has_next) *reinterpret_cast<vec_t *>(lds + CW * LDVT + uoff[q]) = su[q];
    }
    __syncthreads();

    acc_t accy[KP / 16];
#pragma unroll
    for (int t = 0; t < KP / 16; ++t) accy[t] = acc_t{0, 0, 0, 0};
    int cb = 0;  // current buffer
    for (int c0 = 0; c0 < np; c0 += CW, cb ^= 1) {
        const T *Vt = lds + cb * C::buf;
        const T *Us = Vt + CW * LDVT;
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[t][i] = nx[t * HV + i / VEC][i % VEC];
        const int c1 = c0 + CW;
        if (c1 < np) {  // next chunk's loads stay in flight during this chunk's products
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                sv[q] = *(DSU_GLOBAL const vec_t *)(vcur + goff[q] + c1);
                if (has_next) su[q] = *(DSU_GLOBAL const vec_t *)(unext + goff[q] + c1);
            }
#pragma unroll
            for (int h = 0; h < NT * HV; ++h)
                nx[h] = *(DSU_GLOBAL const vec_t *)(rp + c1 + (h / HV) * 16 + (h % HV) * VEC);
        }
        const T *ap = Vt + tcol<T>(lane & 15) * LDVT + (lane >> 4) * KQ;
#pragma unroll
        for (int j = 0; j < KQ / VEC; ++j) {
            vec_t a[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[t] = *reinterpret_cast<const vec_t *>(ap + 16 * t * LDVT + j * VEC);
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = Mma<T>::mma(a[t][e], wa[j * VEC + e], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                vec_t o;
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = acc[t][h * VEC + e];
                *(DSU_GLOBAL vec_t *)(rp + c0 + 16 * t + h * VEC) = o;
                if (wv) *(DSU_GLOBAL vec_t *)(vp + c0 + 16 * t + h * VEC) = o;
            }
        if (has_next) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                vec_t ub[KP / 16][HV];
#pragma unroll
                for (int jt = 0; jt < KP / 16; ++jt)
#pragma unroll
                    for (int h = 0; h < HV; ++h)
                        ub[jt][h] = *reinterpret_cast<const vec_t *>(Us + (16 * jt + (lane & 15)) * LDU + 16 * t +
                                                                     4 * (lane >> 4) + h * VEC);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jt = 0; jt < KP / 16; ++jt)
                        accy[jt] = Mma<T>::mma(acc[t][i], ub[jt][i / VEC][i % VEC], accy[jt]);
            }
        }
        if (c1 < np) {
            // the other buffer was last read before the previous barrier
            T *nb = lds + (cb ^ 1) * C::buf;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) nb[voff[q] + e * LDVT] = sv[q][e];
                if (has_next) *reinterpret_cast<vec_t *>(nb + CW * LDVT + uoff[q]) = su[q];
            }
        }
        __syncthreads();
    }
    if (has_next) {
        const int drow = 16 * wave + Mma<T>::row0(lane);
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) y[(size_t)(r0 + drow + i * RS) * kp + 16 * t + (lane & 15)] = accy[t][i];
    }
}

// FP32 variant with 32 x 32 x 2 matrix-core tiles (K = 32 and 64): 128 rows
// per workgroup, 32 per wave.  Each operand fragment read from LDS now feeds
// twice the flops.  v_mfma_f32_32x32x2_f32: lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; acc[i] holds D[8*(i/4) + 4*(l/32) + i%4][l%32].  As above
// the BT tile is transposed in the accumulators: a lane holds row
// 32w + l%32 and, per 32-column tile, the column groups 8g + 4*(l/32) + 0..3.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kRowBlock32 = 128;

// W = Y' C^{-T} for the wave's 16 rows of a 64-row half (Y' staged in LDS,
// ldy floats a row), on 16x16x4 matrix cores: the B operand straight from
// the FP32 copy of C^{-1} the decisions wrote (cfl32_index layout, one
// 16-byte load per tile and four steps; L2-resident, shared by the
// determinant's workgroups), so no staging, conversion or barrier.
template <int KP>
__device__ __forceinline__ void w_from_y32(const float *ylds, int ldy, const float *__restrict__ c32,
                                           f32x4 (&wacc)[KP / 16]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < KP / 16; ++t) wacc[t] = f32x4{0, 0, 0, 0};
    DSU_GLOBAL const f32x4 *cg = (DSU_GLOBAL const f32x4 *)c32 + lane;
    const float *yrow = ylds + (16 * wave + (lane & 15)) * ldy + (lane >> 4);
#pragma unroll 2
    for (int q = 0; q < KP / 16; ++q) {
        f32x4 b[KP / 16];
#pragma unroll
        for (int t = 0; t < KP / 16; ++t) b[t] = cg[(t * (KP / 16) + q) * 64];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float a = yrow[4 * (4 * q + e)];
#pragma unroll
            for (int t = 0; t < KP / 16; ++t) wacc[t] = Mma<float>::mma(a, b[t][e], wacc[t]);
        }
    }
}

template <int KP> struct Stream32Cfg {
    static constexpr int CW = KP <= 64 ? 64 : 32, VEC = 4, KH = KP / 2;
    static constexpr int LDVT = KP + 4, LDU = CW + 4, LDY = KP + 4;
    static constexpr int NV = KP * (CW / VEC) / kThreads;
    static constexpr int buf = CW * LDVT + KP * LDU;
    static constexpr int chunk = 2 * buf;
    static constexpr int wpart = 64 * LDY;  // one 64-row half of Y' at a time
    static constexpr int elems = chunk > wpart ? chunk : wpart;
    static_assert(NV >= 1 && NV * kThreads == KP * (CW / VEC), "staging split");
};

template <int KP>
__global__ __launch_bounds__(kThreads, 2) void k_flush_stream32(const DetDesc<float> *__restrict__ descs, int np, int nblk,
                                                             int kp, int kslots, int cur, int has_next, int e0n,
                                                             int kwn) {
    typedef Stream32Cfg<KP> C;
    typedef typename Vec16<float>::type vec_t;
    constexpr int CW = C::CW, LDVT = C::LDVT, LDU = C::LDU, LDY = C::LDY, NV = C::NV, KH = C::KH;
    constexpr int NT = CW / 32, JT = KP / 32;
    __shared__ __attribute__((aligned(16))) float lds[C::elems];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * kRowBlock32;
    const DetDesc<float> dd = descs[d];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    DSU_GLOBAL const float *vcur = gmem<const float>(cur ? dd.vg2 : dd.vg);
    DSU_GLOBAL const float *unext = gmem<const float>(cur ? dd.u : dd.u2);
    DSU_GLOBAL float *y = gmem(dd.y);
    const int rows = np - r0 < kRowBlock32 ? np - r0 : kRowBlock32;  // 64 or 128
    const bool wvalid = 32 * wave < rows;                              // wave-uniform

    // W = (y - E) C^{-T} for this block's rows, one 64-row half at a time;
    // waves 0-1 keep the first half's rows as B operands, waves 2-3 the second's
    float wa[KH];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int h0 = 64 * half;
        {
            // 16-byte loads, all in flight before their stores (scalar loads
            // batched the same way cost the K = 128 kernel registers it has not
            // got); rows past the block read row r0 and are zeroed
            constexpr int NQ = 16 * KP / kThreads;
            f32x4 yv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int v = tid + q * kThreads, i = v / (KP / 4), jq = v % (KP / 4);
                const bool in = h0 + i < rows;
                yv[q] = *(DSU_GLOBAL const f32x4 *)(y + (size_t)(r0 + (in ? h0 + i : 0)) * kp + 4 * jq);
                if (!in) yv[q] = f32x4{0, 0, 0, 0};
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int v = tid + q * kThreads, i = v / (KP / 4), jq = v % (KP / 4);
                *reinterpret_cast<f32x4 *>(lds + i * LDY + 4 * jq) = yv[q];
            }
        }
        __syncthreads();
        for (int j = tid; j < kslots; j += kThreads) {
            const int e = dd.idx[j] - r0 - h0;
            if (e >= 0 && e < 64 && h0 + e < rows) lds[e * LDY + j] -= 1.0f;
        }
        __syncthreads();
        f32x4 w[KP / 16];
        w_from_y32<KP>(lds, LDY, dd.cfl32, w);
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[(16 * wave + 4 * (lane >> 4) + i) * LDY + 16 * t + (lane & 15)] = w[t][i];
        __syncthreads();
        // B operand of the V^T W^T product; contraction over slot (lane/32)*KH + s
        if ((wave >> 1) == half)
#pragma unroll
            for (int s = 0; s < KH; ++s) wa[s] = -lds[(32 * (wave & 1) + (lane & 31)) * LDY + (lane >> 5) * KH + s];
        __syncthreads();
    }

    const int lrow = 32 * wave + (lane & 31);
    DSU_GLOBAL float *rp = gmem(dd.bt) + (size_t)(r0 + (wvalid ? lrow : 0)) * np + 4 * (lane >> 5);
    const int g = r0 + lrow - e0n;
    const bool wv = wvalid && has_next && g >= 0 && g < kwn;
    DSU_GLOBAL float *vp = gmem(cur ? dd.vg : dd.vg2) + (size_t)(wv ? g : 0) * np + 4 * (lane >> 5);
    int goff[NV], voff[NV], uoff[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int v = tid + q * kThreads, r = v / (CW / 4), cc = (v % (CW / 4)) * 4;
        goff[q] = r * np + cc;
        voff[q] = cc * LDVT + r;
        uoff[q] = r * LDU + cc;
    }
    vec_t sv[NV], su[NV], nx[NT * 4];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        sv[q] = *(DSU_GLOBAL const vec_t *)(vcur + goff[q]);
        if (has_next) su[q] = *(DSU_GLOBAL const vec_t *)(unext + goff[q]);
    }
#pragma unroll
    for (int h = 0; h < NT * 4; ++h)
        nx[h] = wvalid ? *(DSU_GLOBAL const vec_t *)(rp + (h / 4) * 32 + (h % 4) * 8) : vec_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) lds[voff[q] + e * LDVT] = sv[q][e];
        if (has_next) *reinterpret_cast<vec_t *>(lds + CW * LDVT + uoff[q]) = su[q];
    }
    __syncthreads();

    f32x16 accy[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) accy[t][i] = 0.0f;
    int cb = 0;
    for (int c0 = 0; c0 < np; c0 += CW, cb ^= 1) {
        const float *Vt = lds + cb * C::buf;
        const float *Us = Vt + CW * LDVT;
        f32x16 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[t][i] = nx[t * 4 + i / 4][i % 4];
        const int c1 = c0 + CW;
        if (c1 < np) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                sv[q] = *(DSU_GLOBAL const vec_t *)(vcur + goff[q] + c1);
                if (has_next) su[q] = *(DSU_GLOBAL const vec_t *)(unext + goff[q] + c1);
            }
            if (wvalid)
#pragma unroll
                for (int h = 0; h < NT * 4; ++h)
                    nx[h] = *(DSU_GLOBAL const vec_t *)(rp + c1 + (h / 4) * 32 + (h % 4) * 8);
        }
        // operands of the next group of products are read from LDS while the
        // current group runs
        const float *ap = Vt + (lane & 31) * LDVT + (lane >> 5) * KH;
        vec_t a[2][NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) a[0][t] = *reinterpret_cast<const vec_t *>(ap + 32 * t * LDVT);
#pragma unroll
        for (int j = 0; j < KH / 4; ++j) {
            if (j + 1 < KH / 4)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    a[(j + 1) & 1][t] = *reinterpret_cast<const vec_t *>(ap + 32 * t * LDVT + 4 * (j + 1));
            __builtin_amdgcn_sched_barrier(0);  // keep those reads ahead of this group's products
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j & 1][t][e], wa[4 * j + e], acc[t], 0, 0, 0);
        }
        if (wvalid)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const vec_t o = {acc[t][4 * gq], acc[t][4 * gq + 1], acc[t][4 * gq + 2], acc[t][4 * gq + 3]};
                    *(DSU_GLOBAL vec_t *)(rp + c0 + 32 * t + 8 * gq) = o;
                    if (wv) *(DSU_GLOBAL vec_t *)(vp + c0 + 32 * t + 8 * gq) = o;
                }
        if (has_next) {
            const float *up = Us + (lane & 31) * LDU + 4 * (lane >> 5);
            // read one group ahead, except at K = 128 where a group is already
            // 16 products long and the registers are needed elsewhere
            constexpr int UB = JT >= 4 ? 1 : 2;
            vec_t ub[UB][JT];
#pragma unroll
            for (int jt = 0; jt < JT; ++jt) ub[0][jt] = *reinterpret_cast<const vec_t *>(up + 32 * jt * LDU);
#pragma unroll
            for (int q = 0; q < NT * 4; ++q) {  // q = 4t + gq
                if (UB == 2 && q + 1 < NT * 4) {
#pragma unroll
                    for (int jt = 0; jt < JT; ++jt)
                        ub[(q + 1) % UB][jt] = *reinterpret_cast<const vec_t *>(
                            up + 32 * jt * LDU + 32 * ((q + 1) / 4) + 8 * ((q + 1) % 4));
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (UB == 1 && q > 0)
#pragma unroll
                    for (int jt = 0; jt < JT; ++jt)
                        ub[0][jt] = *reinterpret_cast<const vec_t *>(up + 32 * jt * LDU + 32 * (q / 4) + 8 * (q % 4));
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int jt = 0; jt < JT; ++jt)
                        accy[jt] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[q / 4][4 * (q % 4) + e],
                                                                        ub[q % UB][jt][e], accy[jt], 0, 0, 0);
            }
        }
        if (c1 < np) {
            float *nb = lds + (cb ^ 1) * C::buf;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
#pragma unroll
                for (int e = 0; e < 4; ++e) nb[voff[q] + e * LDVT] = sv[q][e];
                if (has_next) *reinterpret_cast<vec_t *>(nb + CW * LDVT + uoff[q]) = su[q];
            }
        }
        __syncthreads();
    }
    if (has_next && wvalid) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                y[(size_t)(r0 + 32 * wave + 8 * (i / 4) + 4 * (lane >> 5) + i % 4) * kp + 32 * jt + (lane & 31)] =
                    accy[jt][i];
    }
}

template <typename T>
hipError_t launch_flush_stream(const DetDesc<T> *d, int ndesc, int np, int ktile, int kp, int kslots, int cur,
                               int has_next, int e0n, int kwn, hipStream_t s) {
    if (sizeof(T) == 4 && (ktile == 32 || ktile == 64 || ktile == 128)) {
        const int nblk = (np + kRowBlock32 - 1) / kRowBlock32;
        const DetDesc<float> *df = (const DetDesc<float> *)d;
        if (ktile == 32)
            hipLaunchKernelGGL((k_flush_stream32<32>), dim3(ndesc * nblk), dim3(kThreads), 0, s, df, np, nblk, kp,
                               kslots, cur, has_next, e0n, kwn);
        else if (ktile == 64)
            hipLaunchKernelGGL((k_flush_stream32<64>), dim3(ndesc * nblk), dim3(kThreads), 0, s, df, np, nblk, kp,
                               kslots, cur, has_next, e0n, kwn);
        else
            hipLaunchKernelGGL((k_flush_stream32<128>), dim3(ndesc * nblk), dim3(kThreads), 0, s, df, np, nblk, kp,
                               kslots, cur, has_next, e0n, kwn);
        return hipGetLastError();
    }
    const int nblk = np / kRowBlock;
    const dim3 grid(ndesc * nblk);
#define DSU_S(KPV)                                                                                           \
    if (ktile == KPV) {                                                                                      \
        hipLaunchKernelGGL((k_flush_stream<T, KPV>), grid, dim3(kThreads), 0, s, d, np, nblk, kp, kslots, cur, \
                           has_next, e0n, kwn);                                                              \
        return hipGetLastError();                                                                            \
    }
    DSU_S(16) DSU_S(32) DSU_S(64) DSU_S(128) DSU_S(256)
#undef DSU_S
    return hipErrorInvalidValue;
}
template hipError_t launch_flush_stream<float>(const DetDesc<float> *, int, int, int, int, int, int, int, int, int,
                                               hipStream_t);
template hipError_t launch_flush_stream<double>(const DetDesc<double> *, int, int, int, int, int, int, int, int, int,
                                                hipStream_t);

}  // namespace dsu
