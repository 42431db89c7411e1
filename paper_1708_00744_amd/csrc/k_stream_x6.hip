// k_stream_x6.hip -- the streaming Woodbury flush of the batched FP32 form
// (eq. (4)) fused with the next window's look-ahead products (eq. (3)), with
// both matrix products on the bf16 matrix cores at FP32 accuracy.
//
// Every FP32 operand x is split into three bf16 parts, x = h + m + l: h is x
// rounded to bf16, m the rounding of x - h, l the rounding of what is left
// (each remainder is exact in FP32, so the split holds x to within 2^-26
// relative).  A product of two split operands keeps the six cross terms with
// weight >= 2^-16 (hh, hm, mh, hl, lh, mm); the dropped ones (ml, lm, ll) are
// below 2^-25 of |x||y|.  Products of bf16 pairs are exact in the FP32
// accumulator, so the result carries FP32 rounding only: the same error
// budget as FP32 products, at 6/16 of their matrix-core time (bf16 runs 16x
// the FP32 rate on gfx950).
//
// Layout as in the FP32 streaming kernel: 128 rows of BT per workgroup, 32 per
// wave; per 32-column tile the BT tile sits transposed in the accumulators
// (lane l: row 32w + l%32, columns 8q + 4*(l/32) + 0..3), so the same
// registers, split, are the A operand of BT_new U_next^T.
// v_mfma_f32_32x32x16_bf16: lane l supplies A[l%32][8*(l/32) + 0..7] and
// B[8*(l/32) + 0..7][l%32]; acc[i] holds D[8*(i/4) + 4*(l/32) + i%4][l%32].
//
// Each column chunk of V (this window's stale rows) and U (the next window's
// proposal rows) is split once per workgroup while it is staged into LDS as
// three bf16 planes: V^T as [column][slot], U as [slot][column'] where
// column' swaps bits 2 and 3 of the column inside each 16-column group, so
// that the eight columns a lane contracts over in one product are contiguous.
#include "dsu_internal.hpp"
#include "tiles.hpp"

namespace dsu {

typedef float x6acc_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

struct Split3 {
    bf16x8 h, m, l;
};

// Split a pair: one conversion per part (bf16 round to nearest even), the
// remainders exact in FP32.  Returns the packed pairs of h, m, l.
__device__ __forceinline__ void split2(float x0, float x1, unsigned &h, unsigned &m, unsigned &l) {
    const bf16x2 hp = {(__bf16)x0, (__bf16)x1};
    h = __builtin_bit_cast(unsigned, hp);
    const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xffff0000u);
    const bf16x2 mp = {(__bf16)r0, (__bf16)r1};
    m = __builtin_bit_cast(unsigned, mp);
    const float s0 = r0 - __uint_as_float(m << 16), s1 = r1 - __uint_as_float(m & 0xffff0000u);
    const bf16x2 lp = {(__bf16)s0, (__bf16)s1};
    l = __builtin_bit_cast(unsigned, lp);
}

__device__ __forceinline__ void split8(const float (&x)[8], Split3 &o) {
    u32x4 h, m, l;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned a, b, c;
        split2(x[2 * i], x[2 * i + 1], a, b, c);
        h[i] = a;
        m[i] = b;
        l[i] = c;
    }
    o.h = __builtin_bit_cast(bf16x8, h);
    o.m = __builtin_bit_cast(bf16x8, m);
    o.l = __builtin_bit_cast(bf16x8, l);
}

__device__ __forceinline__ x6acc_t mma6(const Split3 &a, const Split3 &b, x6acc_t c) {
    // smallest terms first
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.m, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h, b.l, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.m, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h, b.h, c, 0, 0, 0);
    return c;
}

constexpr int kRowBlockX6 = 128;

template <int KP> struct X6Cfg {
    static constexpr int CW = KP <= 64 ? 64 : 32;          // columns per chunk
    static constexpr int NT = CW / 32;                     // 32-column tiles per wave
    static constexpr int NS = KP / 16;                     // update products of 16 slots
    static constexpr int JT = KP / 32;                     // 32-slot tiles of y
    static constexpr int QW = CW / 4;                      // column quads per chunk
    static constexpr int SPT = KP * CW / (4 * kThreads);   // staged slots per thread (4 columns each)
    static constexpr int LDV = KP + 8;                     // bf16 per column of a V^T plane
    static constexpr int LDU = CW + 8;                     // bf16 per slot of a U plane
    static constexpr int VPL = CW * LDV, UPL = KP * LDU;   // plane sizes (bf16)
    static constexpr int BUF = 3 * VPL + 3 * UPL;          // one chunk (bf16)
    static constexpr int NBUF = KP <= 64 ? 1 : 2;          // LDS chunk buffers
    static constexpr int LDY = KP + 4;
    static constexpr int chunk_bytes = NBUF * BUF * 2;
    static constexpr int w_bytes = 4 * (64 * LDY + WCfg<float, KP>::elems);
    static constexpr int bytes = chunk_bytes > w_bytes ? chunk_bytes : w_bytes;
    static constexpr int occ = KP >= 128 ? 1 : 2;          // workgroups per CU (registers, LDS)
    static_assert(SPT >= 1 && SPT * 4 * kThreads == KP * CW, "staging split");
};

// Split one chunk's staged V (SPT slots x 4 columns per thread) and U into
// the planes of buffer `buf`.
template <int KP>
__device__ __forceinline__ void x6_put(__bf16 *buf, const f32x4 (&sv)[X6Cfg<KP>::SPT],
                                       const f32x4 (&su)[X6Cfg<KP>::SPT], bool has_next, int cq, int sg, int pq) {
    typedef X6Cfg<KP> C;
    constexpr int SPT = C::SPT;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        unsigned h[2], m[2], l[2];  // SPT <= 4 slots, packed in pairs
        if constexpr (SPT == 1) {
            unsigned a, b, c;
            split2(sv[0][e], 0.0f, a, b, c);
            h[0] = a;
            m[0] = b;
            l[0] = c;
        } else {
#pragma unroll
            for (int i = 0; i < SPT / 2; ++i) split2(sv[2 * i][e], sv[2 * i + 1][e], h[i], m[i], l[i]);
        }
        __bf16 *p = buf + (4 * cq + e) * C::LDV + SPT * sg;
        if constexpr (SPT == 4) {
            *reinterpret_cast<u32x2 *>(p) = u32x2{h[0], h[1]};
            *reinterpret_cast<u32x2 *>(p + C::VPL) = u32x2{m[0], m[1]};
            *reinterpret_cast<u32x2 *>(p + 2 * C::VPL) = u32x2{l[0], l[1]};
        } else if constexpr (SPT == 2) {
            *reinterpret_cast<unsigned *>(p) = h[0];
            *reinterpret_cast<unsigned *>(p + C::VPL) = m[0];
            *reinterpret_cast<unsigned *>(p + 2 * C::VPL) = l[0];
        } else {
            *reinterpret_cast<unsigned short *>(p) = (unsigned short)h[0];
            *reinterpret_cast<unsigned short *>(p + C::VPL) = (unsigned short)m[0];
            *reinterpret_cast<unsigned short *>(p + 2 * C::VPL) = (unsigned short)l[0];
        }
    }
    if (has_next)
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            unsigned h0, m0, l0, h1, m1, l1;
            split2(su[i][0], su[i][1], h0, m0, l0);
            split2(su[i][2], su[i][3], h1, m1, l1);
            __bf16 *p = buf + 3 * C::VPL + (SPT * sg + i) * C::LDU + 4 * pq;
            *reinterpret_cast<u32x2 *>(p) = u32x2{h0, h1};
            *reinterpret_cast<u32x2 *>(p + C::UPL) = u32x2{m0, m1};
            *reinterpret_cast<u32x2 *>(p + 2 * C::UPL) = u32x2{l0, l1};
        }
}

template <int KP>
__global__ __launch_bounds__(kThreads, X6Cfg<KP>::occ) void k_flush_stream_x6(
    const DetDesc<float> *__restrict__ descs, int np, int nblk, int kp, int kslots, int cur, int has_next, int e0n,
    int kwn) {
    typedef X6Cfg<KP> C;
    typedef f32x4 vec_t;
    constexpr int NT = C::NT, NS = C::NS, JT = C::JT, SPT = C::SPT, LDV = C::LDV, LDU = C::LDU, LDY = C::LDY,
                  CW = C::CW, QW = C::QW;
    __shared__ __attribute__((aligned(16))) char smem[C::bytes];
    float *lds = reinterpret_cast<float *>(smem);
    __bf16 *bl = reinterpret_cast<__bf16 *>(smem);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * kRowBlockX6;
    const DetDesc<float> dd = descs[d];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
    DSU_GLOBAL const float *vcur = gmem<const float>(cur ? dd.vg2 : dd.vg);
    DSU_GLOBAL const float *unext = gmem<const float>(cur ? dd.u : dd.u2);
    DSU_GLOBAL float *y = gmem(dd.y);
    const int rows = np - r0 < kRowBlockX6 ? np - r0 : kRowBlockX6;  // 64 or 128
    const bool wvalid = 32 * wave < rows;                             // wave-uniform

    // W = (y - E) C^{-T} for this block's rows, one 64-row half at a time;
    // each wave keeps -W of its 32 rows, split, as the B operands of the update
    Split3 wb[NS];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int h0 = 64 * half;
        {
            // loads in batches of 8 before their stores; rows past the block read row r0
            constexpr int NYL = 64 * KP / kThreads, NB = NYL < 8 ? NYL : 8;
#pragma unroll
            for (int q0 = 0; q0 < NYL; q0 += NB) {
                float yv[NB];
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const int v = tid + (q0 + q) * kThreads, i = v / KP, j = v % KP;
                    const bool in = h0 + i < rows;
                    yv[q] = y[(size_t)(r0 + (in ? h0 + i : 0)) * kp + j];
                    if (!in) yv[q] = 0.0f;
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
            const int e = dd.idx[j] - r0 - h0;
            if (e >= 0 && e < 64 && h0 + e < rows) lds[e * LDY + j] -= 1.0f;
        }
        __syncthreads();
        f32x4 w[KP / 16];
        w_from_y<float, KP>(lds, LDY, dd.cfl, kp, kslots, lds + 64 * LDY, w);
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[(16 * wave + 4 * (lane >> 4) + i) * LDY + 16 * t + (lane & 15)] = w[t][i];
        __syncthreads();
        if ((wave >> 1) == half)
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                float x[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) x[v] = -lds[(32 * (wave & 1) + (lane & 31)) * LDY + 16 * t + 8 * g + v];
                split8(x, wb[t]);
            }
        __syncthreads();
    }

    const int lrow = 32 * wave + (lane & 31);
    DSU_GLOBAL float *rp = gmem(dd.bt) + (size_t)(r0 + (wvalid ? lrow : 0)) * np + 4 * g;
    const int gi = r0 + lrow - e0n;
    const bool wv = wvalid && has_next && gi >= 0 && gi < kwn;
    DSU_GLOBAL float *vp = gmem(cur ? dd.vg : dd.vg2) + (size_t)(wv ? gi : 0) * np + 4 * g;
    // staging: thread = (slot group sg, column quad cq); U quads go to position pq
    const int cq = tid % QW, sg = tid / QW;
    const int pq = (cq & ~3) | ((cq & 1) << 1) | ((cq >> 1) & 1);
    const int goff = SPT * sg * np + 4 * cq;
    vec_t sv[SPT], su[SPT], nx[4 * NT];
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
        sv[i] = *(DSU_GLOBAL const vec_t *)(vcur + goff + i * np);
        su[i] = has_next ? *(DSU_GLOBAL const vec_t *)(unext + goff + i * np) : vec_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int h = 0; h < 4 * NT; ++h)
        nx[h] = wvalid ? *(DSU_GLOBAL const vec_t *)(rp + 32 * (h / 4) + 8 * (h % 4)) : vec_t{0, 0, 0, 0};
    x6_put<KP>(bl, sv, su, has_next, cq, sg, pq);
    __syncthreads();

    x6acc_t accy[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) accy[t][i] = 0.0f;
    int cb = 0;
    for (int c0 = 0; c0 < np; c0 += CW) {
        const __bf16 *buf = bl + cb * C::BUF;
        x6acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[t][i] = nx[4 * t + i / 4][i % 4];
        const int c1 = c0 + CW;
        if (c1 < np) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                sv[i] = *(DSU_GLOBAL const vec_t *)(vcur + goff + i * np + c1);
                if (has_next) su[i] = *(DSU_GLOBAL const vec_t *)(unext + goff + i * np + c1);
            }
            if (wvalid)
#pragma unroll
                for (int h = 0; h < 4 * NT; ++h)
                    nx[h] = *(DSU_GLOBAL const vec_t *)(rp + c1 + 32 * (h / 4) + 8 * (h % 4));
        }
        // BT_chunk^T += V^T (-W)^T
        const __bf16 *ap = buf + (lane & 31) * LDV + 8 * g;
#pragma unroll
        for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                Split3 a;
                a.h = *reinterpret_cast<const bf16x8 *>(ap + 32 * nt * LDV + 16 * t);
                a.m = *reinterpret_cast<const bf16x8 *>(ap + C::VPL + 32 * nt * LDV + 16 * t);
                a.l = *reinterpret_cast<const bf16x8 *>(ap + 2 * C::VPL + 32 * nt * LDV + 16 * t);
                acc[nt] = mma6(a, wb[t], acc[nt]);
            }
        if (wvalid)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const vec_t o = {acc[nt][4 * gq], acc[nt][4 * gq + 1], acc[nt][4 * gq + 2], acc[nt][4 * gq + 3]};
                    *(DSU_GLOBAL vec_t *)(rp + c0 + 32 * nt + 8 * gq) = o;
                    if (wv) *(DSU_GLOBAL vec_t *)(vp + c0 + 32 * nt + 8 * gq) = o;
                }
        if (has_next) {
            // y += BT_new U_next^T over this chunk's columns (products of 16)
            const __bf16 *up = buf + 3 * C::VPL + (lane & 31) * LDU + 8 * g;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    Split3 xa;
                    float x[8];
#pragma unroll
                    for (int v = 0; v < 8; ++v) x[v] = acc[nt][8 * s + v];
                    split8(x, xa);
#pragma unroll
                    for (int jt = 0; jt < JT; ++jt) {
                        Split3 u;
                        const int o = 32 * jt * LDU + 32 * nt + 16 * s;
                        u.h = *reinterpret_cast<const bf16x8 *>(up + o);
                        u.m = *reinterpret_cast<const bf16x8 *>(up + C::UPL + o);
                        u.l = *reinterpret_cast<const bf16x8 *>(up + 2 * C::UPL + o);
                        accy[jt] = mma6(xa, u, accy[jt]);
                    }
                }
        }
        if (c1 < np) {
            if constexpr (C::NBUF == 1) {
                __syncthreads();  // every wave is done with the buffer
                x6_put<KP>(bl, sv, su, has_next, cq, sg, pq);
            } else {
                // the other buffer was last read before the previous barrier
                cb ^= 1;
                x6_put<KP>(bl + cb * C::BUF, sv, su, has_next, cq, sg, pq);
            }
        }
        __syncthreads();
    }
    if (has_next && wvalid) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                y[(size_t)(r0 + 32 * wave + 8 * (i / 4) + 4 * g + i % 4) * kp + 32 * jt + (lane & 31)] = accy[jt][i];
    }
}

hipError_t launch_flush_stream_x6(const DetDesc<float> *d, int ndesc, int np, int ktile, int kp, int kslots, int cur,
                                  int has_next, int e0n, int kwn, hipStream_t s) {
    const int nblk = (np + kRowBlockX6 - 1) / kRowBlockX6;
    const dim3 grid(ndesc * nblk);
#define DSU_X6(KPV)                                                                                              \
    if (ktile == KPV) {                                                                                          \
        hipLaunchKernelGGL((k_flush_stream_x6<KPV>), grid, dim3(kThreads), 0, s, d, np, nblk, kp, kslots, cur,   \
                           has_next, e0n, kwn);                                                                  \
        return hipGetLastError();                                                                                \
    }
    DSU_X6(32) DSU_X6(64) DSU_X6(128)
#undef DSU_X6
    return hipErrorInvalidValue;
}

}  // namespace dsu
