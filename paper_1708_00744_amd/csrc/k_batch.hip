// k_batch.hip -- kernels of the batched (device-driven) form.
//
// A window is K consecutive proposals of one determinant (electrons e0..e0+kw-1
// of the current sweep).  Every electron moves at most once per window, so all
// kw proposed rows are known before any decision is made: a proposal only
// depends on its electron's position at the start of the window and on the
// random stream.  The look-ahead quantities of eq. (3) for the whole window
// are then entries of one small product,
//     G[a][b] = phi_a . BT[e0 + b, :]        (kw x kw, on matrix cores)
// and the sequential part -- the Metropolis decisions in proposal order with
// the bordered inverse of C -- needs only G:
//     for accepted set S:  R_a = G[a][a] - G[a][S] C_S^{-1} G[S][a]
// which equals det(A_new)/det(A) of the one-move-at-a-time method (Sec. II).
// Rejected proposals keep their slot (uniform work, Sec. II's second variant)
// but their rows and columns of the flush's C^{-1} are zero.
#include "dsu_internal.hpp"
#include "tiles.hpp"

#include <type_traits>
#include <utility>

namespace dsu {

// ------------------------------------------------------------ random stream
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64 x 64 -> 128-bit
// products; the high halves are xor-ed with the other two counter words and
// the round key; the key advances by the Weyl increments after each round.
struct P4 { uint64_t w[4]; };

__device__ __forceinline__ P4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                            uint64_t k1) {
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t inc0 = 0x9E3779B97F4A7C15ull, inc1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo_a = m0 * c0, hi_a = __umul64hi(m0, c0);
        const uint64_t lo_b = m1 * c2, hi_b = __umul64hi(m1, c2);
        const uint64_t n0 = hi_b ^ c1 ^ k0, n2 = hi_a ^ c3 ^ k1;
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
        k0 += inc0; k1 += inc1;
    }
    return P4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Gaussian step and Metropolis uniform of one proposal.  Box-Muller (1958) on
// the first pair (x, y) and the second pair's cosine branch (z); uniform from
// block 1.  Counter = (sweep, spin*n + e, block, 0); key = (seed, walker).
__device__ __forceinline__ void move_draw(uint64_t seed, uint64_t wid, uint64_t sweep, uint64_t slot, double g[3],
                                          double &u) {
#pragma clang fp contract(off)
    const P4 a = philox4x64_10(sweep, slot, 0, 0, seed, wid);
    const P4 b = philox4x64_10(sweep, slot, 1, 0, seed, wid);
    const double twopi = 6.283185307179586476925286766559;
    const double r1 = sqrt(-2.0 * log(1.0 - unit53(a.w[0])));
    const double t1 = twopi * unit53(a.w[1]);
    const double r2 = sqrt(-2.0 * log(1.0 - unit53(a.w[2])));
    const double t2 = twopi * unit53(a.w[3]);
    g[0] = r1 * cos(t1);
    g[1] = r1 * sin(t1);
    g[2] = r2 * cos(t2);
    u = unit53(b.w[0]);
}

// Plane-wave orbital: 1, cos(k.r) or sin(k.r), k = (2 pi / L)(nx, ny, nz).
__device__ __forceinline__ double pw_orbital(int4 kv, double twopi_l, double x, double y, double z) {
#pragma clang fp contract(off)
    if (kv.w == 0) return 1.0;
    const double t = ((double)kv.x * x + (double)kv.y * y) + (double)kv.z * z;
    const double ph = twopi_l * t;
    return kv.w == 1 ? cos(ph) : sin(ph);
}

// ------------------------------------------------------- window proposals
// grid (ndesc, nsplit): every block draws the window's kw moves (cheap) and
// fills its column range of U (proposed orbital rows, zero past kw and n) and
// Vg (the stale BT rows e0..e0+kw-1, zero past kw).  Block 0 of a determinant
// also stores the proposals for the decision kernel.
//
// Orbitals from per-axis phase factors: with q = 2 pi / L,
// exp(i q (nx x + ny y + nz z)) = Ex^nx Ey^ny Ez^nz and E^-n = conj(E^n), so a
// group of proposals needs only cos/sin(q n r_axis) for 0 <= n <= nmax (one
// sincos each), and every orbital is two complex products (cos = real part,
// sin = imaginary part).  Used when nmax <= kPwTab; otherwise cos/sin per
// orbital.
constexpr int kPwTab = 24;
constexpr int kPwGroup = 32;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_window_rows(const DetDesc<T> *__restrict__ descs, int n, int np,
                                                          int ktile, int e0, int kw, const int4 *__restrict__ kvec,
                                                          double twopi_l, int buf, int copy_vg, int nmax) {
#pragma clang fp contract(off)
    __shared__ double s_r[DSU_KMAX_LDS][3];
    __shared__ double s_c[kPwGroup][3][kPwTab + 1], s_s[kPwGroup][3][kPwTab + 1];
    const DetDesc<T> d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    const long long sweep = d.st->sweep;
    for (int a = tid; a < kw; a += kThreads) {
        double g[3], u;
        const int e = e0 + a;
        move_draw(d.seed, d.wid, (uint64_t)sweep, (uint64_t)d.spin * (uint64_t)n + (uint64_t)e, g, u);
        const double x = d.pos[3 * e + 0] + d.sigma * g[0];
        const double y = d.pos[3 * e + 1] + d.sigma * g[1];
        const double z = d.pos[3 * e + 2] + d.sigma * g[2];
        s_r[a][0] = x; s_r[a][1] = y; s_r[a][2] = z;
        if (blockIdx.y == 0) {
            double *pr = buf ? d.prop2 : d.prop;
            pr[4 * a + 0] = x; pr[4 * a + 1] = y; pr[4 * a + 2] = z; pr[4 * a + 3] = u;
        }
    }
    __syncthreads();
    const int cols = np / gridDim.y;
    const int c_begin = blockIdx.y * cols;
    T *uo = buf ? d.u2 : d.u;
    T *vo = buf ? d.vg2 : d.vg;
    if (nmax > kPwTab) {
        for (int v = tid; v < ktile * cols; v += kThreads) {
            const int a = v / cols, c = c_begin + v % cols;
            T val = T(0), vgv = T(0);
            if (a < kw) {
                if (c < n) val = T(pw_orbital(kvec[c], twopi_l, s_r[a][0], s_r[a][1], s_r[a][2]));
                if (copy_vg) vgv = d.bt[(size_t)(e0 + a) * np + c];
            }
            uo[(size_t)a * np + c] = val;
            if (copy_vg) vo[(size_t)a * np + c] = vgv;
        }
        return;
    }
    for (int a0 = 0; a0 < ktile; a0 += kPwGroup) {
        const int ga = min(kPwGroup, ktile - a0);
        __syncthreads();
        for (int v = tid; v < ga * 3 * (nmax + 1); v += kThreads) {
            const int a = v / (3 * (nmax + 1)), r = v % (3 * (nmax + 1)), ax = r / (nmax + 1), m = r % (nmax + 1);
            double sn = 0.0, cs = 1.0;
            if (a0 + a < kw) sincos(twopi_l * ((double)m * s_r[a0 + a][ax]), &sn, &cs);
            s_c[a][ax][m] = cs;
            s_s[a][ax][m] = sn;
        }
        __syncthreads();
        if (cols == kThreads) {
            // one column per thread (uniform): its plane wave decoded once, the
            // group's proposals unrolled into independent chains; the same
            // operations per orbital as below
            const int c = c_begin + tid;
            const bool live = c < n;
            const int4 kv = live ? kvec[c] : make_int4(0, 0, 0, 0);
            const int mm[3] = {kv.x < 0 ? -kv.x : kv.x, kv.y < 0 ? -kv.y : kv.y, kv.z < 0 ? -kv.z : kv.z};
            const bool ng[3] = {kv.x < 0, kv.y < 0, kv.z < 0};
#pragma unroll 4
            for (int a = 0; a < ga; ++a) {
                const int ag = a0 + a;
                T val = T(0), vgv = T(0);
                if (ag < kw) {
                    if (live) {
                        double o = 1.0;
                        if (kv.w != 0) {
                            double re = 1.0, im = 0.0;
#pragma unroll
                            for (int ax = 0; ax < 3; ++ax) {
                                const double fc = s_c[a][ax][mm[ax]];
                                const double fs = ng[ax] ? -s_s[a][ax][mm[ax]] : s_s[a][ax][mm[ax]];
                                const double t = re * fc - im * fs;
                                im = re * fs + im * fc;
                                re = t;
                            }
                            o = kv.w == 1 ? re : im;
                        }
                        val = T(o);
                    }
                    if (copy_vg) vgv = d.bt[(size_t)(e0 + ag) * np + c];
                }
                uo[(size_t)ag * np + c] = val;
                if (copy_vg) vo[(size_t)ag * np + c] = vgv;
            }
            continue;
        }
        for (int v = tid; v < ga * cols; v += kThreads) {
            const int a = v / cols, c = c_begin + v % cols, ag = a0 + a;
            T val = T(0), vgv = T(0);
            if (ag < kw) {
                if (c < n) {
                    const int4 kv = kvec[c];
                    double o = 1.0;
                    if (kv.w != 0) {
                        const int ax_n[3] = {kv.x, kv.y, kv.z};
                        double re = 1.0, im = 0.0;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            const int m = ax_n[ax] < 0 ? -ax_n[ax] : ax_n[ax];
                            const double fc = s_c[a][ax][m];
                            const double fs = ax_n[ax] < 0 ? -s_s[a][ax][m] : s_s[a][ax][m];
                            const double t = re * fc - im * fs;
                            im = re * fs + im * fc;
                            re = t;
                        }
                        o = kv.w == 1 ? re : im;
                    }
                    val = T(o);
                }
                if (copy_vg) vgv = d.bt[(size_t)(e0 + ag) * np + c];
            }
            uo[(size_t)ag * np + c] = val;
            if (copy_vg) vo[(size_t)ag * np + c] = vgv;
        }
    }
}

template <typename T>
hipError_t launch_window_props(const DetDesc<T> *d, int ndesc, int n, int np, int ktile, int e0, int kw,
                               const int4 *kvec, double twopi_over_l, int buf, int copy_vg, int nmax, hipStream_t s) {
    int nsplit = np / 256;
    if (nsplit < 1) nsplit = 1;
    while (np % nsplit) --nsplit;
    hipLaunchKernelGGL((k_window_rows<T>), dim3(ndesc, nsplit), dim3(kThreads), 0, s, d, n, np, ktile, e0, kw, kvec,
                       twopi_over_l, buf, copy_vg, nmax);
    return hipGetLastError();
}
template hipError_t launch_window_props<float>(const DetDesc<float> *, int, int, int, int, int, int, const int4 *,
                                               double, int, int, int, hipStream_t);
template hipError_t launch_window_props<double>(const DetDesc<double> *, int, int, int, int, int, int, const int4 *,
                                                double, int, int, int, hipStream_t);

// ------------------------------------------------------ window decisions
// One workgroup (max(64, KP) threads) per determinant.  Thread i owns row i
// of the bordered inverse C_S^{-1} (S = accepted proposals so far).
template <int KP> struct DecideCfg {
    static constexpr int threads = KP < 64 ? 64 : KP;
    static constexpr int ld = KP + 1;
    static constexpr bool g_lds = KP <= 64;
    static constexpr bool c_lds = KP <= 128;
    static constexpr int lds_g = g_lds ? KP * ld : 1;
    static constexpr int lds_c = c_lds ? KP * ld : 1;
};

template <typename T, int KP>
__global__ __launch_bounds__(DecideCfg<KP>::threads) void k_window_decide(const DetDesc<T> *__restrict__ descs,
                                                                          int kp, int e0, int kw, int force_accept,
                                                                          int last_window, int pbuf) {
    typedef DecideCfg<KP> C;
    constexpr int LD = C::ld, NT = C::threads;
    __shared__ double s_g[C::lds_g];
    __shared__ double s_c[C::lds_c];
    __shared__ double s_q[KP], s_p[KP], s_t[KP], s_b[KP], s_u[KP], s_red[NT / 64];
    __shared__ int s_acc[KP], s_pos[KP];
    __shared__ double s_ratio[KP];
    __shared__ int s_ok[KP];
    const DetDesc<T> d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *G = C::g_lds ? s_g : d.gwork;
    double *Cm = C::c_lds ? s_c : d.cwork;

    // G[a][b] = phi_a . BT[e0 + b, :], formed by the previous flush pass
    for (int v = tid; v < kw * kw; v += NT) {
        const int a = v / kw, b = v % kw;
        G[a * LD + b] = (double)d.y[(size_t)(e0 + b) * kp + a];
    }
    for (int a = tid; a < KP; a += NT) {
        s_u[a] = a < kw ? (pbuf ? d.prop2 : d.prop)[4 * a + 3] : 0.0;
        s_pos[a] = -1;
    }
    __syncthreads();

    int m = 0;
    double logdet = 0.0;
    int sgn = 1, bad = 0;
    for (int a = 0; a < kw; ++a) {
        if (tid < m) {
            s_q[tid] = G[s_acc[tid] * LD + a];
            s_p[tid] = G[a * LD + s_acc[tid]];
        }
        __syncthreads();
        double part = 0.0;
        if (tid < m) {
            double t = 0.0, bb = 0.0;
            const double *crow = Cm + tid * LD;
            for (int j = 0; j < m; ++j) {
                t += crow[j] * s_q[j];
                bb += s_p[j] * Cm[j * LD + tid];
            }
            s_t[tid] = t;
            s_b[tid] = bb;
            part = s_p[tid] * t;
        }
        // block reduction of p.t
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if (NT > 64) {
            if (lane == 0) s_red[wave] = part;
            __syncthreads();
            part = 0.0;
            for (int q = 0; q < NT / 64; ++q) part += s_red[q];
        } else {
            __syncthreads();
        }
        const double r = G[a * LD + a] - part;
        const bool finite_nz = fabs(r) > RatioFloor<T>::value && fabs(r) <= 1.7976931348623157e308;
        const bool ok = finite_nz && (force_accept || s_u[a] < r * r);
        if (!finite_nz) ++bad;
        if (tid == 0) { s_ratio[a] = r; s_ok[a] = ok; }
        if (ok) {
            const double rinv = 1.0 / r;
            if (tid < m) {
                double *crow = Cm + tid * LD;
                const double ti = s_t[tid] * rinv;
                for (int j = 0; j < m; ++j) crow[j] += ti * s_b[j];
                crow[m] = -ti;
            } else if (tid == m) {
                double *crow = Cm + m * LD;
                for (int j = 0; j < m; ++j) crow[j] = -s_b[j] * rinv;
                crow[m] = rinv;
                s_acc[m] = a;
                s_pos[a] = m;
            }
            logdet += log(fabs(r));
            if (r < 0.0) sgn = -sgn;
            ++m;
        }
        __syncthreads();
    }

    // zero-embedded C^{-1} for the flush, electrons, positions, state, trace
    for (int v = tid; v < KP * KP; v += NT) {
        const int i = v / KP, j = v % KP;
        const int pi = s_pos[i], pj = s_pos[j];
        d.cfl[(size_t)i * kp + j] = (pi >= 0 && pj >= 0) ? Cm[pi * LD + pj] : 0.0;
    }
    for (int a = tid; a < KP; a += NT) d.idx[a] = a < kw ? e0 + a : -1;
    for (int v = tid; v < kw * 3; v += NT) {
        const int a = v / 3, c = v % 3;
        if (s_ok[a]) d.pos[3 * (e0 + a) + c] = (pbuf ? d.prop2 : d.prop)[4 * a + c];
    }
    if (tid == 0) {
        DetState *st = d.st;
        if (d.trace_r) {
            const long long p0 = st->trace_pos;
            for (int a = 0; a < kw; ++a)
                if (p0 + a < d.trace_cap) {
                    d.trace_r[p0 + a] = s_ratio[a];
                    d.trace_a[p0 + a] = (uint8_t)s_ok[a];
                }
            st->trace_pos = p0 + kw;
        }
        st->logdet += logdet;
        st->sign *= sgn;
        st->accepted += m;
        st->bad += bad;
        if (last_window) st->sweep += 1;
    }
}

// The same decisions for windows of up to 128 slots as an in-place
// Gauss-Jordan sweep over G in slot order, pivoting only on accepted slots:
// before slot a is decided, G[a][a] has had every earlier accepted slot
// eliminated, so it is the Schur complement r0 - p^T C^{-1} q of the
// look-ahead; after the window, G restricted to the accepted slots is C^{-1}.
// Four waves; wave w holds rows w*KP/4 .. of G, lane y columns y (and y + 64
// at K = 128), in registers (the loop over slots is unrolled, so every
// register index is fixed).  A step is one LDS exchange of the pivot row and
// one barrier; the pivot column comes from one lane of each wave.
template <typename T, int KP>
__global__ __launch_bounds__(256) void k_window_decide_gj(const DetDesc<T> *__restrict__ descs, int kp, int e0,
                                                          int kw, int force_accept, int last_window, int pbuf) {
    constexpr int RW = KP / 4, CPL = KP > 64 ? KP / 64 : 1, NC = 64 * CPL;
    static_assert(KP >= 16 && KP <= 128 && RW % 4 == 0, "window tile");
    __shared__ double s_row[2][2][NC];
    __shared__ double s_u[KP], s_ratio[KP];
    __shared__ int s_ok[KP];
    const DetDesc<T> d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double g[RW][CPL];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            const int a = wave * RW + r, b = lane + 64 * h;
            double v = a == b ? 1.0 : 0.0;
            if (a < kw && b < kw) v = (double)d.y[(size_t)(e0 + b) * kp + a];
            g[r][h] = v;
        }
    for (int a = tid; a < KP; a += 256) {
        s_u[a] = a < kw ? (pbuf ? d.prop2 : d.prop)[4 * a + 3] : 0.0;
        s_ok[a] = 0;
    }
    __syncthreads();
    // |prod R| kept as mantissa * 2^exponent; one log at the end
    int m = 0, sgn = 1, bad = 0, pexp = 0;
    double pman = 1.0;
    // Decision and elimination step of slot j = jb * RW + JJ, whose pivot
    // column lies in column half JH; rv holds this lane's entries of the pivot
    // row and r = its entry in column j.  Both JJ and JH are compile-time
    // constants, so every register index is fixed and each row costs one FMA
    // per column half.  If nx is given, the step is also applied to that copy
    // of another row whose column-j entry is fx.
    auto slot = [&](auto jh_c, auto jj_c, int jb, const double *rv, double r, double uj, double *nx, double fx)
        __attribute__((always_inline)) {
        constexpr int JH = decltype(jh_c)::value, JJ = decltype(jj_c)::value;
        const int j = jb * RW + JJ;
        const bool finite_nz = fabs(r) > RatioFloor<T>::value && fabs(r) <= 1.7976931348623157e308;
        const bool ok = finite_nz && (force_accept || uj < r * r);
        if (!finite_nz) ++bad;
        if (tid == 0) {
            s_ratio[j] = r;
            s_ok[j] = ok;
        }
        if (!ok) return;
        const double dinv = 1.0 / r;
        const int jl = j & 63;
        const bool pl = lane == jl, prow = wave == jb;
        // Scaled pivot row (its own column becomes 1/r) and, for the other
        // rows, new = a * g - f * c: in lane j & 63 of half JH a = -1/r and
        // c = 0 (the pivot column's entry g = f becomes -f/r), elsewhere a = 1
        // and c = row / r.  Both forms round exactly as -f/r and g - f * row/r.
        double rj[CPL], c[CPL];
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            rj[h] = (h == JH && pl) ? dinv : rv[h] * dinv;
            c[h] = (h == JH && pl) ? 0.0 : rj[h];
        }
        const double a = pl ? -dinv : 1.0;
        if (nx)
#pragma unroll
            for (int h = 0; h < CPL; ++h) nx[h] = __builtin_fma(-fx, c[h], h == JH ? a * nx[h] : nx[h]);
        // pivot-column entries of QB rows at a time, read before their updates
        constexpr int QB = RW < 8 ? RW : 8;
#pragma unroll
        for (int q0 = 0; q0 < RW; q0 += QB) {
            double f[QB];
#pragma unroll
            for (int i = 0; i < QB; ++i) {
                const int lo = __builtin_amdgcn_readlane(__double2loint(g[q0 + i][JH]), jl);
                const int hi = __builtin_amdgcn_readlane(__double2hiint(g[q0 + i][JH]), jl);
                f[i] = __hiloint2double(hi, lo);
            }
#pragma unroll
            for (int i = 0; i < QB; ++i) {
                const int q = q0 + i;
#pragma unroll
                for (int h = 0; h < CPL; ++h) {
                    const double t = h == JH ? a * g[q][h] : g[q][h];
                    const double u = __builtin_fma(-f[i], c[h], t);
                    g[q][h] = (q == JJ && prow) ? rj[h] : u;
                }
            }
        }
        int e;
        pman *= frexp(fabs(r), &e);
        pexp += e;
        pman = frexp(pman, &e);
        pexp += e;
        if (r < 0.0) sgn = -sgn;
        ++m;
    };
    // Slots j and j + 1 (j = jb * RW + 2P; both rows in wave jb, both pivot
    // columns in half JH) with one LDS exchange and one barrier: the owner
    // publishes both rows, every wave applies slot j's step to its copy of
    // row j + 1 -- the same operations on the same values as the owner's own
    // update of that row -- and decides slot j + 1 from it.
    auto pair = [&](auto jh_c, auto p_c, int jb) __attribute__((always_inline)) {
        constexpr int P = decltype(p_c)::value, JJ = 2 * P, JH = decltype(jh_c)::value;
        const int j = jb * RW + JJ;
        if (j >= kw) return;
        double *row0 = s_row[P & 1][0], *row1 = s_row[P & 1][1];  // RW / 2 is even: buffers alternate
        const double u0 = s_u[j], u1 = s_u[j + 1];                 // read-only after the set-up barrier
        if (wave == jb)
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                row0[lane + 64 * h] = g[JJ][h];
                row1[lane + 64 * h] = g[JJ + 1][h];
            }
        __syncthreads();
        double v0[CPL], v1[CPL];
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            v0[h] = row0[lane + 64 * h];
            v1[h] = row1[lane + 64 * h];
        }
        const double r0 = row0[j], f1 = row1[j];
        slot(jh_c, std::integral_constant<int, JJ>{}, jb, v0, r0, u0, v1, f1);
        if (j + 1 >= kw) return;
        const int jl1 = (j + 1) & 63;
        const int lo = __builtin_amdgcn_readlane(__double2loint(v1[JH]), jl1);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v1[JH]), jl1);
        slot(jh_c, std::integral_constant<int, JJ + 1>{}, jb, v1, __hiloint2double(hi, lo), u1, nullptr, 0.0);
    };
    // blocks of RW slots whose pivot columns lie in column half 0, then half 1
    constexpr int NJB0 = CPL > 1 ? 2 : 4;
#pragma unroll 1
    for (int jb = 0; jb < NJB0; ++jb)
        static_for(std::make_integer_sequence<int, RW / 2>{},
                   [&](auto pp) __attribute__((always_inline)) { pair(std::integral_constant<int, 0>{}, pp, jb); });
    if constexpr (CPL > 1) {
#pragma unroll 1
        for (int jb = NJB0; jb < 4; ++jb)
            static_for(std::make_integer_sequence<int, RW / 2>{},
                       [&](auto pp) __attribute__((always_inline)) { pair(std::integral_constant<int, 1>{}, pp, jb); });
    }
    const double logdet = log(pman) + (double)pexp * 0.69314718055994530942;
    __syncthreads();
    // zero-embedded C^{-1} for the flush, electrons, positions, state, trace
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            const int a = wave * RW + r, b = lane + 64 * h;
            if (b < KP) d.cfl[(size_t)a * kp + b] = (s_ok[a] && s_ok[b]) ? g[r][h] : 0.0;
        }
    // the FP32 form's streaming flush reads the same matrix in FP32, laid out
    // as its W product's B operand
    if constexpr (sizeof(T) == 4 && KP >= 32)
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                const int a = wave * RW + r, b = lane + 64 * h;
                if (b < KP) d.cfl32[cfl32_index<KP>(a, b)] = (s_ok[a] && s_ok[b]) ? (float)g[r][h] : 0.0f;
            }
    for (int a = tid; a < KP; a += 256) d.idx[a] = a < kw ? e0 + a : -1;
    for (int v = tid; v < kw * 3; v += 256) {
        const int a = v / 3, c = v % 3;
        if (s_ok[a]) d.pos[3 * (e0 + a) + c] = (pbuf ? d.prop2 : d.prop)[4 * a + c];
    }
    if (tid == 0) {
        DetState *st = d.st;
        if (d.trace_r) {
            const long long p0 = st->trace_pos;
            for (int a = 0; a < kw; ++a)
                if (p0 + a < d.trace_cap) {
                    d.trace_r[p0 + a] = s_ratio[a];
                    d.trace_a[p0 + a] = (uint8_t)s_ok[a];
                }
            st->trace_pos = p0 + kw;
        }
        st->logdet += logdet;
        st->sign *= sgn;
        st->accepted += m;
        st->bad += bad;
        if (last_window) st->sweep += 1;
    }
}

template <typename T>
hipError_t launch_window_decide(const DetDesc<T> *d, int ndesc, int ktile, int kp, int e0, int kw, int force_accept,
                                int last_window, int pbuf, hipStream_t s) {
#define DSU_G(KPV)                                                                                                \
    if (ktile == KPV) {                                                                                           \
        hipLaunchKernelGGL((k_window_decide_gj<T, KPV>), dim3(ndesc), dim3(256), 0, s, d, kp, e0, kw,             \
                           force_accept, last_window, pbuf);                                                      \
        return hipGetLastError();                                                                                 \
    }
#define DSU_D(KPV)                                                                                                \
    if (ktile == KPV) {                                                                                           \
        hipLaunchKernelGGL((k_window_decide<T, KPV>), dim3(ndesc), dim3(DecideCfg<KPV>::threads), 0, s, d, kp,    \
                           e0, kw, force_accept, last_window, pbuf);                                              \
        return hipGetLastError();                                                                                 \
    }
    DSU_G(16) DSU_G(32) DSU_G(64) DSU_G(128) DSU_D(256)
#undef DSU_D
#undef DSU_G
    return hipErrorInvalidValue;
}
template hipError_t launch_window_decide<float>(const DetDesc<float> *, int, int, int, int, int, int, int, int,
                                                hipStream_t);
template hipError_t launch_window_decide<double>(const DetDesc<double> *, int, int, int, int, int, int, int, int,
                                                 hipStream_t);

// ------------------------------------------------------- streaming path
// y[i][a] = BT[i,:] . U[buf][a,:] for every row i (the look-ahead products of
// the first window of a sweep, for all rows at once).
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_window_prime(const DetDesc<T> *__restrict__ descs, int np, int nblk,
                                                           int kp, int buf) {
    constexpr int LDU = 128 / (int)sizeof(T) + 16 / (int)sizeof(T);
    __shared__ __attribute__((aligned(16))) T lds[KP * LDU];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int d = b / nblk, r0 = (b % nblk) * kRowBlock;
    const DetDesc<T> dd = descs[d];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    typename Mma<T>::acc_t acc[KP / 16];
    rowblock_times_ut<T, KP>(dd.bt + (size_t)r0 * np, np, kRowBlock, buf ? dd.u2 : dd.u, np, 0, np, lds, acc);
#pragma unroll
    for (int t = 0; t < KP / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r0 + 16 * wave + Mma<T>::row0(lane) + i * Mma<T>::row_step;
            dd.y[(size_t)row * kp + 16 * t + (lane & 15)] = acc[t][i];
        }
}

template <typename T>
hipError_t launch_window_prime(const DetDesc<T> *d, int ndesc, int np, int ktile, int kp, int buf, hipStream_t s) {
    const int nblk = np / kRowBlock;
    const dim3 grid(ndesc * nblk);
#define DSU_P(KPV)                                                                                          \
    if (ktile == KPV) {                                                                                     \
        hipLaunchKernelGGL((k_window_prime<T, KPV>), grid, dim3(kThreads), 0, s, d, np, nblk, kp, buf);     \
        return hipGetLastError();                                                                           \
    }
    DSU_P(16) DSU_P(32) DSU_P(64) DSU_P(128) DSU_P(256)
#undef DSU_P
    return hipErrorInvalidValue;
}
template hipError_t launch_window_prime<float>(const DetDesc<float> *, int, int, int, int, int, hipStream_t);
template hipError_t launch_window_prime<double>(const DetDesc<double> *, int, int, int, int, int, hipStream_t);

// ------------------------------------------------- Slater matrix, FP64
// M[j][i] = phi_j(r_i) for i, j < n (the transpose of A), identity padding.
__global__ __launch_bounds__(kThreads) void k_build_pw_transpose(const double *const *__restrict__ pos_all,
                                                                 double *const *__restrict__ m_all, int n, int np,
                                                                 const int4 *__restrict__ kvec, double twopi_l) {
    const double *pos = pos_all[blockIdx.z];
    double *m = m_all[blockIdx.z];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= np) return;
    double v;
    if (i < n && j < n) v = pw_orbital(kvec[j], twopi_l, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    else v = (i == j) ? 1.0 : 0.0;
    m[(size_t)j * np + i] = v;
}

hipError_t launch_build_pw_transpose(const double *const *pos_dev, double *const *m_dev, int ndesc, int n, int np,
                                     const int4 *kvec, double twopi_over_l, hipStream_t s) {
    hipLaunchKernelGGL(k_build_pw_transpose, dim3((np + kThreads - 1) / kThreads, np, ndesc), dim3(kThreads), 0, s,
                       pos_dev, m_dev, n, np, kvec, twopi_over_l);
    return hipGetLastError();
}

// rows[c][j] = phi_j(pos_c) for c < count, j < n (FP64).
__global__ __launch_bounds__(kThreads) void k_pw_rows(const double *__restrict__ pos, double *__restrict__ rows, int n,
                                                      const int4 *__restrict__ kvec, double twopi_l) {
    const int c = blockIdx.y;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    rows[(size_t)c * n + j] = pw_orbital(kvec[j], twopi_l, pos[3 * c], pos[3 * c + 1], pos[3 * c + 2]);
}

hipError_t launch_pw_rows(const double *pos_dev, double *rows_dev, int n, int count, const int4 *kvec,
                          double twopi_over_l, hipStream_t s) {
    hipLaunchKernelGGL(k_pw_rows, dim3((n + kThreads - 1) / kThreads, count), dim3(kThreads), 0, s, pos_dev, rows_dev,
                       n, kvec, twopi_over_l);
    return hipGetLastError();
}

// After a recompute: drift = running - fresh, then re-base.
template <typename T>
__global__ void k_reset_state(const DetDesc<T> *__restrict__ d, const GjDesc *__restrict__ gj, double *drift,
                              int ndesc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndesc) return;
    DetState *st = d[i].st;
    const double fresh = *gj[i].logdet;
    if (drift) drift[i] = st->logdet - fresh;
    st->logdet = fresh;
    st->sign = *gj[i].sign;
}

template <typename T>
hipError_t launch_reset_state(const DetDesc<T> *d, const GjDesc *gj, double *drift, int ndesc, hipStream_t s) {
    hipLaunchKernelGGL((k_reset_state<T>), dim3((ndesc + 63) / 64), dim3(64), 0, s, d, gj, drift, ndesc);
    return hipGetLastError();
}
template hipError_t launch_reset_state<float>(const DetDesc<float> *, const GjDesc *, double *, int, hipStream_t);
template hipError_t launch_reset_state<double>(const DetDesc<double> *, const GjDesc *, double *, int, hipStream_t);

// ------------------------------------------------- sampled inverse residual
// Sec. III checks the determinants against a direct calculation; between FP64
// recomputes the batched form checks its inverse X against the Slater matrix
// itself (rebuilt in FP64 from the positions) on a rotating sample of rows.
// With S samples, stride = n / S and t = sweep mod stride:
//   right: rows e_s = s * stride + t of A X - I,
//          res[s][j] = phi(r_{e_s}) . BT[j, :] - delta(j, e_s)
//          (BT = X^T row-major: column j of X is row j of BT);
//   left:  rows i = t * S + s of X A - I,
//          res[s][j] = sum_k BT[k][i] phi_j(r_k) - delta(i, j).
// Both are skinny products on FP64 matrix cores (X converted exactly to FP64)
// and end in a max |res| per determinant, kept as the bit pattern of a
// non-negative double (those order like unsigned integers; a non-finite entry
// counts as +inf).
//
// Operand layout of v_mfma_f64_16x16x4f64 with the k index permuted: at step
// s (0..3) of a 16-wide k block c0, lane l supplies A[l%16][k] and B[k][l%16]
// for k = c0 + 4 (l/16) + s, so each lane reads 4 consecutive k of its own
// row; every k of the block is used exactly once, which is all the product
// needs.

__device__ __forceinline__ double resid_abs(double v) {
    const double av = fabs(v);
    return av <= 1.79769313486231570815e308 ? av : __builtin_inf();
}

__device__ __forceinline__ void resid_store_max(double m, unsigned long long *out) {
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// rows[d][s][c] = phi_c(r_{e_s}) for c < n, 0 for n <= c < np and for the
// padding samples s >= S (eidx = -1 there); grid (ndesc, SP).  Also clears
// the determinant's result word.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resid_rows(const DetDesc<T> *__restrict__ descs, int n, int np, int S,
                                                         int SP, const int4 *__restrict__ kvec, double twopi_l,
                                                         double *__restrict__ rows, int *__restrict__ eidx,
                                                         unsigned long long *__restrict__ out_bits) {
    const DetDesc<T> d = descs[blockIdx.x];
    const int s = blockIdx.y;
    const int stride = n / S;
    const int e = s < S ? s * stride + (int)(d.st->sweep % (long long)stride) : -1;
    double *r = rows + ((size_t)blockIdx.x * SP + s) * np;
    if (threadIdx.x == 0) {
        eidx[blockIdx.x * SP + s] = e;
        if (s == 0) out_bits[blockIdx.x] = 0ull;
    }
    const double x = e >= 0 ? d.pos[3 * e + 0] : 0.0, y = e >= 0 ? d.pos[3 * e + 1] : 0.0,
                 z = e >= 0 ? d.pos[3 * e + 2] : 0.0;
    for (int c = threadIdx.x; c < np; c += kThreads)
        r[c] = (e >= 0 && c < n) ? pw_orbital(kvec[c], twopi_l, x, y, z) : 0.0;
}

// Four consecutive elements of a row, as FP64.
template <typename T> struct Quad;
template <> struct Quad<float> {
    static __device__ __forceinline__ void load(const float *p, double (&v)[4]) {
        const f32x4 x = *reinterpret_cast<const DSU_GLOBAL f32x4 *>(gmem(p));
        v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
    }
};
template <> struct Quad<double> {
    static __device__ __forceinline__ void load(const double *p, double (&v)[4]) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 a = *reinterpret_cast<const DSU_GLOBAL d2 *>(gmem(p));
        const d2 b = *reinterpret_cast<const DSU_GLOBAL d2 *>(gmem(p + 2));
        v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
    }
};

// Right residual: one wave per (64 rows j of BT, determinant); the 64 x SP
// block BT[j, :] . rows[s, :] as 4 x SP/16 tiles, operands straight from
// global memory (BT streamed once, the sample rows from L2), the next block's
// loads issued before the current block's products.
template <typename T, int SP>
__global__ __launch_bounds__(64) void k_resid_prod(const DetDesc<T> *__restrict__ descs, int n, int np, int nblk,
                                                   const double *__restrict__ rows, const int *__restrict__ eidx,
                                                   unsigned long long *__restrict__ out_bits) {
    constexpr int NT = SP / 16;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int di = blk / nblk, j0 = (blk % nblk) * 64;
    const DetDesc<T> d = descs[di];
    const int lane = threadIdx.x, lr = lane & 15, lk = lane >> 4;
    const T *bp = d.bt + (size_t)(j0 + lr) * np + 4 * lk;
    const double *rp = rows + ((size_t)di * SP + lr) * np + 4 * lk;
    f64x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f64x4{0, 0, 0, 0};
    double a[4][4], b[NT][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) Quad<T>::load(bp + (size_t)16 * m * np, a[m]);
#pragma unroll
    for (int t = 0; t < NT; ++t) Quad<double>::load(rp + (size_t)16 * t * np, b[t]);
    for (int c0 = 0; c0 < np; c0 += 16) {
        double an[4][4], bn[NT][4];
        const int cn = c0 + 16 < np ? c0 + 16 : c0;
#pragma unroll
        for (int m = 0; m < 4; ++m) Quad<T>::load(bp + (size_t)16 * m * np + cn, an[m]);
#pragma unroll
        for (int t = 0; t < NT; ++t) Quad<double>::load(rp + (size_t)16 * t * np + cn, bn[t]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[m][t] = Mma<double>::mma(a[m][s], b[t][s], acc[m][t]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[m][q] = an[m][q];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) b[t][q] = bn[t][q];
    }
    // D[i][n] of tile (m, t): i = row0 + q * row_step (rows of BT), n = lr (sample)
    double mx = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int e = eidx[di * SP + 16 * t + lr];
        if (e < 0) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + 16 * m + Mma<double>::row0(lane) + q * Mma<double>::row_step;
                if (j < n) mx = fmax(mx, resid_abs(acc[m][t][q] - (j == e ? 1.0 : 0.0)));
            }
    }
    resid_store_max(mx, out_bits + di);
}

template <typename T>
hipError_t launch_resid(const DetDesc<T> *d, int ndesc, int n, int np, int samples, const int4 *kvec,
                        double twopi_over_l, double *rows, int *eidx, unsigned long long *out_bits, hipStream_t s) {
    if (samples < 1 || samples > 64 || samples > n) return hipErrorInvalidValue;
    const int sp = samples <= 16 ? 16 : (samples <= 32 ? 32 : 64);
    hipLaunchKernelGGL((k_resid_rows<T>), dim3(ndesc, sp), dim3(kThreads), 0, s, d, n, np, samples, sp, kvec,
                       twopi_over_l, rows, eidx, out_bits);
    const int nblk = np / 64;
    const dim3 grid(ndesc * nblk);
    if (sp == 16)
        hipLaunchKernelGGL((k_resid_prod<T, 16>), grid, dim3(64), 0, s, d, n, np, nblk, rows, eidx, out_bits);
    else if (sp == 32)
        hipLaunchKernelGGL((k_resid_prod<T, 32>), grid, dim3(64), 0, s, d, n, np, nblk, rows, eidx, out_bits);
    else
        hipLaunchKernelGGL((k_resid_prod<T, 64>), grid, dim3(64), 0, s, d, n, np, nblk, rows, eidx, out_bits);
    return hipGetLastError();
}
template hipError_t launch_resid<float>(const DetDesc<float> *, int, int, int, int, const int4 *, double, double *,
                                        int *, unsigned long long *, hipStream_t);
template hipError_t launch_resid<double>(const DetDesc<double> *, int, int, int, int, const int4 *, double, double *,
                                         int *, unsigned long long *, hipStream_t);

// Left residual: one workgroup per (256 columns j, determinant), wave w on
// columns 64w .. 64w+63, all S rows i0 .. i0+S-1 (i0 = t S) as SP/16 x 4
// tiles per wave.  A operand X[i][k] = BT[k][i0+i] (16 consecutive elements
// of row k per load); B operand A[k][j] = phi_j(r_k) evaluated by the lane
// from per-electron phase tables in LDS: with q = 2 pi / L,
// exp(i q n.r) = Ex^nx Ey^ny Ez^nz and E^-m = conj(E^m), so 16 electrons need
// 3 (nmax + 1) sincos each for all 256 columns (the workgroup fills the table
// together), and an orbital is two complex products.  nmax <= kPwTab (true
// for every n the batched form takes: nmax is about (3 n / 8 pi)^(1/3)).
template <typename T, int SP>
__global__ __launch_bounds__(kThreads) void k_resid_left(const DetDesc<T> *__restrict__ descs, int n, int np, int S,
                                                         int nblk, const int4 *__restrict__ kvec, double twopi_l,
                                                         int nmax, unsigned long long *__restrict__ out_bits) {
#pragma clang fp contract(off)
    constexpr int NT = SP / 16;
    constexpr int XL = (16 * SP + kThreads - 1) / kThreads;  // X elements each thread stages per step
    __shared__ double s_c[16][3][kPwTab + 1], s_s[16][3][kPwTab + 1];
    __shared__ double s_x[16][SP + 1];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int di = blk / nblk;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    const int j0 = (blk % nblk) * 256 + 64 * wave;
    const DetDesc<T> d = descs[di];
    DSU_GLOBAL const T *bt = gmem(d.bt);
    DSU_GLOBAL const double *pos = gmem(d.pos);
    const int stride = n / S;
    const int i0 = (int)(d.st->sweep % (long long)stride) * S;
    int4 kv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int j = j0 + 16 * u + lr;
        kv[u] = j < n ? kvec[j] : int4{0, 0, 0, 3};
    }
    f64x4 acc[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = f64x4{0, 0, 0, 0};
    // X[i][k] = BT[k][i0 + i] for the 16 electrons of a step: element v of the
    // step is (e = v / SP, i = v % SP); loads of the next step are in flight
    // while the current one is computed
    T xr[XL];
    auto load_x = [&](int c) {
#pragma unroll
        for (int q = 0; q < XL; ++q) {
            const int v = tid + q * kThreads, e = v / SP, i = v % SP, k = c + e;
            const bool in = v < 16 * SP && k < n && i < S;
            xr[q] = bt[in ? (size_t)k * np + i0 + i : 0];
            if (!in) xr[q] = T(0);
        }
    };
    load_x(0);
#pragma unroll 1
    for (int c0 = 0; c0 < n; c0 += 16) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < XL; ++q) {
            const int v = tid + q * kThreads;
            if (v < 16 * SP) s_x[v / SP][v % SP] = (double)xr[q];
        }
        if (c0 + 16 < n) load_x(c0 + 16);
        for (int v = tid; v < 16 * 3 * (nmax + 1); v += kThreads) {
            const int e = v / (3 * (nmax + 1)), r = v % (3 * (nmax + 1)), ax = r / (nmax + 1), m = r % (nmax + 1);
            const int k = c0 + e < n ? c0 + e : 0;
            double sn, cs;
            sincos(twopi_l * ((double)m * pos[3 * k + ax]), &sn, &cs);
            s_c[e][ax][m] = cs;
            s_s[e][ax][m] = sn;
        }
        __syncthreads();
        // one electron of the lane's four at a time: its four orbitals, then
        // the step's products (keeps the live registers to one step's operands)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = 4 * lk + s;
            const bool kin = c0 + e < n;
            double bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double o;
                if (kv[u].w == 0) {
                    o = 1.0;
                } else if (kv[u].w == 3) {
                    o = 0.0;
                } else {
                    const int ax_n[3] = {kv[u].x, kv[u].y, kv[u].z};
                    double re = 1.0, im = 0.0;
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const int m = ax_n[ax] < 0 ? -ax_n[ax] : ax_n[ax];
                        const double fc = s_c[e][ax][m];
                        const double fs = ax_n[ax] < 0 ? -s_s[e][ax][m] : s_s[e][ax][m];
                        const double tt = re * fc - im * fs;
                        im = re * fs + im * fc;
                        re = tt;
                    }
                    o = kv[u].w == 1 ? re : im;
                }
                bv[u] = kin ? o : 0.0;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double a = s_x[e][16 * t + lr];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[t][u] = Mma<double>::mma(a, bv[u], acc[t][u]);
            }
        }
    }
    double mx = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int j = j0 + 16 * u + lr;
        if (j >= n) continue;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * t + Mma<double>::row0(lane) + q * Mma<double>::row_step;
                if (i < S) mx = fmax(mx, resid_abs(acc[t][u][q] - (i0 + i == j ? 1.0 : 0.0)));
            }
    }
    resid_store_max(mx, out_bits + di);
}

__global__ void k_zero_u64(unsigned long long *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

template <typename T>
hipError_t launch_resid_left(const DetDesc<T> *d, int ndesc, int n, int np, int samples, const int4 *kvec,
                             double twopi_over_l, int nmax, unsigned long long *out_bits, hipStream_t s) {
    if (samples < 1 || samples > 64 || samples > n || nmax > kPwTab) return hipErrorInvalidValue;
    const int sp = samples <= 16 ? 16 : (samples <= 32 ? 32 : 64);
    hipLaunchKernelGGL(k_zero_u64, dim3((ndesc + 255) / 256), dim3(256), 0, s, out_bits, ndesc);
    const int nblk = (np + 255) / 256;
    const dim3 grid(ndesc * nblk);
#define DSU_L(SPV)                                                                                              \
    if (sp == SPV)                                                                                              \
        hipLaunchKernelGGL((k_resid_left<T, SPV>), grid, dim3(kThreads), 0, s, d, n, np, samples, nblk, kvec,   \
                           twopi_over_l, nmax, out_bits);
    DSU_L(16) DSU_L(32) DSU_L(64)
#undef DSU_L
    return hipGetLastError();
}
template hipError_t launch_resid_left<float>(const DetDesc<float> *, int, int, int, int, const int4 *, double, int,
                                             unsigned long long *, hipStream_t);
template hipError_t launch_resid_left<double>(const DetDesc<double> *, int, int, int, int, const int4 *, double, int,
                                              unsigned long long *, hipStream_t);

}  // namespace dsu
