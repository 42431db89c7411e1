// host_common.hip -- implementation of host_common.hpp.
#include "host_common.hpp"

#include <utility>

#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace dsu {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }

int kpad(int k) {
    int p = 16;
    while (p < k) p *= 2;
    return p;
}

int dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return DSU_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(DSU_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    // hipMemset runs on the null stream, which does not order with the
    // library's non-blocking streams: wait for it before anyone uses *p.
    e = hipMemset(*p, 0, bytes);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return fail(DSU_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
    return DSU_OK;
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

int make_stream(void *given, hipStream_t *s, bool *own) {
    if (given) {
        *s = (hipStream_t)given;
        *own = false;
        return DSU_OK;
    }
    HIPCHK(hipStreamCreateWithFlags(s, hipStreamNonBlocking));
    *own = true;
    return DSU_OK;
}

// Panel buffers hold the widest panel (64 columns), so any blocking fits;
// a panel pair adds the second panel buffer, its pivot rows and row maps.
static constexpr int kGjPanelMax = 64;

size_t GjWork::bytes_per(int np_, int n) {
    (void)n;
    const size_t nb_ = kGjPanelMax;
    return (size_t)np_ * np_ * 8 * 2 + (size_t)np_ * nb_ * 8 * 4 + (size_t)np_ * 16 + nb_ * 4 + 128;
}

// Pieces of the workspace in carve order (bytes, each 256-byte aligned).
static constexpr int kGjPieces = 18;
static void gj_pieces(int g, int np, int nb, size_t out[kGjPieces]) {
    const size_t np2 = (size_t)np * np;
    const size_t d = sizeof(double), i = sizeof(int);
    const size_t v[kGjPieces] = {np2 * g * d,          np2 * g * d,        (size_t)np * nb * g * d,
                                 (size_t)np * nb * g * d, (size_t)g * d,   (size_t)np * g * i,
                                 (size_t)np * g * i,   (size_t)np * g * i, (size_t)g * i,
                                 (size_t)g * i,        (size_t)g * d,      sizeof(GjDesc) * g,
                                 sizeof(GjDesc) * g,   sizeof(double *) * g, (size_t)np * nb * g * d,
                                 (size_t)np * nb * g * d, (size_t)np * g * i, (size_t)nb * g * i};
    for (int k = 0; k < kGjPieces; ++k) out[k] = (v[k] + 255) & ~(size_t)255;
}

size_t GjWork::block_bytes(int groups, int np_, int n) {
    size_t p[kGjPieces], b = 0;
    (void)n;
    gj_pieces(groups, np_, kGjPanelMax, p);
    for (size_t x : p) b += x;
    return b;
}

int GjWork::alloc(int groups, int np_, int n, void *block) {
    g = groups;
    np = np_;
    nb = kGjPanelMax;
    tiles = gj_tiles_default(n, np_);
    owned = block == nullptr;
    const size_t np2 = (size_t)np * np;
    void **dst[kGjPieces] = {(void **)&m,      (void **)&m2,    (void **)&panel, (void **)&w,
                             (void **)&logdet, (void **)&piv,   (void **)&perm,  (void **)&rowsrc,
                             (void **)&sign,   (void **)&status, (void **)&pmax, (void **)&gdesc,
                             (void **)&gdesc_b, (void **)&mptr, (void **)&panel_b, (void **)&q2,
                             (void **)&rowsrc_b, (void **)&qrow};
    size_t p[kGjPieces];
    gj_pieces(g, np, nb, p);
    char *c = static_cast<char *>(block);
    if (c) HIPCHK(hipMemset(c, 0, block_bytes(groups, np_, n)));
    for (int k = 0; k < kGjPieces; ++k) {
        if (c) {
            *dst[k] = c;
            c += p[k];
        } else {
            CHK(dev_alloc(dst[k], p[k]));
        }
    }
    std::vector<GjDesc> ga(g), gb(g);
    std::vector<double *> mp(g);
    for (int i = 0; i < g; ++i) {
        ga[i] = GjDesc{m + np2 * i,           m2 + np2 * i,       panel + (size_t)np * nb * i,
                       w + (size_t)np * nb * i, piv + (size_t)np * i, perm + (size_t)np * i,
                       rowsrc + (size_t)np * i, logdet + i,         sign + i,
                       status + i,              pmax + i,           panel_b + (size_t)np * nb * i,
                       q2 + (size_t)np * nb * i, rowsrc_b + (size_t)np * i, qrow + (size_t)nb * i};
        gb[i] = ga[i];
        std::swap(gb[i].m, gb[i].m2);
        mp[i] = ga[i].m;
    }
    HIPCHK(hipMemcpy(gdesc, ga.data(), sizeof(GjDesc) * g, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(gdesc_b, gb.data(), sizeof(GjDesc) * g, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(mptr, mp.data(), sizeof(double *) * g, hipMemcpyHostToDevice));
    return DSU_OK;
}

void GjWork::release() {
    if (owned)
        for (void *p : {(void *)m, (void *)m2, (void *)panel, (void *)w, (void *)logdet, (void *)piv,
                        (void *)perm, (void *)rowsrc, (void *)sign, (void *)status, (void *)gdesc, (void *)gdesc_b,
                        (void *)mptr, (void *)pmax, (void *)panel_b, (void *)q2, (void *)rowsrc_b, (void *)qrow})
            dfree(p);
    m = m2 = panel = w = logdet = pmax = panel_b = q2 = nullptr;
    piv = perm = rowsrc = sign = status = rowsrc_b = qrow = nullptr;
    gdesc = gdesc_b = nullptr;
    mptr = nullptr;
}

}  // namespace dsu

extern "C" const char *dsu_last_error(void) { return dsu::last_error(); }
extern "C" int dsu_version(void) { return 100; }
