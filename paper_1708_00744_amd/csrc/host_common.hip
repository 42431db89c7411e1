// host_common.hip -- implementation of host_common.hpp.
#include "host_common.hpp"

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

static int gj_panel_width(int n) { return n >= 512 ? 64 : (n >= 64 ? 32 : 16); }

size_t GjWork::bytes_per(int np_, int n) {
    const size_t nb_ = gj_panel_width(n);
    return (size_t)np_ * np_ * 8 + (size_t)np_ * nb_ * 8 * 3 + (size_t)np_ * 8 + 128;
}

int GjWork::alloc(int groups, int np_, int n) {
    g = groups;
    np = np_;
    nb = gj_panel_width(n);
    const size_t np2 = (size_t)np * np;
    CHK(dalloc(&m, np2 * g));
    CHK(dalloc(&panel, (size_t)np * nb * g));
    CHK(dalloc(&w, (size_t)np * nb * g));
    CHK(dalloc(&q, (size_t)np * nb * g));
    CHK(dalloc(&logdet, g));
    CHK(dalloc(&piv, (size_t)np * g));
    CHK(dalloc(&perm, (size_t)np * g));
    CHK(dalloc(&sign, g));
    CHK(dalloc(&status, g));
    CHK(dalloc(&pmax, g));
    CHK(dalloc(&gdesc, g));
    CHK(dalloc(&rdesc, g));
    CHK(dalloc(&mptr, g));
    std::vector<GjDesc> gd(g);
    std::vector<RankDesc> rd(g);
    std::vector<double *> mp(g);
    for (int i = 0; i < g; ++i) {
        gd[i] = GjDesc{m + np2 * i, panel + (size_t)np * nb * i, w + (size_t)np * nb * i, q + (size_t)np * nb * i,
                       piv + (size_t)np * i, perm + (size_t)np * i, logdet + i, sign + i, status + i, pmax + i};
        rd[i] = RankDesc{gd[i].m, gd[i].w, gd[i].q};
        mp[i] = gd[i].m;
    }
    HIPCHK(hipMemcpy(gdesc, gd.data(), sizeof(GjDesc) * g, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(rdesc, rd.data(), sizeof(RankDesc) * g, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(mptr, mp.data(), sizeof(double *) * g, hipMemcpyHostToDevice));
    return DSU_OK;
}

void GjWork::release() {
    for (void *p : {(void *)m, (void *)panel, (void *)w, (void *)q, (void *)logdet, (void *)piv, (void *)perm,
                    (void *)sign, (void *)status, (void *)gdesc, (void *)rdesc, (void *)mptr, (void *)pmax})
        dfree(p);
    m = panel = w = q = logdet = pmax = nullptr;
    piv = perm = sign = status = nullptr;
    gdesc = nullptr;
    rdesc = nullptr;
    mptr = nullptr;
}

}  // namespace dsu

extern "C" const char *dsu_last_error(void) { return dsu::last_error(); }
extern "C" int dsu_version(void) { return 100; }
