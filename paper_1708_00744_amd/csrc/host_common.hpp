// host_common.hpp -- host-side helpers shared by the walker, batch and
// server implementations of the C ABI (error reporting, device allocation,
// the Gauss-Jordan workspace, the plane-wave table).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dsu.h"
#include "dsu_internal.hpp"

namespace dsu {

// Record `code` and a printf-style message as the thread's last error.
int fail(int code, const char *fmt, ...);

#define HIPCHK(x)                                                                                           \
    do {                                                                                                    \
        hipError_t e_ = (x);                                                                                \
        if (e_ != hipSuccess)                                                                               \
            return ::dsu::fail(e_ == hipErrorOutOfMemory ? DSU_ENOMEM : DSU_EDEVICE, "%s: %s (%s:%d)", #x,  \
                               hipGetErrorString(e_), __FILE__, __LINE__);                                  \
    } while (0)
#define CHK(x)                       \
    do {                             \
        int r_ = (x);                \
        if (r_ != DSU_OK) return r_; \
    } while (0)

// Padded delay: the smallest of 16, 32, 64, 128, 256 that holds k.
int kpad(int k);
// hipMalloc + zero fill, complete before return.
int dev_alloc(void **p, size_t bytes);
template <typename P> inline int dalloc(P **p, size_t count) {
    return dev_alloc(reinterpret_cast<void **>(p), count * sizeof(P));
}
void dfree(void *p);
int make_stream(void *given, hipStream_t *s, bool *own);
inline size_t elem_size(int prec) { return prec == DSU_FP64 ? sizeof(double) : sizeof(float); }

// Workspace of the blocked Gauss-Jordan inversion for `g` matrices at once.
struct GjWork {
    int g = 0, np = 0, nb = 64;  // nb: panel columns the buffers hold
    GjTiles tiles;               // blocking used by invert()
    double *m = nullptr, *m2 = nullptr, *panel = nullptr, *w = nullptr, *logdet = nullptr,
           *pmax = nullptr;
    int *piv = nullptr, *perm = nullptr, *rowsrc = nullptr, *sign = nullptr, *status = nullptr;
    double *panel_b = nullptr, *q2 = nullptr;  // panel pairs
    int *rowsrc_b = nullptr, *qrow = nullptr;
    GjDesc *gdesc = nullptr;   // set A: m = first buffer (the input, see mptr)
    GjDesc *gdesc_b = nullptr; // set B: the buffers exchanged
    double **mptr = nullptr;   // per matrix: the input buffer (set A's m)
    // Invert the first `cnt` matrices (inputs in mptr); returns the descriptor
    // set holding the result.
    hipError_t invert(int cnt, int n, hipStream_t s, const GjDesc **final_set) const {
        return launch_gj_invert(gdesc, gdesc_b, cnt, n, np, tiles, s, final_set);
    }
    // Allocate for `groups` matrices; with `block` (block_bytes(groups, np_, n)
    // bytes of device memory the caller owns) every buffer is carved from it
    // and nothing is allocated.
    int alloc(int groups, int np_, int n, void *block = nullptr);
    void release();
    static size_t bytes_per(int np_, int n);
    static size_t block_bytes(int groups, int np_, int n);
    bool owned = true;
};

}  // namespace dsu
