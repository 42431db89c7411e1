// dsu_server.hip -- serving pool (continuous batching of walkers of mixed n).
#include <hip/hip_runtime.h>

#include "dsu.h"

struct dsu_server {
    int dummy;
};

extern "C" int dsu_server_create(int32_t, int32_t, double, size_t, int32_t, dsu_server **out) {
    if (out) *out = nullptr;
    return DSU_ESTATE;
}
extern "C" int dsu_server_destroy(dsu_server *) { return DSU_ESTATE; }
extern "C" int dsu_server_run(dsu_server *, const dsu_request *, int32_t, dsu_result *, double *, int64_t, int64_t *) {
    return DSU_ESTATE;
}
