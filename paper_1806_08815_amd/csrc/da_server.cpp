// da_server.cpp -- continuous-batching server (entry points; not yet running jobs).
#include "da_runtime.h"

using namespace dapt;

extern "C" {
int da_server_create(size_t, const da_server_opts *, da_server **out) {
    if (out) *out = nullptr;
    return fail(nullptr, DA_EINVAL, "server not available in this build");
}
int da_submit(da_server *, const da_job *, uint64_t *) { return fail(nullptr, DA_EINVAL, "no server"); }
int da_poll(da_server *, uint64_t, da_result *, da_job_stats *) { return fail(nullptr, DA_ENOTFOUND, "no server"); }
int da_wait(da_server *, uint64_t, da_result *, da_job_stats *) { return fail(nullptr, DA_ENOTFOUND, "no server"); }
int64_t da_job_footprint(int32_t, int32_t, int32_t, int32_t) { return -1; }
void da_server_destroy(da_server *) {}
}
