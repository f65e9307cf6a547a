// Serving runtime (continuous batching) -- placeholder until implemented.
#include "internal.hpp"

using namespace br;

extern "C" {
int br_server_create(br_server**, int, int64_t, int32_t) { return fail(BR_EINVAL, "server: not built yet"); }
int br_submit(br_server*, const int32_t*, int64_t, int32_t, uint64_t*) { return fail(BR_EINVAL, "server: not built yet"); }
int br_poll(br_server*, uint64_t, int32_t*, int64_t, int64_t*, int*) { return fail(BR_EINVAL, "server: not built yet"); }
int br_wait(br_server*, uint64_t, int32_t*, int64_t, int64_t*) { return fail(BR_EINVAL, "server: not built yet"); }
int br_server_stats(br_server*, br_server_stats_t*, int) { return fail(BR_EINVAL, "server: not built yet"); }
int br_server_destroy(br_server*) { return BR_OK; }
}
