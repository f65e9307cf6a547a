// Batched bridge queries (first version: one br_bridges_find per graph).
#include <algorithm>

#include "internal.hpp"

namespace br {
void batched_release(br_ctx*) {}
}  // namespace br

using namespace br;

extern "C" {

int32_t br_batched_max_v(void) { return 4096; }

int br_bridges_find_batched(br_ctx* c, const int32_t* d_edges, const int64_t* h_edge_off, const int32_t* h_V,
                            int32_t G, int32_t chunk_edges, int32_t* h_bridges, int64_t cap, int64_t* h_bridge_off,
                            void* stream) {
    if (!c || !h_edge_off || !h_V || !h_bridge_off || G < 0 || chunk_edges < 0 || cap < 0 || (cap > 0 && !h_bridges))
        return fail(BR_EINVAL, "br_bridges_find_batched: bad argument");
    h_bridge_off[0] = 0;
    int64_t total = 0;
    std::vector<int32_t> tmp;
    int status = BR_OK;
    for (int32_t g = 0; g < G; g++) {
        const int64_t E = h_edge_off[g + 1] - h_edge_off[g];
        if (E < 0) return fail(BR_EINVAL, "batched: offsets decrease at graph %d", g);
        const int32_t V = h_V[g];
        tmp.resize(2 * (size_t)std::max(V, 1));
        int64_t n = 0;
        int rc = br_bridges_find(c, d_edges + 2 * h_edge_off[g], E, V, 1, tmp.data(), std::max(V, 1), &n, stream);
        if (rc) return rc;
        if (total + n <= cap) std::copy(tmp.begin(), tmp.begin() + 2 * n, h_bridges + 2 * total);
        else status = BR_ECAP;
        total += n;
        h_bridge_off[g + 1] = total;
    }
    if (status) return fail(BR_ECAP, "batched: %lld bridges, capacity %lld", (long long)total, (long long)cap);
    return BR_OK;
}

}  // extern "C"
