// C ABI of libbridges: contexts, workspace, the phase tree orchestration
// (paper, Section III) and the synchronous bridge query.
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "internal.hpp"

namespace br {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? BR_ENOMEM : BR_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

int32_t block_size();
int32_t tile_size();

int g_cus = 0;
int g_max_lds = 64 * 1024;

// BR_SOLO (1 on, 0 off, unset: by size) and BR_SOLO_TOP (merge levels inside
// the one-workgroup-per-node kernel) override the plan's choice
static int env_int(const char* name, int dflt) {
    const char* s = getenv(name);
    return s && *s ? atoi(s) : dflt;
}

std::string plain_tune_key(int device, int64_t E, int32_t V, int32_t M) {
    return arch_name(device) + "|plain|v" + std::to_string(log2_bucket(V)) + "|e" + std::to_string(log2_bucket(E)) +
           "|m" + std::to_string(M);
}

Plan plan_for(int device, int64_t E, int32_t V, int32_t M) {
    TuneEntry t;
    const bool have = tune_get(plain_tune_key(device, E, V, M), t);
    return make_plan(E, V, M, true, have ? &t : nullptr);
}

Plan make_plan(int64_t E, int32_t V, int32_t M, bool allow_solo, const TuneEntry* tuned) {
    auto knob = [&](const char* env, const char* name, int dflt) {
        int v = dflt;
        if (tuned) {
            auto it = tuned->find(name);
            if (it != tuned->end()) v = (int)it->second;
        }
        return env_int(env, v);
    };
    Plan P;
    P.E = E;
    P.V = V;
    P.M = M;
    while ((int64_t(1) << P.rounds) < M) P.rounds++;
    // phase-0 tiles fill the LDS stage; merge rounds size their own tiles
    P.tile = tile_size();
    const int64_t per = (E + M - 1) / M;   // largest chunk
    P.tpc = (int32_t)std::max<int64_t>(1, (per + P.tile - 1) / P.tile);
    P.xcd_map = M >= 8 ? 1 : 0;
    const int64_t chunk_slots = P.xcd_map ? 8 * ((M + 7) / 8) : M;
    P.blocks0 = E > 0 ? chunk_slots * P.tpc : 0;
    // Stages within each chunk, separated by a full path compression: the
    // first 2V edges form most components (many hooks, contention), the next
    // ones up to 8V mostly finish F', and the rest is then mostly rejected by
    // comparing the endpoints' representatives.  Chunks of at most 2V edges
    // run in one stage.
    P.stages = {0};
    for (int64_t b : {2 * (int64_t)V, 8 * (int64_t)V})
        if (b < per) P.stages.push_back(b);
    P.stages.push_back(per);
    // state layout: one vertex per 32 bytes while all M states stay within
    // 128 MB (measured faster at M = 1, 16 and 32 on the dense workload),
    // packed 8 bytes per vertex otherwise (more chunks: capacity wins)
    P.qs = (int64_t)M * V * 32 <= (int64_t(128) << 20) ? 8 : 2;
    auto lo = [&](int64_t i) { return i * (E / M) + (i * (E % M)) / M; };
    const int64_t bound = 2 * (int64_t(V) - 1);
    P.off.resize(M);
    P.cap.resize(M);
    int64_t acc = 0;
    for (int64_t i = 0; i < M; i++) {
        int64_t span = M;   // node 0 ends up covering every chunk
        if (i != 0) {
            int z = __builtin_ctzll((unsigned long long)i);
            span = std::min<int64_t>(int64_t(1) << z, M - i);
        }
        const int64_t edges = lo(std::min<int64_t>(M, i + span)) - lo(i);
        P.cap[i] = std::min(edges, bound);
        P.off[i] = acc;
        acc += P.cap[i];
    }
    P.cert_pairs = acc;
    // One workgroup per node when there is at least one chunk per workgroup
    // in flight (chunks of at most a few V edges: the hook-bound regime) and
    // the LDS bitmaps of the hooks fit: merge levels 1..top inside that
    // kernel, while each level still has about a merge per workgroup.
    const int cus = g_cus > 0 ? g_cus : 256;
    P.tile0_max = knob("BR_TILE0", "tile", 0);
    P.prem = knob("BR_PREM", "prem", 0) != 0;
    // the whole tree in LDS: V within a workgroup's LDS, chunks short enough
    // for one CU each (a CU offers about 10^9 edges/s in LDS)
    const int lds = knob("BR_LDS", "lds", -1);
    if (allow_solo && E > 0 && V <= batched_max_v_big() && M < (1 << 20) &&
        (lds == 1 || (lds < 0 && per <= (int64_t(1) << 18)))) {
        P.lds = true;
        P.lds_big = V > batched_max_v_dev();
        P.lds_blocks = (int32_t)std::min<int64_t>(M, (int64_t)cus * (P.lds_big ? 1 : batched_blocks_per_cu()));
        P.lds_counters = (int64_t)P.rounds * (((int64_t)M + 1) / 2) + 2;
        return P;
    }
    const int want = knob("BR_SOLO", "solo", -1);
    if (allow_solo && E > 0 && V <= solo_max_v() &&
        (want == 1 || (want < 0 && M >= cus && per <= (int64_t)V && V >= (1 << 17)))) {
        P.solo = true;
        P.solo_variant = std::max(0, std::min(knob("BR_SOLO_VARIANT", "variant", 2), solo_variants() - 1));
        // 1,024 threads of workers per CU where registers and LDS hold them
        // (large workload, M = 4096: 64 → 256 workers of 1,024 threads
        // 276 → 149 ms, but 768 workers of 512 threads slower than 512)
        // written-bits maps in LDS where they fit beside the claim tables
        P.solo_wm = knob("BR_SOLO_WM", "wm", 1) != 0 && solo_wm_fits(V);
        const int fit = std::min(solo_blocks_per_cu(P.solo_variant, V, P.solo_wm),
                                 std::max(1, 1024 / solo_block(P.solo_variant)));
        const int wpc = std::max(1, std::min(knob("BR_SOLO_WPC", "wpc", fit), fit));
        // every worker needs a slot of 8 V bytes; all slots within 8 GiB
        const int64_t max_slots = std::max<int64_t>(1, (int64_t(8) << 30) / (8 * (int64_t)V));
        P.workers = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)knob("BR_SOLO_WORKERS", "workers", cus * wpc),
                                                                  (int64_t)cus * wpc, max_slots}));
        // merge levels inside the kernel while they still hold four merges
        // per worker (measured on the large workload at M = 4096: two levels
        // 193 ms, three 206 ms, four 203 ms, five 210 ms)
        int top = 0;
        while (top < P.rounds && (int64_t)(M >> (top + 1)) >= 4 * (int64_t)P.workers) top++;
        P.solo_top = std::max(0, std::min(P.rounds, knob("BR_SOLO_TOP", "top", top)));
        P.nslots = (int)std::min<int64_t>(3 * (int64_t)P.workers, max_slots);
        P.solo_cmp = std::max(1, knob("BR_SOLO_CMP", "cmp", 16));
        // phase 0 reads each chunk bucketed by (smaller endpoint / V/8,
        // larger endpoint / V/128): large workload, M = 4096, merge level 1
        // in the kernel: 190.0 ms per query in input order, 181.6 with 256
        // buckets by the smaller endpoint, 175.2 with 1,024 by the larger,
        // 173.8 / 170.5 / 169.7 with 4x64 / 4x256 / 8x128
        P.solo_nbk = std::max(0, std::min(1024, knob("BR_SOLO_NBK", "nbk", 8)));
        P.solo_nbk2 = std::max(1, knob("BR_SOLO_NBK2", "nbk2", 128));
        // the merges inside the kernel can read the sibling's certificate
        // the same way (off by default: large workload, M = 4096, two merge
        // levels in the kernel, 161.5 ms per query with the siblings in
        // their written order, 166.0 bucketed)
        P.solo_mbk = knob("BR_SOLO_MBK", "mbk", 0) != 0;
        P.qs = 2;
    }
    return P;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ctx_begin(br_ctx* c, hipStream_t s) {
    if (c->done_recorded) BR_HIP(hipStreamWaitEvent(s, c->ev_done, 0));
    return BR_OK;
}

int ctx_end(br_ctx* c, hipStream_t s) {
    BR_HIP(hipEventRecord(c->ev_done, s));
    c->done_recorded = true;
    return BR_OK;
}

int ensure_workspace(br_ctx* c, size_t bytes, hipStream_t s) {
    if (c->ws.size >= bytes) return BR_OK;
    // a context that serves requests under a memory budget holds exactly what
    // it was charged for; others grow by a quarter to avoid reallocating often
    size_t want = c->exact_ws ? bytes : std::max(bytes, c->ws.size + c->ws.size / 4);
    BR_HIP(hipStreamSynchronize(s));
    if (c->done_recorded) BR_HIP(hipEventSynchronize(c->ev_done));
    if (c->ws.base) BR_HIP(hipFree(c->ws.base));
    c->ws.base = nullptr;
    c->ws.size = 0;
    c->solo_key_base = nullptr;    // new memory: the solo slots start over
    hipError_t e = hipMalloc(&c->ws.base, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&c->ws.base, bytes);
        want = bytes;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    c->ws.size = want;
    return BR_OK;
}

int ensure_pinned(br_ctx* c, size_t bytes) {
    if (c->pinned_size >= bytes) return BR_OK;
    if (c->pinned) BR_HIP(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_size = 0;
    BR_HIP(hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault));
    c->pinned_size = bytes;
    return BR_OK;
}

// Workspace layout: [err | cnt | state | packed state | cert | off | cap |
// solo: pool | park + arrivals | queue | dense node states | slot tags | slots |
// bridge step]; everything before `cert` is cleared per call.
struct Layout {
    size_t err, cnt, state, packed, cert, off, cap, pool, park, queue, dense, tags, slots, sbuf, lmeta, rootw, bws,
        total;
};
// the one-graph batch description of the LDS plan: eoff[2], then V, M,
// rbase, cbase, vbase, n_items (one int64 word each), then the M work items
constexpr size_t kLdsMetaWords = 8;
// the largest chunk, in edges
static int64_t solo_chunk_max(const Plan& P) { return P.M > 0 ? (P.E + P.M - 1) / P.M : 0; }
// edges of a worker's reordering buffer: a chunk, and with bucketed merges
// also the largest right sibling merged inside the kernel (a node of level
// top - 1 spans 2^(top-1) chunks; a certificate holds at most 2(V-1) edges)
static int64_t solo_sbuf_stride(const Plan& P) {
    int64_t s = solo_chunk_max(P);
    const int64_t bound = 2 * (int64_t(P.V) - 1);
    if (P.solo_mbk)
        for (int l = 2; l <= P.solo_top && s < bound; l++) s = std::max(s, std::min(bound, 2 * s));
    return s;
}

static Layout layout(const Plan& P, bool device_final) {
    Layout L;
    size_t o = 0;
    L.err = o; o += 256;
    L.cnt = o; o = align256(o + sizeof(uint32_t) * 2 * (size_t)P.M);
    L.state = o;
    if (P.lds) o = align256(o + sizeof(uint32_t) * (size_t)P.lds_counters);     // arrivals, queue
    else if (!P.solo) o = align256(o + sizeof(uint32_t) * (size_t)P.qs * (size_t)P.V * (size_t)P.M);
    L.packed = o; if (!P.solo && !P.lds && P.qs != 2 && P.M > 1) o = align256(o + sizeof(uint32_t) * 2 * (size_t)P.V * (size_t)P.M);
    L.cert = o; o = align256(o + sizeof(int2) * (size_t)std::max<int64_t>(P.cert_pairs, 1));
    L.off = o; o = align256(o + sizeof(int64_t) * (size_t)P.M);
    L.cap = o; o = align256(o + sizeof(int64_t) * (size_t)P.M);
    L.pool = L.park = L.queue = L.dense = L.tags = L.slots = L.sbuf = L.lmeta = L.rootw = o;
    if (P.lds) {
        L.lmeta = o; o = align256(o + sizeof(int64_t) * (kLdsMetaWords + (size_t)P.M));
        L.rootw = o; o = align256(o + sizeof(uint32_t) * (size_t)P.V);
    }
    if (P.solo) {
        const int64_t top_nodes = ((int64_t)P.M + (int64_t(1) << P.solo_top) - 1) >> P.solo_top;
        L.pool = o; o = align256(o + 4 * (size_t)((P.nslots + 31) / 32));
        L.park = o; o = align256(o + 4 * 2 * (size_t)P.M);
        L.queue = o; o = align256(o + 4);
        L.dense = o; o = align256(o + 4 * 2 * (size_t)P.V * (size_t)top_nodes);
        L.tags = o; o = align256(o + 4 * (size_t)P.nslots);
        L.slots = o; o = align256(o + 4 * 2 * (size_t)P.V * (size_t)P.nslots);
        L.sbuf = o;
        if (P.solo_nbk > 0) o = align256(o + sizeof(int2) * (size_t)solo_sbuf_stride(P) * (size_t)P.workers);
    }
    L.bws = o; if (device_final) o = align256(o + sizeof(int32_t) * (size_t)device_bridges_words(P.V));
    L.total = o;
    return L;
}

size_t plan_workspace_bytes(const Plan& P, bool device_final) { return layout(P, device_final).total; }

static void ev_record(br_ctx* c, int k, hipStream_t s) {
    if (c->profiling) (void)hipEventRecord(c->ev[k], s);
}
static double ev_ms(br_ctx* c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return ms;
}

int run_certificate_with(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, hipStream_t s, Plan& P,
                         DevBufs& B, bool device_final, const TuneEntry* plan_knobs) {
    return run_certificate(c, d_edges, E, nullptr, 0, V, M, s, P, B, device_final, plan_knobs);
}

int run_certificate(br_ctx* c, const int32_t* d_a, int64_t Ea, const int32_t* d_b, int64_t Eb, int32_t V, int32_t M,
                    hipStream_t s, Plan& P, DevBufs& B, bool device_final, const TuneEntry* plan_knobs) {
    const int64_t E = Ea + Eb;
    P = plan_knobs ? make_plan(E, V, M, true, plan_knobs) : plan_for(c->device, E, V, M);
    if (Eb > 0 && P.lds) P = make_plan(E, V, M, false, nullptr);   // the LDS kernel reads one edge array
    const Layout L = layout(P, device_final);
    int rc = ensure_workspace(c, L.total, s);
    if (rc) return rc;
    rc = ensure_pinned(c, 64 << 10);
    if (rc) return rc;
    char* base = static_cast<char*>(c->ws.base);
    B.edges = reinterpret_cast<const int2*>(d_a);
    B.edges2 = reinterpret_cast<const int2*>(d_b);
    B.split = Ea;
    B.err = reinterpret_cast<uint32_t*>(base + L.err);
    B.cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
    B.state = reinterpret_cast<uint32_t*>(base + L.state);
    B.qs = P.qs;
    B.packed = P.qs != 2 && P.M > 1 ? reinterpret_cast<uint32_t*>(base + L.packed) : nullptr;
    B.cert = reinterpret_cast<int2*>(base + L.cert);
    B.off = reinterpret_cast<const int64_t*>(base + L.off);
    B.cap = reinterpret_cast<const int64_t*>(base + L.cap);
    c->bws = reinterpret_cast<int32_t*>(base + L.bws);
    // node regions: staged through pinned memory (the previous call's copy has
    // completed: every entry point ends with a stream synchronisation or an
    // event wait on the staging copy)
    const size_t meta_words = 2 * (size_t)M + (P.lds ? kLdsMetaWords + (size_t)M : 0);
    if (c->h_meta_n < meta_words) {
        if (c->h_meta) BR_HIP(hipHostFree(c->h_meta));
        c->h_meta = nullptr;
        c->h_meta_n = 0;
        BR_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_meta), sizeof(int64_t) * meta_words, hipHostMallocDefault));
        c->h_meta_n = meta_words;
    }
    std::memcpy(c->h_meta, P.off.data(), sizeof(int64_t) * M);
    std::memcpy(c->h_meta + M, P.cap.data(), sizeof(int64_t) * M);
    ev_record(c, 0, s);
    BR_HIP(hipMemcpyAsync(base + L.off, c->h_meta, sizeof(int64_t) * M, hipMemcpyHostToDevice, s));
    BR_HIP(hipMemcpyAsync(base + L.cap, c->h_meta + M, sizeof(int64_t) * M, hipMemcpyHostToDevice, s));
    if (P.lds) {
        int64_t* lm = c->h_meta + 2 * M;
        lm[0] = 0;                 // eoff: graph 0 is edges [0, E)
        lm[1] = E;
        lm[2] = V | ((int64_t)M << 32);   // V[0] and Mg[0] as two int32 words
        lm[3] = 1;                 // rbase: node k > 0 of graph 0 at index k
        lm[4] = 0;                 // cbase
        lm[5] = 0;                 // vbase
        lm[6] = 0;
        lm[7] = 0;
        for (int64_t k = 0; k < M; k++) lm[kLdsMetaWords + k] = k;   // items: graph 0, chunk k
        BR_HIP(hipMemcpyAsync(base + L.lmeta, lm, sizeof(int64_t) * (kLdsMetaWords + (size_t)M), hipMemcpyHostToDevice, s));
    }
    BR_HIP(hipEventRecord(c->ev[7], s));
    // all-singleton forests, zero counters and error word
    BR_HIP(hipMemsetAsync(base, 0, L.cert, s));
    c->prof.launches = 1;
    c->prof.plan_kind = P.lds ? 2 : (P.solo ? 1 : 0);
    int32_t first_step = 1;
    if (P.lds) {
        c->solo_key_base = nullptr;
        const int64_t* lm = reinterpret_cast<const int64_t*>(base + L.lmeta);
        BatchDev BD{};
        BD.edges = B.edges;
        BD.eoff = lm;
        BD.V = reinterpret_cast<const int32_t*>(lm + 2);
        BD.Mg = reinterpret_cast<const int32_t*>(lm + 2) + 1;
        BD.rbase = lm + 3;
        BD.cbase = lm + 4;
        BD.vbase = lm + 5;
        BD.noff = B.off;
        BD.ncap = B.cap;
        BD.items = lm + kLdsMetaWords;
        BD.n_items = M;
        BD.cert = B.cert;
        BD.ncnt = B.cnt;
        BD.arrive = reinterpret_cast<uint32_t*>(base + L.state);
        BD.queue = BD.arrive + P.lds_counters - 1;
        BD.err = B.err;
        BD.rootw = reinterpret_cast<uint32_t*>(base + L.rootw);
        ev_record(c, 1, s);
        launch_batched(BD, P.lds_blocks, s, P.lds_big);
        // the bridge step reads F's roots from the flags the kernel wrote (0 at a root)
        B.state = BD.rootw;
        B.qs = 1;
        B.packed = nullptr;
        first_step = M;            // every merge ran inside the kernel
    } else if (P.solo) {
        rc = solo_prepare(V);
        if (rc) return rc;
        SoloBufs Sb;
        Sb.slots = reinterpret_cast<uint32_t*>(base + L.slots);
        Sb.slot_tag = reinterpret_cast<uint32_t*>(base + L.tags);
        Sb.pool = reinterpret_cast<uint32_t*>(base + L.pool);
        Sb.park = reinterpret_cast<uint32_t*>(base + L.park);
        Sb.queue = reinterpret_cast<uint32_t*>(base + L.queue);
        Sb.dense = reinterpret_cast<uint32_t*>(base + L.dense);
        Sb.sbuf = P.solo_nbk > 0 ? reinterpret_cast<int2*>(base + L.sbuf) : nullptr;
        Sb.sbuf_stride = solo_sbuf_stride(P);
        Sb.nslots = P.nslots;
        Sb.workers = P.workers;
        // slot words carry tags from earlier calls on this workspace; a new
        // workspace, V or slot count starts them over from "all roots"
        if (c->solo_key_base != base + L.slots || c->solo_key_v != V || c->solo_key_slots != P.nslots) {
            launch_fill_u32(Sb.slot_tag, (int64_t)(L.bws - L.tags) / 4, 0u, s);
            c->solo_key_base = base + L.slots;
            c->solo_key_v = V;
            c->solo_key_slots = P.nslots;
            c->prof.launches++;
        }
        B.state = Sb.dense;
        B.qs = 2;
        B.packed = nullptr;
        B.shift = P.solo_top;
        ev_record(c, 1, s);
        launch_solo(P, B, Sb, s);
        first_step = 1 << P.solo_top;
    } else {
        c->solo_key_base = nullptr;    // this call's layout overwrites where slots may have been
        ev_record(c, 1, s);
        launch_phase0(P, B, s);
    }
    BR_HIP(hipGetLastError());
    c->prof.launches += phase0_launches(P);
    ev_record(c, 2, s);
    for (int32_t step = first_step; step < M; step *= 2) {
        c->prof.launches += launch_merge_round(P, B, step, s);
        BR_HIP(hipGetLastError());
    }
    ev_record(c, 3, s);
    c->prof.rounds = P.rounds;
    return BR_OK;
}

}  // namespace br

using namespace br;

extern "C" {

const char* br_last_error(void) { return g_err; }

int br_create(br_ctx** out, int device) {
    if (!out) return fail(BR_EINVAL, "br_create: null output pointer");
    int n = 0;
    BR_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(BR_EINVAL, "br_create: device %d not in [0,%d)", device, n);
    BR_HIP(hipSetDevice(device));
    if (g_cus == 0) {
        int cus = 0, lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess && lds > 0)
            g_max_lds = lds;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) g_cus = cus;
        (void)hipGetLastError();
    }
    br_ctx* c = new br_ctx();
    c->device = device;
    for (auto& e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            br_destroy(c);
            return hip_fail(hipGetLastError(), "hipEventCreate");
        }
    }
    if (hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess) {
        br_destroy(c);
        return hip_fail(hipGetLastError(), "hipEventCreate");
    }
    const int rc = static_scratch_init(device);
    if (rc) {
        br_destroy(c);
        return rc;
    }
    *out = c;
    return BR_OK;
}

int br_destroy(br_ctx* c) {
    if (!c) return BR_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    br::batched_release(c);
    if (c->ws.base) (void)hipFree(c->ws.base);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->h_meta) (void)hipHostFree(c->h_meta);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    delete c;
    return BR_OK;
}

int br_set_profiling(br_ctx* c, int on) {
    if (!c) return fail(BR_EINVAL, "br_set_profiling: null context");
    c->profiling = on <= 0 ? 0 : (on == 1 ? 1 : 2);
    return BR_OK;
}

int br_set_final_step(br_ctx* c, int mode) {
    if (!c || mode < 0 || mode > 1) return fail(BR_EINVAL, "br_set_final_step: bad argument");
    c->final_step = mode;
    return BR_OK;
}

int br_get_profile(br_ctx* c, br_profile* out) {
    if (!c || !out) return fail(BR_EINVAL, "br_get_profile: null argument");
    *out = c->prof;
    return BR_OK;
}

static int check_common(const void* edges, int64_t E, int32_t V) {
    if (E < 0) return fail(BR_EINVAL, "E = %lld < 0", (long long)E);
    if (V < 1) return fail(BR_EINVAL, "V = %d < 1", V);
    if (E > 0 && !edges) return fail(BR_EINVAL, "null edge list with E = %lld", (long long)E);
    return BR_OK;
}

int br_cert_build(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* d_cert,
                  int64_t cert_cap, int64_t* d_counts, void* stream) {
    if (!c || !d_counts || (!d_cert && cert_cap > 0)) return fail(BR_EINVAL, "br_cert_build: null argument");
    int rc = check_common(d_edges, E, V);
    if (rc) return rc;
    if (M < 1) return fail(BR_EINVAL, "M = %d < 1", M);
    if (cert_cap < 0) return fail(BR_EINVAL, "cert_cap < 0");
    const int64_t need = std::min<int64_t>(E, 2 * (int64_t(V) - 1));
    if (cert_cap < need)
        return fail(BR_ECAP, "br_cert_build: cert_cap %lld < min(E, 2(V-1)) = %lld", (long long)cert_cap,
                    (long long)need);
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BR_HIP(hipEventSynchronize(c->ev[7]));
    rc = ctx_begin(c, s);
    if (rc) return rc;
    Plan P;
    DevBufs B;
    rc = run_certificate(c, d_edges, E, nullptr, 0, V, M, s, P, B, false);
    if (rc) return rc;
    launch_copy_out(P, B, d_cert, cert_cap, d_counts, s);
    BR_HIP(hipGetLastError());
    return ctx_end(c, s);
}

int br_cert_merge(br_ctx* c, const int32_t* d_a, int64_t Ea, const int32_t* d_b, int64_t Eb, int32_t V,
                  int32_t* d_out, int64_t cap, int64_t* d_counts, void* stream) {
    if (!c || !d_counts || (!d_out && cap > 0)) return fail(BR_EINVAL, "br_cert_merge: null argument");
    if (Ea < 0 || Eb < 0) return fail(BR_EINVAL, "negative edge count");
    if ((Ea > 0 && !d_a) || (Eb > 0 && !d_b)) return fail(BR_EINVAL, "null edge list");
    if (V < 1) return fail(BR_EINVAL, "V = %d < 1", V);
    const int64_t need = std::min<int64_t>(Ea + Eb, 2 * (int64_t(V) - 1));
    if (cap < need)
        return fail(BR_ECAP, "br_cert_merge: cap %lld < min(Ea+Eb, 2(V-1)) = %lld", (long long)cap,
                    (long long)need);
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BR_HIP(hipEventSynchronize(c->ev[7]));
    int rc = ctx_begin(c, s);
    if (rc) return rc;
    // Certificate(A u B): one fused pass over the concatenation (Section III's
    // merge step re-runs the certificate algorithm on the union).
    Plan P;
    DevBufs B;
    rc = run_certificate(c, d_a, Ea, d_b, Eb, V, 1, s, P, B, false);
    if (rc) return rc;
    launch_copy_out(P, B, d_out, cap, d_counts, s);
    BR_HIP(hipGetLastError());
    return ctx_end(c, s);
}

int br_bridges_find(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_bridges,
                    int64_t cap, int64_t* n_bridges, void* stream) {
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    if (!c || !n_bridges || (!h_bridges && cap > 0)) return fail(BR_EINVAL, "br_bridges_find: null argument");
    int rc = check_common(d_edges, E, V);
    if (rc) return rc;
    if (M < 1) return fail(BR_EINVAL, "M = %d < 1", M);
    if (cap < 0) return fail(BR_EINVAL, "cap < 0");
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    auto t0 = std::chrono::steady_clock::now();
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BR_HIP(hipEventSynchronize(c->ev[7]));
    rc = ctx_begin(c, s);
    if (rc) return rc;
    const int mode = c->final_step;   // read once: the workspace layout depends on it
    Plan P;
    DevBufs B;
    rc = run_certificate(c, d_edges, E, nullptr, 0, V, M, s, P, B, mode == 1);
    if (rc) return rc;
    const int64_t cap0 = P.cap[0];
    uint32_t n1 = 0, n2 = 0, err = 0;
    std::chrono::steady_clock::time_point t1, t2;
    c->keys.clear();
    if (mode == 1) {
        // final step on the device: only the bridges come back
        uint64_t* d_keys = nullptr;
        uint32_t* d_n = nullptr;
        rc = device_bridges(P, B, c->bws, &d_keys, &d_n, s);
        if (rc) return rc;
        BR_HIP(hipGetLastError());
        ev_record(c, 5, s);
        // counters, error word and the first keys in one copy (the status block
        // precedes the keys); more keys than last time take a second copy
        rc = ensure_pinned(c, 256 + 8 * (size_t)V);
        if (rc) return rc;
        uint32_t* hc = static_cast<uint32_t*>(c->pinned);
        uint64_t* hk = reinterpret_cast<uint64_t*>(static_cast<char*>(c->pinned) + 256);
        const size_t guess = std::min<size_t>(std::max<size_t>(c->keys_hint, 1024), (size_t)V);
        BR_HIP(hipMemcpyAsync(hc, d_n - 1, 256 + 8 * guess, hipMemcpyDeviceToHost, s));
        rc = ctx_end(c, s);
        if (rc) return rc;
        BR_HIP(hipStreamSynchronize(s));
        n1 = hc[2]; n2 = hc[3]; err = hc[4];
        const uint32_t nk = std::min<uint32_t>(hc[1], (uint32_t)std::max(V - 1, 0));
        if (nk > guess) {
            BR_HIP(hipMemcpyAsync(hk + guess, d_keys + guess, 8 * (size_t)(nk - guess), hipMemcpyDeviceToHost, s));
            BR_HIP(hipStreamSynchronize(s));
        }
        c->keys_hint = nk;
        ev_record(c, 4, s);
        t1 = std::chrono::steady_clock::now();
        if (err & 1u) return fail(BR_ERANGE, "br_bridges_find: an edge has a vertex id outside [0, %d)", V);
        if (err != 0 || (int64_t)n1 + n2 > cap0)
            return fail(BR_EINTERNAL, "br_bridges_find: certificate region overflow");
        c->keys.assign(hk, hk + nk);
        t2 = std::chrono::steady_clock::now();
    } else {
        // node 0's whole region plus its counters and the error word
        const size_t need = sizeof(int2) * (size_t)std::max<int64_t>(cap0, 1) + 64;
        rc = ensure_pinned(c, need);
        if (rc) return rc;
        char* h = static_cast<char*>(c->pinned);
        uint32_t* hc = reinterpret_cast<uint32_t*>(h);
        int2* hx = reinterpret_cast<int2*>(h + 64);
        BR_HIP(hipMemcpyAsync(hc, B.cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BR_HIP(hipMemcpyAsync(hc + 2, B.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (cap0 > 0) BR_HIP(hipMemcpyAsync(hx, B.cert + P.off[0], sizeof(int2) * cap0, hipMemcpyDeviceToHost, s));
        ev_record(c, 4, s);
        rc = ctx_end(c, s);
        if (rc) return rc;
        BR_HIP(hipStreamSynchronize(s));
        t1 = std::chrono::steady_clock::now();
        n1 = hc[0]; n2 = hc[1]; err = hc[2];
        if (err & 1u) return fail(BR_ERANGE, "br_bridges_find: an edge has a vertex id outside [0, %d)", V);
        if (err != 0 || (int64_t)n1 + n2 > cap0)
            return fail(BR_EINTERNAL, "br_bridges_find: certificate region overflow (|F|=%u |F'|=%u cap=%lld)", n1,
                        n2, (long long)cap0);
        // adjacency with F's arcs first in every list (measured faster to walk
        // than a device-built adjacency in arbitrary order)
        certificate_bridges(hx, n1, hx + cap0 - n2, n2, V, c->dfs, c->keys);
        t2 = std::chrono::steady_clock::now();
    }
    canonical_sort(c->keys);
    auto t3 = std::chrono::steady_clock::now();
    const int64_t nb = (int64_t)c->keys.size();
    *n_bridges = nb;
    if (c->profiling) {
        c->prof.ms_phase0 = ev_ms(c, 1, 2);
        c->prof.ms_merge = ev_ms(c, 2, 3);
        c->prof.ms_cert = ev_ms(c, 0, 3);
        c->prof.ms_d2h = ev_ms(c, 3, 4);
        c->prof.ms_bridge_dev = mode == 1 ? ev_ms(c, 3, 5) : 0.0;
        c->prof.cert_f1 = n1;
        c->prof.cert_f2 = n2;
        c->prof.alg_bytes = 0;
        if (c->profiling >= 2 && !P.lds) {
            // every node's final region size (after the call: outside the
            // timed phases)
            std::vector<uint32_t> hn(2 * (size_t)P.M);
            BR_HIP(hipMemcpy(hn.data(), B.cnt, sizeof(uint32_t) * hn.size(), hipMemcpyDeviceToHost));
            int64_t bytes = 8 * E;
            for (int64_t i = 0; i < P.M; i++) {
                const int64_t x = std::min<int64_t>((int64_t)hn[2 * i] + hn[2 * i + 1], P.cap[i]);
                bytes += (i == 0 ? 8 : 16) * x;      // written; read once more by the merge of a right node
            }
            c->prof.alg_bytes = bytes;
        }
    }
    c->prof.ms_dfs = std::chrono::duration<double, std::milli>(t2 - t1).count();
    c->prof.ms_canon = std::chrono::duration<double, std::milli>(t3 - t2).count();
    c->prof.ms_total = std::chrono::duration<double, std::milli>(t3 - t0).count();
    if (nb > cap) return fail(BR_ECAP, "br_bridges_find: %lld bridges, capacity %lld", (long long)nb, (long long)cap);
    for (int64_t i = 0; i < nb; i++) {
        h_bridges[2 * i] = (int32_t)(c->keys[i] >> 32);
        h_bridges[2 * i + 1] = (int32_t)(c->keys[i] & 0xffffffffu);
    }
    return BR_OK;
}

// 2-edge-connected classes, and with h_tree the bridge tree's edges too
// (br_two_edge_components, br_bridge_tree)
static int classes_common(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_label,
                          int64_t* n_classes, int32_t* h_tree, int64_t cap, int64_t* n_tree, void* stream,
                          const char* who) {
    int rc = check_common(d_edges, E, V);
    if (rc) return rc;
    if (M < 1) return fail(BR_EINVAL, "M = %d < 1", M);
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BR_HIP(hipEventSynchronize(c->ev[7]));
    rc = ctx_begin(c, s);
    if (rc) return rc;
    const int mode = c->final_step;   // read once: the workspace layout depends on it
    Plan P;
    DevBufs B;
    rc = run_certificate(c, d_edges, E, nullptr, 0, V, M, s, P, B, mode == 1);
    if (rc) return rc;
    std::vector<uint64_t>& tkeys = c->keys;
    tkeys.clear();
    if (mode == 1) {
        // bridges and classes on the device: one copy of the status block and
        // labels (and one of the tree's edges)
        int32_t* d_label = nullptr;
        uint32_t* d_n = nullptr;
        uint64_t* d_tkeys = nullptr;
        rc = h_tree ? device_bridge_tree(P, B, c->bws, &d_label, &d_n, &d_tkeys, s)
                    : device_classes(P, B, c->bws, &d_label, &d_n, s);
        if (rc) return rc;
        BR_HIP(hipGetLastError());
        rc = ensure_pinned(c, 256 + 4 * (size_t)V);
        if (rc) return rc;
        uint32_t* hc = static_cast<uint32_t*>(c->pinned);
        BR_HIP(hipMemcpyAsync(hc, d_n - 1, 256 + 4 * (size_t)V, hipMemcpyDeviceToHost, s));
        rc = ctx_end(c, s);
        if (rc) return rc;
        BR_HIP(hipStreamSynchronize(s));
        const uint32_t err = hc[4];
        if (err & 1u) return fail(BR_ERANGE, "%s: an edge has a vertex id outside [0, %d)", who, V);
        if (err != 0 || (int64_t)hc[2] + hc[3] > P.cap[0]) return fail(BR_EINTERNAL, "%s: region overflow", who);
        std::memcpy(h_label, reinterpret_cast<const char*>(hc) + 256, 4 * (size_t)V);
        *n_classes = hc[1];
        if (h_tree) {
            const uint32_t nt = hc[5];
            if (nt > (uint32_t)std::max(V - 1, 0)) return fail(BR_EINTERNAL, "%s: %u tree edges", who, nt);
            tkeys.resize(nt);
            if (nt) {
                BR_HIP(hipMemcpyAsync(tkeys.data(), d_tkeys, 8 * (size_t)nt, hipMemcpyDeviceToHost, s));
                BR_HIP(hipStreamSynchronize(s));
            }
        }
    } else {
        const int64_t cap0 = P.cap[0];
        rc = ensure_pinned(c, sizeof(int2) * (size_t)std::max<int64_t>(cap0, 1) + 64);
        if (rc) return rc;
        char* h = static_cast<char*>(c->pinned);
        uint32_t* hc = reinterpret_cast<uint32_t*>(h);
        int2* hx = reinterpret_cast<int2*>(h + 64);
        BR_HIP(hipMemcpyAsync(hc, B.cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BR_HIP(hipMemcpyAsync(hc + 2, B.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (cap0 > 0) BR_HIP(hipMemcpyAsync(hx, B.cert + P.off[0], sizeof(int2) * cap0, hipMemcpyDeviceToHost, s));
        rc = ctx_end(c, s);
        if (rc) return rc;
        BR_HIP(hipStreamSynchronize(s));
        const uint32_t n1 = hc[0], n2 = hc[1], err = hc[2];
        if (err & 1u) return fail(BR_ERANGE, "%s: an edge has a vertex id outside [0, %d)", who, V);
        if (err != 0 || (int64_t)n1 + n2 > cap0) return fail(BR_EINTERNAL, "%s: region overflow", who);
        std::vector<uint64_t> bkeys;
        certificate_bridges(hx, n1, hx + cap0 - n2, n2, V, c->dfs, bkeys);
        canonical_sort(bkeys);
        // union of the certificate's non-bridge edges (a bridge has no parallel copy)
        std::vector<int32_t> par((size_t)V);
        for (int32_t v = 0; v < V; v++) par[v] = v;
        auto find = [&](int32_t x) {
            while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
            return x;
        };
        int64_t classes = V;
        auto join = [&](const int2& e) {
            const uint64_t k = (uint64_t)(uint32_t)std::min(e.x, e.y) << 32 | (uint32_t)std::max(e.x, e.y);
            if (std::binary_search(bkeys.begin(), bkeys.end(), k)) return;
            int32_t a = find(e.x), b = find(e.y);
            if (a == b) return;
            if (a < b) std::swap(a, b);
            par[a] = b;     // the smaller id stays the root: the label is the class minimum
            classes--;
        };
        for (uint32_t k = 0; k < n1; k++) join(hx[k]);
        for (uint32_t k = 0; k < n2; k++) join(hx[cap0 - n2 + k]);
        for (int32_t v = 0; v < V; v++) h_label[v] = find(v);
        *n_classes = classes;
        if (h_tree)
            for (uint64_t k : bkeys) {
                const uint32_t a = (uint32_t)h_label[k >> 32], b = (uint32_t)h_label[k & 0xffffffffu];
                tkeys.push_back((uint64_t)std::min(a, b) << 32 | std::max(a, b));
            }
    }
    if (!h_tree) return BR_OK;
    canonical_sort(tkeys);
    const int64_t nt = (int64_t)tkeys.size();
    *n_tree = nt;
    if (nt > cap) return fail(BR_ECAP, "%s: %lld tree edges, capacity %lld", who, (long long)nt, (long long)cap);
    for (int64_t i = 0; i < nt; i++) {
        h_tree[2 * i] = (int32_t)(tkeys[i] >> 32);
        h_tree[2 * i + 1] = (int32_t)(tkeys[i] & 0xffffffffu);
    }
    return BR_OK;
}

int br_two_edge_components(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_label,
                           int64_t* n_classes, void* stream) {
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    if (!c || !h_label || !n_classes) return fail(BR_EINVAL, "br_two_edge_components: null argument");
    return classes_common(c, d_edges, E, V, M, h_label, n_classes, nullptr, 0, nullptr, stream,
                          "br_two_edge_components");
}

int br_bridge_tree(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_label,
                   int32_t* h_tree, int64_t cap, int64_t* n_classes, int64_t* n_tree, void* stream) {
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    if (!c || !h_label || !n_classes || !n_tree || cap < 0 || (cap > 0 && !h_tree))
        return fail(BR_EINVAL, "br_bridge_tree: null argument");
    int32_t dummy[2];
    return classes_common(c, d_edges, E, V, M, h_label, n_classes, h_tree ? h_tree : dummy, cap, n_tree, stream,
                          "br_bridge_tree");
}

int br_articulation_points(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t* h_out, int64_t cap,
                           int64_t* n_out, void* stream) {
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    if (!c || !n_out || (!h_out && cap > 0)) return fail(BR_EINVAL, "br_articulation_points: null argument");
    int rc = check_common(d_edges, E, V);
    if (rc) return rc;
    if (cap < 0) return fail(BR_EINVAL, "cap < 0");
    if (E > 2147483647LL) return fail(BR_EINVAL, "br_articulation_points: E = %lld above 2^31 - 1", (long long)E);
    if (V > kFinalStepMaxV) return fail(BR_EINVAL, "V = %d above the final step's limit 2^29", V);
    auto t0 = std::chrono::steady_clock::now();
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BR_HIP(hipEventSynchronize(c->ev[7]));
    rc = ctx_begin(c, s);
    if (rc) return rc;
    const int mode = c->final_step;   // read once: the workspace layout depends on it
    const size_t ws_cert = 4 * (size_t)scan_first_words(E, V);
    const size_t ws_test = mode == 1 ? 4 * (size_t)device_bridges_words(V) : 0;
    c->solo_key_base = nullptr;        // the scan-first search reuses the workspace
    rc = ensure_workspace(c, ws_cert + ws_test + 256, s);
    if (rc) return rc;
    rc = ensure_pinned(c, 256 + 2 * sizeof(int2) * (size_t)std::max(V, 1));
    if (rc) return rc;
    char* h = static_cast<char*>(c->pinned);
    uint32_t* hs = reinterpret_cast<uint32_t*>(h);
    uint32_t n1 = 0, n2 = 0;
    int l1 = 0, l2 = 0;
    std::vector<int32_t> aps;
    std::chrono::steady_clock::time_point t1;
    char* wsb = static_cast<char*>(c->ws.base);
    if (mode == 1) {
        // test on the device: only the articulation points come back
        int2 *f1 = nullptr, *f2 = nullptr;
        uint32_t *cnt = nullptr, *err = nullptr, *roots = nullptr;
        rc = scan_first_device(reinterpret_cast<const int2*>(d_edges), E, V, wsb, s, hs, &l1, &l2, &f1, &f2, &cnt, &err,
                               &roots);
        if (rc) return rc;
        int32_t* tws = reinterpret_cast<int32_t*>(wsb + ((ws_cert + 255) & ~size_t(255)));
        uint64_t* d_keys = nullptr;
        uint32_t* d_n = nullptr;
        rc = device_articulation_cert(f1, f2, 1, cnt, roots, 1, V, tws, &d_keys, &d_n, s);
        if (rc) return rc;
        launch_bridge_status(cnt, err, d_n, s);
        BR_HIP(hipGetLastError());
        uint64_t* hk = reinterpret_cast<uint64_t*>(h + 256);
        const size_t guess = std::min<size_t>(std::max<size_t>(c->keys_hint, 1024), (size_t)std::max(V, 1));
        BR_HIP(hipMemcpyAsync(hs, d_n - 1, 256 + 8 * guess, hipMemcpyDeviceToHost, s));
        rc = ctx_end(c, s);
        if (rc) return rc;
        BR_HIP(hipStreamSynchronize(s));
        n1 = hs[2]; n2 = hs[3];
        const uint32_t e = hs[4], nk = std::min<uint32_t>(hs[1], (uint32_t)std::max(V, 1));
        if (e & 1u) return fail(BR_ERANGE, "br_articulation_points: an edge has a vertex id outside [0, %d)", V);
        if (e) return fail(BR_EINTERNAL, "br_articulation_points: forest larger than V - 1");
        if (nk > guess) {
            BR_HIP(hipMemcpyAsync(hk + guess, d_keys + guess, 8 * (size_t)(nk - guess), hipMemcpyDeviceToHost, s));
            BR_HIP(hipStreamSynchronize(s));
        }
        c->keys_hint = nk;
        t1 = std::chrono::steady_clock::now();
        aps.resize(nk);
        for (uint32_t i = 0; i < nk; i++) aps[i] = (int32_t)hk[i];
        std::sort(aps.begin(), aps.end());
    } else {
        // Algorithm 1's search (vertex test) on the host over the copied certificate
        int2* hf1 = reinterpret_cast<int2*>(h + 256);
        int2* hf2 = hf1 + std::max(V, 1);
        rc = scan_first_certificate(reinterpret_cast<const int2*>(d_edges), E, V, wsb, s, hs, hf1, hf2, &n1, &n2, &l1,
                                    &l2);
        if (rc) return rc;
        rc = ctx_end(c, s);
        if (rc) return rc;
        t1 = std::chrono::steady_clock::now();
        certificate_articulation(hf1, n1, hf2, n2, V, c->dfs, aps);
    }
    auto t2 = std::chrono::steady_clock::now();
    *n_out = (int64_t)aps.size();
    c->prof.cert_f1 = n1;
    c->prof.cert_f2 = n2;
    c->prof.rounds = l1 + l2;          // breadth-first levels of the two forests
    c->prof.ms_cert = std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->prof.ms_dfs = std::chrono::duration<double, std::milli>(t2 - t1).count();
    c->prof.ms_total = c->prof.ms_cert + c->prof.ms_dfs;
    if ((int64_t)aps.size() > cap)
        return fail(BR_ECAP, "br_articulation_points: %lld articulation points, capacity %lld", (long long)aps.size(),
                    (long long)cap);
    std::copy(aps.begin(), aps.end(), h_out);
    return BR_OK;
}

int br_autotune(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, char* out, int64_t out_cap,
                void* stream) {
    if (!c || (out_cap > 0 && !out) || out_cap < 0) return fail(BR_EINVAL, "br_autotune: bad argument");
    int rc = check_common(d_edges, E, V);
    if (rc) return rc;
    if (M < 1) return fail(BR_EINVAL, "M = %d < 1", M);
    BR_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string key = plain_tune_key(c->device, E, V, M);
    TuneEntry best;
    int source = 0;   // 0: from the cache, 1: measured now
    if (!tune_get(key, best)) {
        source = 1;
        // candidate plans: the team path with three first-stage tiles, the
        // whole-tree LDS kernel where V fits, and the one-workgroup-per-node
        // path in each worker shape with the merge depths around its default
        // (and depths 1 and 2)
        std::vector<TuneEntry> cands;
        for (int tile : {4096, 2048, 1024}) cands.push_back({{"lds", 0}, {"solo", 0}, {"tile", tile}});
        if (E > 0 && V <= batched_max_v_big() && M < (1 << 20)) cands.push_back({{"lds", 1}});
        if (E > 0 && V <= solo_max_v()) {
            const Plan d = make_plan(E, V, M, true, nullptr);
            for (int v = 0; v < solo_variants(); v++) {
                TuneEntry on{{"lds", 0}, {"solo", 1}, {"variant", v}};
                const Plan dv = make_plan(E, V, M, true, &on);
                std::vector<int> tops;
                for (int top : {dv.solo_top - 1, dv.solo_top, dv.solo_top + 1, 1, 2})
                    if (top >= 0 && top <= d.rounds && std::find(tops.begin(), tops.end(), top) == tops.end())
                        tops.push_back(top);
                for (int top : tops) cands.push_back({{"lds", 0}, {"solo", 1}, {"variant", v}, {"top", top}});
            }
        }
        double best_ms = 1e30;
        BR_HIP(hipEventSynchronize(c->ev[7]));
        rc = ctx_begin(c, s);
        if (rc) return rc;
        // the certificate (phase 0 and merges) of plan t: one run to settle
        // the workspace, then the best of two
        auto time_plan = [&](const TuneEntry& t, double* ms) -> int {
            *ms = 1e30;
            for (int rep = 0; rep < 3; rep++) {
                Plan P;
                DevBufs B;
                TuneEntry tt = t;
                BR_HIP(hipEventSynchronize(c->ev[7]));
                BR_HIP(hipEventRecord(c->ev[5], s));
                const int r = run_certificate_with(c, d_edges, E, V, M, s, P, B, false, &tt);
                if (r) return r;
                BR_HIP(hipEventRecord(c->ev[6], s));
                BR_HIP(hipEventSynchronize(c->ev[6]));
                float f = 0.f;
                BR_HIP(hipEventElapsedTime(&f, c->ev[5], c->ev[6]));
                if (rep > 0) *ms = std::min(*ms, (double)f);
            }
            return BR_OK;
        };
        for (const TuneEntry& t : cands) {
            double ms = 0;
            rc = time_plan(t, &ms);
            if (rc) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        // then the winner with its team merges requesting each thread's edges
        // of a tile at once (measured: large M = 256 merges 3.12 -> 2.35 ms,
        // dense M = 256 0.83 -> 0.87 ms), and a one-workgroup-per-node winner
        // with the siblings of its own merges bucketed, then with its chunks
        // in input order
        auto try_alt = [&](const char* name, double v) -> int {
            TuneEntry alt = best;
            alt[name] = v;
            double ms = 0;
            const int r = time_plan(alt, &ms);
            if (r) return r;
            if (ms < best_ms) {
                best_ms = ms;
                best = alt;
            }
            return BR_OK;
        };
        if (M > 1 && !(best.count("lds") && best["lds"] == 1)) {
            rc = try_alt("prem", 1);
            if (rc) return rc;
        }
        if (best.count("solo") && best["solo"] == 1) {
            if (!(best.count("top") && best["top"] == 0)) {
                rc = try_alt("mbk", 1);
                if (rc) return rc;
            }
            rc = try_alt("nbk", 0);
            if (rc) return rc;
        }
        rc = ctx_end(c, s);
        if (rc) return rc;
        best["ms"] = best_ms;
        tune_put(key, best);
    }
    if (out_cap > 0) {
        std::string js = "{\"key\": \"" + key + "\", \"source\": \"" + (source ? "measured" : "cache") + "\"";
        for (const auto& kv : best) {
            char buf[96];
            std::snprintf(buf, sizeof buf, ", \"%s\": %.6g", kv.first.c_str(), kv.second);
            js += buf;
        }
        js += "}";
        std::snprintf(out, (size_t)out_cap, "%s", js.c_str());
    }
    return BR_OK;
}

int br_certificate_bridges(const int32_t* h_f1, int64_t n1, const int32_t* h_f2, int64_t n2, int32_t V,
                           int32_t* h_bridges, int64_t cap, int64_t* n_bridges) {
    if (!n_bridges || n1 < 0 || n2 < 0 || (n1 > 0 && !h_f1) || (n2 > 0 && !h_f2) || cap < 0 || (cap > 0 && !h_bridges))
        return fail(BR_EINVAL, "br_certificate_bridges: bad argument");
    if (V < 1 || V > (1 << 29)) return fail(BR_EINVAL, "br_certificate_bridges: V = %d outside [1, 2^29]", V);
    if (n1 + n2 >= (int64_t(1) << 30)) return fail(BR_EINVAL, "br_certificate_bridges: too many edges");
    for (int64_t k = 0; k < 2 * n1; k++)
        if ((uint32_t)h_f1[k] >= (uint32_t)V) return fail(BR_ERANGE, "br_certificate_bridges: id out of range");
    for (int64_t k = 0; k < 2 * n2; k++)
        if ((uint32_t)h_f2[k] >= (uint32_t)V) return fail(BR_ERANGE, "br_certificate_bridges: id out of range");
    thread_local DfsScratch S;
    thread_local std::vector<uint64_t> keys;
    keys.clear();
    certificate_bridges(reinterpret_cast<const int2*>(h_f1), n1, reinterpret_cast<const int2*>(h_f2), n2, V, S, keys);
    canonical_sort(keys);
    const int64_t nb = (int64_t)keys.size();
    *n_bridges = nb;
    if (nb > cap) return fail(BR_ECAP, "br_certificate_bridges: %lld bridges, capacity %lld", (long long)nb, (long long)cap);
    for (int64_t i = 0; i < nb; i++) {
        h_bridges[2 * i] = (int32_t)(keys[i] >> 32);
        h_bridges[2 * i + 1] = (int32_t)(keys[i] & 0xffffffffu);
    }
    return BR_OK;
}

}  // extern "C"
