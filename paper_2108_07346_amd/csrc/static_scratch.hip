// The certificate of br_cert_build computed in a fixed device array instead
// of the context's workspace, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy until the process ends.  Host code never passes its name to a
// kernel (in host code the name is a host-side stand-in); it uses the device
// address hipGetSymbolAddress returns, found once per device when a context
// is created on that device.  Every call on one GPU shares that GPU's array:
// calls that overlap on one GPU race, and each call clears what must start at
// zero itself.
#include <mutex>

#include "internal.hpp"

namespace br {
namespace {

__device__ __align__(256) uint8_t scratch[BR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Node regions of the phase tree on the device, so that nothing is uploaded:
// cap[i] = min(edges under node i, 2(V-1)), off[] its exclusive prefix sum
// (the same numbers make_plan computes on the host).  One workgroup.
constexpr int kRT = 1024;
__global__ void __launch_bounds__(kRT) k_regions(int64_t E, int32_t V, int32_t M, int64_t* off, int64_t* cap) {
    __shared__ int64_t part[kRT];
    auto lo = [&](int64_t i) { return i * (E / M) + (i * (E % M)) / M; };
    const int64_t bound = 2 * ((int64_t)V - 1);
    const int64_t per = ((int64_t)M + kRT - 1) / kRT;
    const int64_t i0 = min((int64_t)M, (int64_t)threadIdx.x * per), i1 = min((int64_t)M, i0 + per);
    int64_t sum = 0;
    for (int64_t i = i0; i < i1; i++) {
        const int64_t span = i == 0 ? (int64_t)M : min(int64_t(1) << __builtin_ctzll((unsigned long long)i), (int64_t)M - i);
        const int64_t c = min(lo(min((int64_t)M, i + span)) - lo(i), bound);
        cap[i] = c;
        sum += c;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int t = 0; t < kRT; t++) {
            const int64_t x = part[t];
            part[t] = acc;
            acc += x;
        }
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int64_t i = i0; i < i1; i++) {
        off[i] = acc;
        acc += cap[i];
    }
}

}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(BR_EINVAL, "static scratch: device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return BR_OK;
    void* p = nullptr;
    BR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));     // the calling thread has `device` current
    if (!p) return fail(BR_EINTERNAL, "static scratch: no device address");
    g_ptr[device] = p;
    return BR_OK;
}

}  // namespace br

using namespace br;

extern "C" int br_cert_build_static(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M,
                                    int32_t* d_cert, int64_t cert_cap, int64_t* d_counts, void* stream) {
    if (!c || !d_counts || (!d_cert && cert_cap > 0)) return fail(BR_EINVAL, "br_cert_build_static: null argument");
    if (E < 0 || V < 1 || (E > 0 && !d_edges)) return fail(BR_EINVAL, "br_cert_build_static: bad edge list or V");
    if (M < 1) return fail(BR_EINVAL, "M = %d < 1", M);
    if (cert_cap < 0) return fail(BR_EINVAL, "cert_cap < 0");
    const int64_t need = std::min<int64_t>(E, 2 * (int64_t(V) - 1));
    if (cert_cap < need)
        return fail(BR_ECAP, "br_cert_build_static: cert_cap %lld < min(E, 2(V-1)) = %lld", (long long)cert_cap,
                    (long long)need);
    Plan P = make_plan(E, V, M, false);
    P.qs = 2;   // packed state only: no spread copy to compress into
    size_t o = 0;
    const size_t o_err = o; o += 256;
    const size_t o_cnt = o; o = a256(o + 4 * 2 * (size_t)M);
    const size_t o_state = o; o = a256(o + 4 * 2 * (size_t)V * (size_t)M);
    const size_t o_cert = o; o = a256(o + 8 * (size_t)std::max<int64_t>(P.cert_pairs, 1));
    const size_t o_off = o; o = a256(o + 8 * (size_t)M);
    const size_t o_cap = o; o = a256(o + 8 * (size_t)M);
    if (o > (size_t)BR_STATIC_SCRATCH_BYTES)
        return fail(BR_ENOMEM, "br_cert_build_static: V = %d, E = %lld, M = %d need %zu bytes of scratch, the fixed array holds %zu",
                    V, (long long)E, M, o, (size_t)BR_STATIC_SCRATCH_BYTES);
    BR_HIP(hipSetDevice(c->device));
    int rc = static_scratch_init(c->device);
    if (rc) return rc;
    char* base = static_cast<char*>(g_ptr[c->device]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = ctx_begin(c, s);
    if (rc) return rc;
    DevBufs B;
    B.edges = reinterpret_cast<const int2*>(d_edges);
    B.edges2 = nullptr;
    B.split = E;
    B.err = reinterpret_cast<uint32_t*>(base + o_err);
    B.cnt = reinterpret_cast<uint32_t*>(base + o_cnt);
    B.state = reinterpret_cast<uint32_t*>(base + o_state);
    B.qs = 2;
    B.packed = nullptr;
    B.cert = reinterpret_cast<int2*>(base + o_cert);
    B.off = reinterpret_cast<const int64_t*>(base + o_off);
    B.cap = reinterpret_cast<const int64_t*>(base + o_cap);
    // all-singleton forests, zero counters and error word (a fill kernel, so
    // that the call can also be captured into a graph)
    launch_fill_u32(reinterpret_cast<uint32_t*>(base), (int64_t)(o_cert / 4), 0u, s);
    hipLaunchKernelGGL(k_regions, dim3(1), dim3(kRT), 0, s, E, V, M, reinterpret_cast<int64_t*>(base + o_off),
                       reinterpret_cast<int64_t*>(base + o_cap));
    launch_phase0(P, B, s);
    for (int32_t step = 1; step < M; step *= 2) launch_merge_round(P, B, step, s);
    launch_copy_out(P, B, d_cert, cert_cap, d_counts, s);
    BR_HIP(hipGetLastError());
    return ctx_end(c, s);
}
