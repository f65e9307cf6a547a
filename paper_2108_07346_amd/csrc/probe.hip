// Measurement utility: one read of a device buffer with 16-byte lane loads,
// so that a benchmark can state the read bandwidth this device actually
// reaches beside the HBM peak.  Not a step of the method.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace br {
namespace {

// each block xor-folds what it read into one word (so the loads cannot be
// dropped) and adds it to *sink
__global__ void __launch_bounds__(256) k_probe_read(const uint4* p, int64_t n16, const uint8_t* tail, int32_t ntail,
                                                    uint64_t* sink) {
    uint32_t x = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n16; i += stride) {
        const uint4 a = p[i];
        x ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (blockIdx.x == 0 && threadIdx.x < (uint32_t)ntail) x ^= tail[threadIdx.x];
    for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(reinterpret_cast<unsigned long long*>(sink), (unsigned long long)x);
}

}  // namespace
}  // namespace br

using namespace br;

extern "C" int br_probe_read(const void* d_buf, int64_t bytes, uint64_t* d_sink, void* stream) {
    if (bytes < 0 || (bytes > 0 && !d_buf) || !d_sink) return fail(BR_EINVAL, "br_probe_read: bad argument");
    if ((reinterpret_cast<uintptr_t>(d_buf) & 15) != 0) return fail(BR_EINVAL, "br_probe_read: buffer not 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n16 = bytes / 16;
    int dev = 0, cus = 256;
    BR_HIP(hipGetDevice(&dev));
    BR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n16 + 1023) / 1024, (int64_t)cus * 16));
    hipLaunchKernelGGL(k_probe_read, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint4*>(d_buf), n16,
                       static_cast<const uint8_t*>(d_buf) + 16 * n16, (int32_t)(bytes - 16 * n16), d_sink);
    BR_HIP(hipGetLastError());
    return BR_OK;
}
