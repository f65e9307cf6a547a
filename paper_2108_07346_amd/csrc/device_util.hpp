// Small device-side helpers shared by the kernel files (included by .hip
// sources only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

// grid-stride loop of this thread over [0, n)
#define GRID_LOOP(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

namespace br {

// blocks of 256 threads for n items, at least 1 and at most 16384 (the
// kernels that take it loop over the rest)
inline int grid_for(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 16384));
}

// place of this lane among the lanes set in a wavefront ballot
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace br
