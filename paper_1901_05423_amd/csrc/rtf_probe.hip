// rtf_probe.hip -- measurement aid (librtf_probe.so): the memory pattern of a
// sampling step with no search, the ceiling for the sampling kernels.  See
// include/rtf_probe.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtf_probe.h"

namespace {

__device__ inline uint64_t mulhi(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

template <bool WANT_X>
__global__ __launch_bounds__(256) void k_probe_gather(const uint4 *__restrict__ table, int64_t m,
                                                      const uint4 *__restrict__ nodes, int64_t n,
                                                      const uint64_t *__restrict__ u, int64_t S,
                                                      int32_t depth, int32_t *__restrict__ idx,
                                                      double *__restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride) {
        const uint64_t us = __builtin_nontemporal_load(u + s);
        const uint4 *rec = table + 4 * (int64_t)mulhi(us, (uint64_t)m);
        uint4 v[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) v[w] = rec[w];  // one record, four loads in flight
        uint64_t h = us;
#pragma unroll
        for (int w = 0; w < 4; ++w)
            h ^= (((uint64_t)v[w].y << 32) | v[w].x) + (((uint64_t)v[w].w << 32) | v[w].z);
        for (int32_t d = 1; d < depth; ++d) {  // further reads, each after the previous
            const uint4 nd = nodes[mulhi(h ^ us, (uint64_t)n)];
            h = (h * 0x9e3779b97f4a7c15ull) ^ (((uint64_t)nd.y << 32) | nd.x) ^
                (((uint64_t)nd.w << 32) | nd.z);
        }
        __builtin_nontemporal_store((int32_t)h, idx + s);
        if (WANT_X) __builtin_nontemporal_store((double)(h >> 11) * 0x1p-53, x + s);
    }
}

}  // namespace

extern "C" int rtf_probe_gather(const void *table, int64_t m, const void *nodes, int64_t n,
                                const uint64_t *u, int64_t S, int32_t depth, int32_t *idx,
                                double *x, hipStream_t stream) {
    if (!table || !u || !idx || m < 1 || S < 0 || depth < 1) return 1;
    if (depth > 1 && (!nodes || n < 1)) return 1;
    if ((reinterpret_cast<uintptr_t>(table) & 63) || (reinterpret_cast<uintptr_t>(nodes) & 15))
        return 1;
    if (S == 0) return 0;
    int64_t blocks = (S + 255) / 256;
    blocks = blocks < 256 * 64 ? blocks : 256 * 64;  // the sampling kernel's grid
    const dim3 g((unsigned)blocks), b(256);
    const uint4 *t4 = static_cast<const uint4 *>(table);
    const uint4 *n4 = static_cast<const uint4 *>(nodes);
    if (x)
        hipLaunchKernelGGL(k_probe_gather<true>, g, b, 0, stream, t4, m, n4, n, u, S, depth, idx,
                           x);
    else
        hipLaunchKernelGGL(k_probe_gather<false>, g, b, 0, stream, t4, m, n4, n, u, S, depth, idx,
                           x);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}
