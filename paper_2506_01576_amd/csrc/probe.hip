// Random-access probe: the coalescing micro-benchmark of Section 5.1
// (Figure 9) re-shaped for MI355X.  Lanes form groups of `group` neighbours;
// every step each group reads `group` consecutive 64-bit words at a random,
// group-aligned position of a large buffer.  Each lane keeps 8 independent
// streams in flight so the measured rate is the memory system's random
// granule throughput, not the latency of one chain.
#include "internal.hpp"

namespace idx {
namespace {

__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kStreams = 8;

__global__ __launch_bounds__(256) void k_probe(const uint64_t *__restrict__ buf, uint64_t groups_in_buf,
                                               uint32_t group_shift, uint32_t steps, uint64_t seed,
                                               uint64_t *__restrict__ sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gid = tid >> group_shift;
    const uint32_t sub = threadIdx.x & ((1u << group_shift) - 1);
    uint64_t acc = 0;
    uint64_t st[kStreams];
#pragma unroll
    for (int u = 0; u < kStreams; ++u) st[u] = mix(seed ^ (gid * kStreams + u));
    for (uint32_t s = 0; s < steps; ++s) {
        uint64_t v[kStreams];
#pragma unroll
        for (int u = 0; u < kStreams; ++u) {
            st[u] = mix(st[u]);
            // multiply-high maps the 64-bit draw onto [0, groups_in_buf)
            const uint64_t gpos = __umul64hi(st[u], groups_in_buf);
            v[u] = buf[(gpos << group_shift) + sub];
        }
#pragma unroll
        for (int u = 0; u < kStreams; ++u) acc ^= v[u];
    }
    if (acc == 0x1234567ull) sink[0] = acc;  // keeps the loads alive
}

}  // namespace
}  // namespace idx

extern "C" int idx_probe_random(const void *buf, uint64_t words, uint32_t group, uint64_t lanes, uint32_t steps,
                                uint64_t seed, uint64_t *sink, idx_stream stream) {
    using namespace idx;
    if (!buf || !sink || words == 0 || group == 0 || group > 64 || (group & (group - 1)) || lanes == 0 ||
        lanes % 256 != 0 || words < group)
        return IDX_ERR_ARG;
    uint32_t shift = 0;
    while ((1u << shift) < group) ++shift;
    const uint64_t groups_in_buf = words >> shift;
    const uint64_t blocks = lanes / 256;
    if (blocks > 0x7FFFFFFFull) return IDX_ERR_ARG;
    hipLaunchKernelGGL(k_probe, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, (const uint64_t *)buf,
                       groups_in_buf, shift, steps, seed, sink);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}
