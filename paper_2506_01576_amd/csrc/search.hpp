// Short-window search on a sorted key array.  Once a binary search has
// narrowed the answer to a window of at most W keys, the window is read with
// independent 16-byte loads and the keys below the target are counted in
// registers.  On MI355X the last binary-search steps fall into lines that
// were just fetched, but with hundreds of thousands of lookups in flight per
// XCD those lines are evicted from L2 between dependent probes; one round of
// independent loads fetches each line once.
#pragma once

#include "internal.hpp"

namespace idx {

// Keys of sorted[b, b + len) (len <= W) below x; `eq` tells whether one of
// them equals x.  Reads whole 16-byte chunks covering the window: up to one
// chunk beyond b + len, which the padded layout allocations keep in bounds.
template <typename K, int W>
__device__ __forceinline__ uint32_t count_below(const K *__restrict__ keys, uint64_t b, uint32_t len, K x, bool &eq,
                                                bool two = true) {
    constexpr int V = 16 / sizeof(K);
    constexpr int CH = W / V + 1;
    const uint64_t a0 = b & ~(uint64_t)(V - 1);
    const uint64_t end = b + len;
    const uint4 *p = (const uint4 *)(keys + a0);
    // Two rounds (two = true): first the chunks in the 128-byte line of the
    // window's first chunk, the rest only when every window key among them is
    // below x (keys ascend, so otherwise the lower bound is among them).  One
    // round reads every chunk at once.
    const uint64_t line0 = (uint64_t)(uintptr_t)p >> 7;
    uint4 w[CH];
    bool got[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        got[c] = a0 + (uint64_t)c * V < end && (!two || ((uint64_t)(uintptr_t)(p + c) >> 7) == line0);
        if (got[c]) w[c] = p[c];
    }
    uint32_t below = 0, in1 = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (!got[c]) continue;
        const uint64_t s = a0 + (uint64_t)c * V;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t slot = s + v;
            const bool in = slot >= b && slot < end;
            uint64_t kv;
            if constexpr (sizeof(K) == 8) kv = v == 0 ? (((uint64_t)w[c].y << 32) | w[c].x) : (((uint64_t)w[c].w << 32) | w[c].z);
            else kv = v == 0 ? w[c].x : v == 1 ? w[c].y : v == 2 ? w[c].z : w[c].w;
            in1 += in ? 1u : 0u;
            below += (in && (K)kv < x) ? 1u : 0u;
        }
    }
    if (two && below == in1) {
#pragma unroll
        for (int c = 0; c < CH; ++c)
            if (!got[c] && a0 + (uint64_t)c * V < end) {
                w[c] = p[c];
                got[c] = true;
            }
    }
    uint32_t cnt = 0;
    bool e = false;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint64_t s = a0 + (uint64_t)c * V;
        if (s >= end || !got[c]) continue;
        K kk[V];
        if constexpr (sizeof(K) == 8) {
            kk[0] = ((uint64_t)w[c].y << 32) | w[c].x;
            kk[1] = ((uint64_t)w[c].w << 32) | w[c].z;
        } else {
            kk[0] = w[c].x;
            kk[1] = w[c].y;
            kk[2] = w[c].z;
            kk[3] = w[c].w;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t slot = s + v;
            const bool in = slot >= b && slot < end;
            cnt += (in && kk[v] < x) ? 1u : 0u;
            e |= in && kk[v] == x;
        }
    }
    eq = e;
    return cnt;
}

}  // namespace idx
