// Level scan of a range lookup on the Eytzinger layouts (Section 5) with the
// hybrid coalesced scanning of Section 5.1, shared by the per-index range
// kernel (range.hip) and the batched mixed stream (batch.hip).
//
// The matches of [lo, hi] on one level of the level-order tree are
// consecutive and start where the lower-bound search path of lo enters the
// level; every match at level-order slot t goes to position
// slot_rank(t) - (rank of lo's lower bound) of the range's output, which
// puts the row IDs in key order.
//
// Each lane first scans its own range alone.  When it meets kHandover (one
// wave's width) matches on one level it pauses (by the property noted in Section 5.1, every deeper
// level then holds more matches still), and once every lane of the wave has
// finished or paused, the wave takes over the paused scans one at a time:
// all 64 lanes read 64 consecutive entries of a level per step, and the
// lower-bound path continues with one pivot per lane and a ballot.
#pragma once

#include "internal.hpp"
#include "access.hpp"

namespace idx {

// Sorted rank of level-order slot t known to lie on level l (t < n).
__host__ __device__ inline uint64_t slot_rank_on(const Geo &G, uint64_t t, uint32_t l) {
    const uint64_t bottom_start = G.start[G.m];
    if (t >= bottom_start) {
        const uint64_t i = t - bottom_start;
        return i + div_g(G, i);
    }
    const uint64_t i = t - G.start[l];
    const uint64_t p = (G.start[G.m - l - 1] + 1) * (1 + i + div_g(G, i)) - 1;
    const uint64_t skip = G.g * (p + 1);
    return p + (skip < G.b ? skip : G.b);
}

// Where a paused scan continues: node c on level lvl (its pivot count below
// lo is j) and the next slot t of that level.
struct ScanState {
    uint64_t c;
    uint64_t t;
    uint32_t lvl;
    uint32_t j;
};

// Matches on one level after which a lane hands its scan to the wave; a
// lane that never hands over (the single-lane scan) uses kNoHandover.
constexpr uint32_t kHandover = kWave;
constexpr uint32_t kNoHandover = 0xFFFFFFFFu;

// Single-lane level scan of [lo, hi] (first rank r0, cnt matches, output at
// out).  Keys and row IDs of level-order slot t are at layout slot off + t.
// Returns true when it paused (state in st) with `handover` matches on a level.
template <typename K, bool AOS>
__device__ __forceinline__ bool eyt_scan_lane(const Load<K, AOS> &L, const Geo &G, uint64_t off, K lo, K hi,
                                              uint64_t r0, uint64_t cnt, uint32_t *__restrict__ out, ScanState &st,
                                              uint32_t handover = kHandover) {
    const uint64_t n = G.n;
    const uint32_t g = G.g, kf = G.k;
    uint64_t c = 0;
    uint32_t lvl = 0;
    while (c * g < n) {
        const uint64_t i = c * g;
        const uint64_t nv = (n - i) < g ? (n - i) : g;
        uint32_t j = 0;
        for (uint32_t e = 0; e < nv; ++e) j += L.key(off + i + e) < lo ? 1u : 0u;
        const uint64_t level_end = G.start[lvl + 1] < n ? G.start[lvl + 1] : n;
        uint32_t seen = 0;
        for (uint64_t t = i + j; t < level_end; ++t) {
            if (L.key(off + t) > hi) break;
            const uint64_t d = slot_rank_on(G, t, lvl) - r0;  // position in key order
            if (d < cnt) out[d] = L.row(off + t);
            if (++seen == handover) {
                st = ScanState{c, t + 1, lvl, j};
                return true;
            }
        }
        c = c * kf + 1 + j;
        ++lvl;
    }
    return false;
}

// ---- vector form for SoA nodes of 16 to 128 bytes starting on 16-byte
// boundaries (EKS with off = 0): a node is read once with independent 16-byte
// loads and counted in registers, and the row IDs of a node's matches come
// from one vector read of the node's row IDs, instead of one dependent load
// per pivot and per match (whose lines L2 evicts between the probes when
// hundreds of thousands of scans are in flight).
constexpr uint32_t kScanNodeBytes = 128;

__host__ __device__ inline bool scan_vec_ok(const Geo &G, uint64_t off, uint32_t key_bytes, bool aos) {
    const uint32_t nb = G.g * key_bytes;
    return !aos && off == 0 && nb % 16 == 0 && nb <= kScanNodeBytes && G.g % 4 == 0;
}

// The g keys of the node starting at slot i (16-byte chunks; padding past n
// is read but never counted).
template <typename K>
__device__ __forceinline__ void node_keys(const K *__restrict__ keys, uint64_t i, uint32_t g, K *kk) {
    constexpr int V = 16 / sizeof(K);
    constexpr int MC = kScanNodeBytes / 16;
    const uint4 *q = (const uint4 *)(keys + i);
    const uint32_t chunks = g / V;
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if ((uint32_t)c < chunks) w = q[c];
        if constexpr (sizeof(K) == 8) {
            kk[2 * c] = ((uint64_t)w.y << 32) | w.x;
            kk[2 * c + 1] = ((uint64_t)w.w << 32) | w.z;
        } else {
            kk[4 * c] = w.x;
            kk[4 * c + 1] = w.y;
            kk[4 * c + 2] = w.z;
            kk[4 * c + 3] = w.w;
        }
    }
}

// Pivots of a node (valid slots only) below x.
template <typename K>
__device__ __forceinline__ uint32_t node_below(const K *kk, uint32_t valid, K x) {
    constexpr int NK = kScanNodeBytes / sizeof(K);
    uint32_t j = 0;
#pragma unroll
    for (int e = 0; e < NK; ++e) j += ((uint32_t)e < valid && kk[e] < x) ? 1u : 0u;
    return j;
}

template <typename K>
__device__ __forceinline__ bool eyt_scan_lane_vec(const K *__restrict__ keys, const uint32_t *__restrict__ rows,
                                                  const Geo &G, K lo, K hi, uint64_t r0, uint64_t cnt,
                                                  uint32_t *__restrict__ out, ScanState &st,
                                                  uint32_t handover = kHandover) {
    constexpr int NK = kScanNodeBytes / sizeof(K);
    constexpr int NR = kScanNodeBytes / sizeof(K) / 4;  // 16-byte row chunks of the largest node
    const uint64_t n = G.n;
    const uint32_t g = G.g, kf = G.k;
    const uint64_t bottom_start = G.start[G.m];
    uint64_t c = 0;
    uint32_t lvl = 0;
    K kk[NK];
    while (c * g < n) {
        const uint64_t i = c * g;
        const uint64_t level_end = G.start[lvl + 1] < n ? G.start[lvl + 1] : n;
        node_keys(keys, i, g, kk);
        uint32_t valid = (n - i) < g ? (uint32_t)(n - i) : g;
        const uint32_t j = node_below(kk, valid, lo);
        uint32_t seen = 0;
        uint64_t nb = i;     // start slot of the node in registers
        uint32_t from = j;   // first match within it
        for (;;) {
            // matches of this node: slots nb + [from, upto)
            // keys ascend along a level: slots [from, upto) hold the keys in [lo, hi]
            const uint32_t upto = hi == key_max<K>() ? valid : node_below(kk, valid, (K)(hi + 1));
            if (upto > from) {
                uint4 rw[NR];
                const uint4 *rq = (const uint4 *)(rows + nb);
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if ((uint32_t)q < g / 4) rw[q] = rq[q];
                const uint64_t d0 = slot_rank_on(G, nb + from, lvl) - r0;
                const bool bottom = nb >= bottom_start;
#pragma unroll
                for (int e = 0; e < NK; ++e) {
                    if ((uint32_t)e < from || (uint32_t)e >= upto) continue;
                    if (seen == handover) {
                        st = ScanState{c, nb + (uint64_t)e, lvl, j};
                        return true;
                    }
                    const uint4 w = rw[e / 4];
                    const uint32_t r = (e & 3) == 0 ? w.x : (e & 3) == 1 ? w.y : (e & 3) == 2 ? w.z : w.w;
                    const uint64_t d = bottom ? d0 + (uint64_t)(e - from) : slot_rank_on(G, nb + e, lvl) - r0;
                    if (d < cnt) out[d] = r;
                    ++seen;
                }
            }
            // the run goes on in the next node of the level only if it reached this node's end
            if (upto < valid || nb + g >= level_end) break;
            nb += g;
            node_keys(keys, nb, g, kk);
            valid = (n - nb) < g ? (uint32_t)(n - nb) : g;
            from = 0;
        }
        c = c * kf + 1 + j;
        ++lvl;
    }
    return false;
}

// The whole wave continues one paused scan (every lane passes the same
// arguments).  Pivots per node g <= kWave.
template <typename K, bool AOS>
__device__ __forceinline__ void eyt_scan_wave(const Load<K, AOS> &L, const Geo &G, uint64_t off, K lo, K hi,
                                              uint64_t r0, uint64_t cnt, uint32_t *__restrict__ out, ScanState st) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t n = G.n;
    const uint32_t g = G.g, kf = G.k;
    uint64_t c = st.c, t = st.t;
    uint32_t lvl = st.lvl, j = st.j;
    bool resume = true;
    while (c * g < n) {
        const uint64_t i = c * g;
        if (!resume) {
            const uint64_t nv = (n - i) < g ? (n - i) : g;
            const bool below = lane < nv && L.key(off + i + lane) < lo;
            j = (uint32_t)__popcll(__ballot(below));
            t = i + j;
        }
        resume = false;
        const uint64_t level_end = G.start[lvl + 1] < n ? G.start[lvl + 1] : n;
        for (uint64_t b = t; b < level_end; b += kWave) {
            const uint64_t s = b + lane;
            bool match = false;
            if (s < level_end && L.key(off + s) <= hi) {
                match = true;
                const uint64_t d = slot_rank_on(G, s, lvl) - r0;
                if (d < cnt) out[d] = L.row(off + s);
            }
            // keys ascend along a level: done once a lane saw a larger key or the level end
            if (__ballot(!match) != 0) break;
        }
        c = c * kf + 1 + j;
        ++lvl;
    }
}

}  // namespace idx
