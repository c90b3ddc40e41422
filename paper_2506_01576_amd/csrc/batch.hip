// Batched point lookups over many independent indexes in one persistent
// launch.  The queries of all indexes are concatenated (index i owns
// queries[offsets[i] .. offsets[i+1])); a persistent grid walks that flat
// array in wave-sized chunks, so load balance is perfect however uneven the
// indexes and their batches are (the static scheduling of Section 7.2, with
// the work split over lookups rather than over indexes).  Each wave finds the
// index of its chunk with one binary search over the offsets (a per-lane
// search only where a chunk straddles an index boundary), reads that index's
// descriptor and runs its descent per lane: BS, EBS, EKS (single lane, whole
// node in registers) or the learned window search -- the form the autotuner
// chose for the index's size class.  Everything the kernel needs is in device
// memory, so the launch can be captured once in a HIP graph and replayed.
//
// The mixed stream (idx_batch_mixed) adds range lookups to the same walk: a
// first persistent launch answers every point lookup and sizes every range
// (first and past-the-end rank of its bounds), an exclusive scan turns the
// sizes into output offsets, and a second persistent launch writes each
// range's row IDs in key order -- a wave-cooperative copy of the run of
// ranks [first, first + count): contiguous on the sorted-array forms, read at
// the slots the layout build wrote those ranks to on the Eytzinger forms (or,
// when a member asks for it, the level scan with rank scatter of Section 5);
// each index's tree geometry is kept in a device table beside its
// descriptor.
#include <new>
#include <vector>

#include "internal.hpp"
#include "access.hpp"
#include "learned_model.hpp"
#include "range_scan.hpp"

namespace idx {
namespace {

enum : uint32_t { F_BS = 0, F_EBS = 1, F_EKS = 2, F_LEARNED = 3 };

struct __align__(16) Desc {
    const void *keys;
    const uint32_t *rows;
    uint64_t n;
    const LeafRec *leaves;  // learned form only
    uint32_t form, k, g, levels;
    uint32_t m_full, early, gshift, lanes;  // lanes: EKS lanes per lookup (1 = whole node per lane)
    const void *pin;        // top levels in LDS order (BS heap order; Eytzinger slot prefix), or null
    uint32_t pin_levels;    // levels served from LDS (0 = none)
    uint32_t pin_keys;      // entries of `pin`
    RootRec root;           // learned form only
    uint32_t vec;           // EKS nodes read with 16-byte loads
    uint32_t rscan;         // Eytzinger ranges: 3 = gather by rank, 1/2 = level scan (range_scan)
    uint64_t kinv;          // ceil(2^64 / k) for the rank-to-slot map (k > 2)
};
static_assert(sizeof(Desc) == 144, "descriptor layout");

constexpr int BT = 256;     // threads per workgroup
constexpr int BR = 4;       // lookups per lane
constexpr uint64_t CW = (uint64_t)kWave * BR;  // queries per wave chunk
constexpr uint64_t CB = (uint64_t)BT * BR;     // queries per workgroup chunk

template <typename K>
__device__ __forceinline__ uint32_t bs_find(const K *__restrict__ keys, const uint32_t *__restrict__ rows,
                                            uint64_t n, K x) {
    if (n == 0) return kMiss;
    uint64_t base = 0, len = n;
    while (len > 1) {
        const uint64_t half = len >> 1;
        base = keys[base + half] < x ? base + half : base;
        len -= half;
    }
    const K kb = keys[base];
    const uint64_t pos = base + (kb < x ? 1 : 0);
    if (pos >= n) return kMiss;
    const K kp = kb < x ? keys[pos] : kb;
    return kp == x ? rows[pos] : kMiss;
}

template <typename K>
__device__ __forceinline__ uint32_t ebs_find(const K *__restrict__ keys, const uint32_t *__restrict__ rows,
                                             uint64_t n, uint32_t m_full, K x) {
    uint64_t i = 1;
    K ck = ~K(0);
    for (uint32_t l = 0; l < m_full; ++l) {
        const K kk = keys[i];
        const bool right = kk < x;
        ck = right ? ck : kk;
        i = 2 * i + (right ? 1 : 0);
    }
    if (i <= n) {
        const K kk = keys[i];
        const bool right = kk < x;
        ck = right ? ck : kk;
        i = 2 * i + (right ? 1 : 0);
    }
    const uint64_t j = i >> (__builtin_ctzll(~i) + 1);
    return (j != 0 && ck == x) ? rows[j] : kMiss;
}

template <typename K>
__device__ __forceinline__ uint32_t eks_find(const K *__restrict__ keys, const uint32_t *__restrict__ rows,
                                             const Desc &d, K x) {
    const uint64_t n = d.n;
    const uint32_t g = d.g, kf = d.k;
    uint64_t c = 0, cand = 0;
    bool ceq = false;
    for (uint32_t lvl = 0; lvl < d.levels; ++lvl) {
        const uint64_t i = c * g;
        if (i >= n) break;
        const uint64_t nv = (n - i) < g ? (n - i) : g;
        uint32_t j = 0;
        bool eq = false;
        for (uint32_t e = 0; e < nv; ++e) {
            const K kk = keys[i + e];
            j += kk < x ? 1u : 0u;
            eq |= kk == x;
        }
        if (j < nv) {
            cand = i + j;
            ceq = eq;
        }
        if (d.early && eq) break;
        c = c * kf + 1 + j;
    }
    return ceq ? rows[cand] : kMiss;
}

template <typename K>
__device__ __forceinline__ uint32_t learned_find(const K *__restrict__ keys, const uint32_t *__restrict__ rows,
                                                 const Desc &d, K x) {
    const uint64_t r = learned_lower_rank(keys, d.n, d.root, d.leaves, x);
    return (r < d.n && keys[r] == x) ? rows[r] : kMiss;
}

// Index owning flat query position p: the last i with offsets[i] <= p, for
// i in [lo, hi).
__device__ __forceinline__ uint32_t owner(const uint64_t *__restrict__ off, uint32_t lo, uint32_t hi, uint64_t p) {
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---- one index per wave chunk: every lane holds up to BR lookups of the
// chunk and advances them level by level together, so their dependent loads
// are in flight at once (the per-lane chains of the single-index kernels).
// `pin` (LDS) holds the index's top `pl` levels, or pl = 0.

// BS: lockstep binary search to a window of at most 15 keys, then the
// short-window scan (independent 16-byte loads counted in registers).
template <typename K>
__device__ __forceinline__ void wave_bs(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                        uint64_t c0, uint64_t c1, const K *pin, uint32_t pl) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const K *__restrict__ keys = (const K *)d.keys;
    const uint64_t n = d.n;
    K x[BR];
    uint64_t base[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        x[r] = p < c1 ? q[p] : K(0);
        base[r] = 0;
    }
    if (n == 0) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const uint64_t p = c0 + (uint64_t)r * kWave + lane;
            if (p < c1) out[p] = kMiss;
        }
        return;
    }
    uint64_t len = n;
    if (pl) {
        uint32_t v[BR];
#pragma unroll
        for (int r = 0; r < BR; ++r) v[r] = 1;
        for (uint32_t l = 0; l < pl; ++l) {
            const uint64_t half = len >> 1;
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const bool go = pin[v[r]] < x[r];
                base[r] += go ? half : 0;
                v[r] = 2 * v[r] + (go ? 1u : 0u);
            }
            len -= half;
        }
    }
    while (len > 15) {
        const uint64_t half = len >> 1;
#pragma unroll
        for (int r = 0; r < BR; ++r) base[r] = keys[base[r] + half] < x[r] ? base[r] + half : base[r];
        len -= half;
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        if (p >= c1) continue;
        const uint64_t sl = (len + 1) < (n - base[r]) ? (len + 1) : (n - base[r]);
        bool eq;
        const uint32_t c = count_below<K, 16>(keys, base[r], (uint32_t)sl, x[r], eq);
        out[p] = eq ? d.rows[base[r] + c] : kMiss;
    }
}

// EBS: lockstep descent; the lower-bound slot is recovered from the final
// position (drop the trailing right turns and the last left turn).
template <typename K>
__device__ __forceinline__ void wave_ebs(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                         uint64_t c0, uint64_t c1, const K *pin, uint32_t pl) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const K *__restrict__ keys = (const K *)d.keys;
    const uint64_t n = d.n;
    K x[BR], ck[BR];
    uint64_t i[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        x[r] = p < c1 ? q[p] : K(0);
        ck[r] = ~K(0);
        i[r] = 1;
    }
    uint32_t l = 0;
    for (; l < pl; ++l) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const K kk = pin[i[r]];
            const bool right = kk < x[r];
            ck[r] = right ? ck[r] : kk;
            i[r] = 2 * i[r] + (right ? 1 : 0);
        }
    }
    for (; l < d.m_full; ++l) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const K kk = keys[i[r]];
            const bool right = kk < x[r];
            ck[r] = right ? ck[r] : kk;
            i[r] = 2 * i[r] + (right ? 1 : 0);
        }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        if (i[r] <= n) {
            const K kk = keys[i[r]];
            const bool right = kk < x[r];
            ck[r] = right ? ck[r] : kk;
            i[r] = 2 * i[r] + (right ? 1 : 0);
        }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        if (p >= c1) continue;
        const uint64_t j = i[r] >> (__builtin_ctzll(~i[r]) + 1);
        out[p] = (j != 0 && ck[r] == x[r]) ? d.rows[j] : kMiss;
    }
}

// EKS (single): one lane per lookup reads a whole node of at most NK keys
// (16-byte loads when the descriptor says the nodes allow it) and counts in
// registers; R lookups per lane in lockstep (NK * R bounds the registers).
template <typename K, int NK, int R>
__device__ __forceinline__ void wave_eks_single(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                                uint64_t c0, uint64_t c1, const K *pin, uint32_t pl) {
    constexpr int V = 16 / sizeof(K);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const K *__restrict__ keys = (const K *)d.keys;
    const uint64_t n = d.n;
    const uint32_t g = d.g, kf = d.k;
    const uint64_t pin_end = pl ? (uint64_t)d.pin_keys : 0;  // slots below come from LDS
    for (uint64_t p0 = c0; p0 < c1; p0 += (uint64_t)kWave * R) {
        K x[R];
        uint64_t c[R], cand[R];
        bool ceq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t p = p0 + (uint64_t)r * kWave + lane;
            x[r] = p < c1 ? q[p] : K(0);
            c[r] = p < c1 ? 0 : ~0ull;
            cand[r] = 0;
            ceq[r] = false;
        }
        for (uint32_t lvl = 0; lvl < d.levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (c[r] == ~0ull) continue;
                const uint64_t i = c[r] * g;
                const uint32_t nv = (n - i) < g ? (uint32_t)(n - i) : g;
                K kk[NK];
                if (i < pin_end) {
#pragma unroll
                    for (int e = 0; e < NK; ++e) kk[e] = (uint32_t)e < nv ? pin[i + e] : ~K(0);
                } else if (d.vec) {
                    // whole 16-byte chunks of the node; a partial last node's
                    // chunks stay inside the padded allocation and are masked
                    const uint4 *pp = (const uint4 *)(keys + i);
#pragma unroll
                    for (int v = 0; v < NK / V; ++v) {
                        uint4 w = make_uint4(0u, 0u, 0u, 0u);
                        if ((uint32_t)(v * V) < g) w = pp[v];
                        if constexpr (sizeof(K) == 8) {
                            kk[2 * v] = ((uint64_t)w.y << 32) | w.x;
                            kk[2 * v + 1] = ((uint64_t)w.w << 32) | w.z;
                        } else {
                            kk[4 * v] = w.x;
                            kk[4 * v + 1] = w.y;
                            kk[4 * v + 2] = w.z;
                            kk[4 * v + 3] = w.w;
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < NK; ++e) kk[e] = (uint32_t)e < nv ? keys[i + e] : ~K(0);
                }
                uint32_t j = 0;
                bool eq = false;
#pragma unroll
                for (int e = 0; e < NK; ++e) {
                    const bool in = (uint32_t)e < nv;
                    j += (in && kk[e] < x[r]) ? 1u : 0u;
                    eq |= in && kk[e] == x[r];
                }
                if (j < nv) {
                    cand[r] = i + j;
                    ceq[r] = eq;
                }
                const uint64_t child = c[r] * kf + 1 + j;
                c[r] = ((d.early && eq) || child * g >= n) ? ~0ull : child;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t p = p0 + (uint64_t)r * kWave + lane;
            if (p < c1) out[p] = ceq[r] ? d.rows[cand[r]] : kMiss;
        }
    }
}

// EKS (group): GL = d.lanes lanes per lookup, each reading VL consecutive
// pivots (VL = 1: one pivot per lane, GL >= k - 1; VL = 16 / sizeof(K): one
// 16-byte chunk per lane); j = popcount of the group's ballot of pivot < x.
template <typename K, int VL>
__device__ __forceinline__ void wave_eks_group(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                               uint64_t c0, uint64_t c1, const K *pin, uint32_t pl) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t GL = d.lanes;
    const uint32_t gpw = kWave / GL;  // lookups per wave per slot
    const uint32_t sub = lane & (GL - 1), grp = lane / GL;
    const uint64_t gmask = GL == kWave ? ~0ull : (((1ull << GL) - 1ull) << (grp * GL));
    const K *__restrict__ keys = (const K *)d.keys;
    const uint64_t n = d.n;
    const uint32_t g = d.g, kf = d.k;
    const uint32_t first = sub * VL;
    const uint64_t pin_end = pl ? (uint64_t)d.pin_keys : 0;
    constexpr int R = BR;
    for (uint64_t p0 = c0; p0 < c1; p0 += (uint64_t)gpw * R) {
        K x[R];
        uint64_t c[R], cand[R];
        bool ceq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t p = p0 + (uint64_t)r * gpw + grp;
            x[r] = p < c1 ? q[p] : K(0);
            c[r] = p < c1 ? 0 : ~0ull;
            cand[r] = 0;
            ceq[r] = false;
        }
        for (uint32_t lvl = 0; lvl < d.levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool live = c[r] != ~0ull;
                const uint64_t i = live ? c[r] * g : n;
                const bool lane_live = live && first < g && i + first < n;
                K kk[VL];
#pragma unroll
                for (int e = 0; e < VL; ++e) kk[e] = ~K(0);
                if (lane_live) {
                    const uint64_t s = i + first;
                    if constexpr (VL == 1) {
                        kk[0] = s < pin_end ? pin[s] : keys[s];
                    } else {
                        const uint4 w = s < pin_end ? *(const uint4 *)(pin + s) : *(const uint4 *)(keys + s);
                        if constexpr (sizeof(K) == 8) {
                            kk[0] = ((uint64_t)w.y << 32) | w.x;
                            kk[1] = ((uint64_t)w.w << 32) | w.z;
                        } else {
                            kk[0] = w.x;
                            kk[1] = w.y;
                            kk[2] = w.z;
                            kk[3] = w.w;
                        }
                    }
                }
                uint32_t j = 0;
                bool eql = false;
#pragma unroll
                for (int e = 0; e < VL; ++e) {
                    const bool valid = lane_live && first + e < g && i + first + e < n;
                    j += (uint32_t)__popcll(__ballot(valid && kk[e] < x[r]) & gmask);
                    eql |= valid && kk[e] == x[r];
                }
                const uint64_t eq = __ballot(eql) & gmask;
                if (live) {
                    const uint64_t nv = (n - i) < g ? (n - i) : g;
                    if (j < nv) {
                        cand[r] = i + j;
                        ceq[r] = eq != 0;
                    }
                    const uint64_t child = c[r] * kf + 1 + j;
                    c[r] = ((d.early && eq != 0) || child * g >= n) ? ~0ull : child;
                }
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t p = p0 + (uint64_t)r * gpw + grp;
                if (p < c1) out[p] = ceq[r] ? d.rows[cand[r]] : kMiss;
            }
        }
    }
}

// Learned: every lookup's root and leaf evaluation, then the window halving
// while any window spans more than 15 keys, then the short-window scans, in
// lockstep over the lane's lookups.
template <typename K>
__device__ __forceinline__ void wave_learned(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                             uint64_t c0, uint64_t c1) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const K *__restrict__ keys = (const K *)d.keys;
    K x[BR];
    uint32_t b[BR], len[BR];  // ranks: n < 2^32
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        x[r] = p < c1 ? q[p] : K(0);
        b[r] = 0;
        len[r] = 0;
        if (p < c1) {
            uint64_t wb, wl;
            learned_window(d.root, d.leaves, (uint64_t)x[r], wb, wl);
            b[r] = (uint32_t)wb;
            len[r] = (uint32_t)wl;
        }
    }
    for (;;) {
        bool more = false;
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            if (len[r] > 15) {
                const uint32_t half = len[r] >> 1;
                b[r] = keys[(uint64_t)b[r] + half - 1] < x[r] ? b[r] + half : b[r];
                len[r] -= half;
            }
            more |= len[r] > 15;
        }
        if (!more) break;
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const uint64_t p = c0 + (uint64_t)r * kWave + lane;
        if (p >= c1) continue;
        bool eq;
        const uint32_t c = count_below<K, 16>(keys, b[r], len[r], x[r], eq);
        out[p] = eq ? d.rows[(uint64_t)b[r] + c] : kMiss;
    }
}

template <typename K>
__device__ __forceinline__ void wave_one_index(const Desc &d, const K *__restrict__ q, uint32_t *__restrict__ out,
                                               uint64_t c0, uint64_t c1, const K *pin, uint32_t pl) {
    switch (d.form) {
        case F_BS: wave_bs<K>(d, q, out, c0, c1, pin, pl); return;
        case F_EBS: wave_ebs<K>(d, q, out, c0, c1, pin, pl); return;
        case F_EKS:
            if (d.lanes > 1) {
                if (d.lanes >= d.g) wave_eks_group<K, 1>(d, q, out, c0, c1, pin, pl);
                else wave_eks_group<K, 16 / sizeof(K)>(d, q, out, c0, c1, pin, pl);
            } else if (d.g <= 4) {
                wave_eks_single<K, 4, 4>(d, q, out, c0, c1, pin, pl);
            } else if (d.g <= 8) {
                wave_eks_single<K, 8, 4>(d, q, out, c0, c1, pin, pl);
            } else if (d.g <= 16) {
                wave_eks_single<K, 16, 2>(d, q, out, c0, c1, pin, pl);
            } else {
                wave_eks_single<K, 32, 1>(d, q, out, c0, c1, pin, pl);
            }
            return;
        default: wave_learned<K>(d, q, out, c0, c1); return;
    }
}

// The persistent walk: each workgroup takes chunks of CB consecutive flat
// query positions, CW per wave.  A chunk inside one index (the usual case:
// the large batches hold most queries) runs that index's form in lockstep,
// with its top levels copied to LDS once per workgroup chunk when the member
// asked for cache pinning; a wave chunk spanning several (small) indexes
// runs each lookup on its own.
template <typename K>
__global__ __launch_bounds__(BT) void k_batch_point(const Desc *__restrict__ descs, uint32_t count,
                                                    const uint64_t *__restrict__ off, const K *__restrict__ q,
                                                    uint32_t *__restrict__ out) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    const uint64_t total = off[count];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    uint32_t pinned = 0xFFFFFFFFu;  // member whose top levels s_pin holds (workgroup-uniform)
    for (uint64_t b0 = (uint64_t)blockIdx.x * CB; b0 < total; b0 += (uint64_t)gridDim.x * CB) {
        const uint64_t b1 = b0 + CB < total ? b0 + CB : total;
        // workgroup-uniform owners of the chunk's first and last query
        const uint32_t j0 = owner(off, 0, count, b0);
        const uint32_t j1 = owner(off, j0, count, b1 - 1);
        uint32_t pl = 0;
        if (j0 == j1 && descs[j0].pin_levels) {
            if (pinned != j0) {
                const Desc &dp = descs[j0];
                const K *src = (const K *)dp.pin;
                __syncthreads();  // every wave is done with the previous member's levels
                for (uint32_t e = threadIdx.x; e < dp.pin_keys; e += BT) s_pin[e] = src[e];
                __syncthreads();
                pinned = j0;
            }
            pl = descs[j0].pin_levels;
        }
        const uint64_t c0 = b0 + (uint64_t)wave * CW;
        if (c0 >= b1) continue;
        const uint64_t c1 = c0 + CW < b1 ? c0 + CW : b1;
        const uint32_t i0 = j0 == j1 ? j0 : owner(off, j0, j1 + 1, c0);
        const uint32_t i1 = j0 == j1 ? j0 : owner(off, i0, j1 + 1, c1 - 1);
        if (i0 == i1) {
            const Desc d = descs[i0];
            wave_one_index<K>(d, q, out, c0, c1, s_pin, pl);
            continue;
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const uint64_t p = c0 + (uint64_t)r * kWave + lane;
            if (p >= c1) continue;
            const uint32_t ii = owner(off, i0, i1 + 1, p);
            const Desc d = descs[ii];
            const K x = q[p];
            const K *keys = (const K *)d.keys;
            uint32_t res;
            switch (d.form) {
                case F_BS: res = bs_find<K>(keys, d.rows, d.n, x); break;
                case F_EBS: res = ebs_find<K>(keys, d.rows, d.n, d.m_full, x); break;
                case F_EKS: res = eks_find<K>(keys, d.rows, d, x); break;
                default: res = learned_find<K>(keys, d.rows, d, x); break;
            }
            out[p] = res;
        }
    }
}

// ------------------------------------------------------------ mixed stream

enum : uint8_t { Q_POINT = 0, Q_RANGE = 1 };
// Where a range's ranks are stored: the sorted array itself, or the slots of
// the binary / k-ary Eytzinger layout the build wrote them to.
enum : uint32_t { MAP_SORTED = 0, MAP_BINARY = 1, MAP_KARY = 2 };

// Sorted rank of the first key >= x in the index of descriptor d.
// Lower-bound rank of x in index d.  EYT selects the forms compiled in:
// false = BS and learned, true = EBS and EKS (the caller routes each index to
// the matching kind).
template <typename K, bool EYT>
__device__ __forceinline__ uint64_t form_lower_rank(const Desc &d, const Geo &G, K x) {
    const K *keys = (const K *)d.keys;
    const uint64_t n = d.n;
    if (n == 0) return 0;
    if constexpr (!EYT) {
        if (d.form == F_LEARNED) return learned_lower_rank(keys, n, d.root, d.leaves, x);
        uint64_t base = 0, len = n;
        while (len > 1) {
            const uint64_t half = len >> 1;
            base = keys[base + half] < x ? base + half : base;
            len -= half;
        }
        return base + (keys[base] < x ? 1 : 0);
    } else {
        // Eytzinger layouts: deepest path position of the lower bound, then its rank
        const uint64_t off = d.form == F_EBS ? 1 : 0;
        const uint32_t g = G.g, kf = G.k;
        uint64_t c = 0, cand = ~0ull;
        if (scan_vec_ok(G, off, sizeof(K), false)) {  // whole nodes in registers
            K kk[kScanNodeBytes / sizeof(K)];
            while (c * g < n) {
                const uint64_t i = c * g;
                const uint32_t nv = (n - i) < g ? (uint32_t)(n - i) : g;
                node_keys(keys, i, g, kk);
                const uint32_t j = node_below(kk, nv, x);
                if (j < nv) cand = i + j;
                c = c * kf + 1 + j;
            }
            return cand == ~0ull ? n : slot_rank(G, cand);
        }
        while (c * g < n) {
            const uint64_t i = c * g;
            const uint64_t nv = (n - i) < g ? (n - i) : g;
            uint32_t j = 0;
            for (uint32_t e = 0; e < nv; ++e) j += keys[off + i + e] < x ? 1u : 0u;
            if (j < nv) cand = i + j;
            c = c * kf + 1 + j;
        }
        return cand == ~0ull ? n : slot_rank(G, cand);
    }
}

// Point answer in index d, with the forms of one kind compiled in (as above).
template <typename K, bool EYT>
__device__ __forceinline__ uint32_t form_find_kind(const Desc &d, K x) {
    const K *keys = (const K *)d.keys;
    if constexpr (!EYT) {
        if (d.form == F_BS) return bs_find<K>(keys, d.rows, d.n, x);
        return learned_find<K>(keys, d.rows, d, x);
    } else {
        if (d.form == F_EBS) return ebs_find<K>(keys, d.rows, d.n, d.m_full, x);
        return eks_find<K>(keys, d.rows, d, x);
    }
}

template <typename K>
__device__ __forceinline__ uint32_t form_find(const Desc &d, K x) {
    const K *keys = (const K *)d.keys;
    switch (d.form) {
        case F_BS: return bs_find<K>(keys, d.rows, d.n, x);
        case F_EBS: return ebs_find<K>(keys, d.rows, d.n, d.m_full, x);
        case F_EKS: return eks_find<K>(keys, d.rows, d, x);
        default: return learned_find<K>(keys, d.rows, d, x);
    }
}

// Pass 1: point answers; range sizes into offs (scanned afterwards) and the
// first rank of every range.
// Both passes come in two kinds, each launched only when the batch holds
// such indexes, so neither carries the other's registers: EYT = false serves
// the sorted-array forms (BS, learned), EYT = true the Eytzinger forms.
__device__ __forceinline__ bool is_eyt(uint32_t form) { return form == F_EBS || form == F_EKS; }

template <typename K, bool EYT>
__global__ __launch_bounds__(BT) void k_batch_mixed_count(const Desc *__restrict__ descs, const Geo *__restrict__ geos,
                                                          uint32_t count, const uint64_t *__restrict__ off, uint64_t m,
                                                          const K *__restrict__ lo, const K *__restrict__ hi,
                                                          const uint8_t *__restrict__ kind,
                                                          uint32_t *__restrict__ out, uint32_t *__restrict__ first,
                                                          uint64_t *__restrict__ offs) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave_global = ((uint64_t)blockIdx.x * BT + threadIdx.x) / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * (BT / kWave);
    constexpr uint64_t CH = (uint64_t)kWave * BR;
    for (uint64_t c0 = wave_global * CH; c0 < m; c0 += waves * CH) {
        const uint64_t c1 = c0 + CH < m ? c0 + CH : m;
        const uint32_t i0 = owner(off, 0, count, c0);
        const uint32_t i1 = owner(off, i0, count, c1 - 1);
        if constexpr (!EYT) {
            // A chunk of one learned index (the usual case): every model
            // lookup of the lane's queries -- one per point, two per range --
            // runs in lockstep, so their leaf records, narrowing probes and
            // window reads are in flight together.
            if (i0 == i1 && descs[i0].form == F_LEARNED) {
                const Desc d = descs[i0];
                const K *keys = (const K *)d.keys;
                constexpr int NL = 2 * BR;
                K xs[NL];
                bool act[NL], eq[NL];
                uint32_t b[NL], len[NL];  // ranks: n < 2^32
                bool live[BR], rng[BR];
#pragma unroll
                for (int r = 0; r < BR; ++r) {
                    const uint64_t p = c0 + (uint64_t)r * kWave + lane;
                    live[r] = p < c1;
                    rng[r] = live[r] && kind[p] == Q_RANGE;
                    const K L = live[r] ? lo[p] : K(0), U = rng[r] ? hi[p] : K(0);
                    xs[2 * r] = L;
                    act[2 * r] = live[r] && (!rng[r] || L <= U);
                    xs[2 * r + 1] = (K)(U + 1);
                    act[2 * r + 1] = rng[r] && L <= U && U != ~K(0);
                }
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    b[j] = 0;
                    len[j] = 0;
                    if (act[j]) {
                        uint64_t wb, wl;
                        learned_window(d.root, d.leaves, (uint64_t)xs[j], wb, wl);
                        b[j] = (uint32_t)wb;
                        len[j] = (uint32_t)wl;
                    }
                }
                for (;;) {
                    bool more = false;
#pragma unroll
                    for (int j = 0; j < NL; ++j) {
                        if (len[j] > 15) {
                            const uint32_t half = len[j] >> 1;
                            b[j] = keys[(uint64_t)b[j] + half - 1] < xs[j] ? b[j] + half : b[j];
                            len[j] -= half;
                        }
                        more |= len[j] > 15;
                    }
                    if (!more) break;
                }
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    eq[j] = false;
                    if (act[j]) b[j] += count_below<K, 16>(keys, b[j], len[j], xs[j], eq[j]);
                }
#pragma unroll
                for (int r = 0; r < BR; ++r) {
                    if (!live[r]) continue;
                    const uint64_t p = c0 + (uint64_t)r * kWave + lane;
                    if (!rng[r]) {
                        out[p] = eq[2 * r] ? d.rows[b[2 * r]] : kMiss;
                        first[p] = 0;
                        offs[p] = 0;
                        continue;
                    }
                    out[p] = kMiss;
                    const uint64_t r0 = act[2 * r] ? b[2 * r] : 0;
                    const uint64_t r1 = !act[2 * r] ? 0 : act[2 * r + 1] ? b[2 * r + 1] : d.n;
                    first[p] = (uint32_t)r0;
                    offs[p] = r1 > r0 ? r1 - r0 : 0;
                }
                continue;
            }
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const uint64_t p = c0 + (uint64_t)r * kWave + lane;
            if (p >= c1) continue;
            const uint32_t ii = (i0 == i1) ? i0 : owner(off, i0, i1 + 1, p);
            const Desc d = descs[ii];
            if (is_eyt(d.form) != EYT) continue;
            if (kind[p] == Q_POINT) {
                out[p] = form_find_kind<K, EYT>(d, lo[p]);
                first[p] = 0;
                offs[p] = 0;
                continue;
            }
            out[p] = kMiss;
            const K L = lo[p], U = hi[p];
            uint64_t r0 = 0, r1 = 0;
            if (L <= U) {
                const Geo &G = geos[ii];
                r0 = form_lower_rank<K, EYT>(d, G, L);
                r1 = (U == ~K(0)) ? d.n : form_lower_rank<K, EYT>(d, G, (K)(U + 1));
            }
            first[p] = (uint32_t)r0;
            offs[p] = r1 > r0 ? r1 - r0 : 0;
        }
    }
}

// Pass 2: row IDs of every range in key order at its offset.
template <typename K, bool EYT>
__global__ __launch_bounds__(BT) void k_batch_mixed_fill(const Desc *__restrict__ descs, const Geo *__restrict__ geos,
                                                         uint32_t count, const uint64_t *__restrict__ off, uint64_t m,
                                                         const K *__restrict__ lo, const K *__restrict__ hi,
                                                         const uint8_t *__restrict__ kind,
                                                         const uint32_t *__restrict__ first,
                                                         const uint64_t *__restrict__ offs,
                                                         uint32_t *__restrict__ rows_out) {
    // per wave: the start of each lane's run in the wave's concatenation of
    // runs, the run's row IDs, its first rank and destination offset by that
    // start, and where its ranks are stored (sorted array: the rank itself;
    // Eytzinger layouts: the slot the layout build wrote the rank to)
    __shared__ uint32_t s_start[BT / kWave][kWave + 1];
    __shared__ const uint32_t *s_rows[BT / kWave][kWave];
    __shared__ int64_t s_rank0[BT / kWave][kWave];
    __shared__ uint32_t *s_dst[BT / kWave][kWave];
    __shared__ const Geo *s_geo[BT / kWave][kWave];
    __shared__ uint64_t s_kinv[BT / kWave][kWave];
    __shared__ uint32_t s_mode[BT / kWave][kWave];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave_global = ((uint64_t)blockIdx.x * BT + threadIdx.x) / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * (BT / kWave);
    constexpr uint64_t CH = (uint64_t)kWave * BR;
    for (uint64_t c0 = wave_global * CH; c0 < m; c0 += waves * CH) {
        const uint64_t c1 = c0 + CH < m ? c0 + CH : m;
        const uint32_t i0 = owner(off, 0, count, c0);
        const uint32_t i1 = owner(off, i0, count, c1 - 1);
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const uint64_t p = c0 + (uint64_t)r * kWave + lane;
            const bool live = p < c1;
            const uint32_t ii = !live ? 0u : (i0 == i1) ? i0 : owner(off, i0, i1 + 1, p);
            // this lane's run: a sorted-array range is copied by the whole
            // wave below; an Eytzinger range is scanned by its own lane
            const uint32_t *run_rows = nullptr;
            uint64_t run_first = 0, run_out = 0, run_len = 0, run_kinv = 0;
            uint32_t run_mode = MAP_SORTED;
            const Geo *run_geo = nullptr;
            bool paused = false;
            ScanState st{};
            uint64_t scan_o = 0, scan_cnt = 0;
            if (live && kind[p] == Q_RANGE) {
                const uint64_t o = offs[p], cnt = offs[p + 1] - o;
                const Desc d = descs[ii];
                if constexpr (!EYT) {
                    if (cnt > 0 && !is_eyt(d.form)) {
                        run_rows = d.rows;
                        run_first = first[p];
                        run_out = o;
                        run_len = cnt;
                    }
                } else if (cnt > 0 && is_eyt(d.form) && d.rscan == 3) {
                    run_rows = d.rows;
                    run_first = first[p];
                    run_out = o;
                    run_len = cnt;
                    run_mode = d.form == F_EBS ? MAP_BINARY : MAP_KARY;
                    run_geo = geos + ii;
                    run_kinv = d.kinv;
                } else if (cnt > 0 && is_eyt(d.form)) {
                    const Geo &Gi = geos[ii];
                    const uint64_t eoff = d.form == F_EBS ? 1 : 0;
                    if (scan_vec_ok(Gi, eoff, sizeof(K), false)) {
                        paused = eyt_scan_lane_vec((const K *)d.keys, d.rows, Gi, lo[p], hi[p], (uint64_t)first[p],
                                                   cnt, rows_out + o, st);
                    } else {
                        Load<K, false> Ld{};
                        Ld.k = (const K *)d.keys;
                        Ld.r = d.rows;
                        Ld.node = 1;
                        paused = eyt_scan_lane(Ld, Gi, eoff, lo[p], hi[p], (uint64_t)first[p], cnt, rows_out + o, st);
                    }
                    if (paused) {
                        scan_o = o;
                        scan_cnt = cnt;
                    }
                }
            }
            // paused Eytzinger scans continue with the whole wave, one at a time
            uint64_t pend = EYT ? __ballot(paused) : 0ull;
            while (pend) {
                const int src = __builtin_ctzll(pend);
                pend &= pend - 1;
                const uint32_t wi = (uint32_t)__shfl((int)ii, src, kWave);
                const uint64_t wp = (uint64_t)__shfl((long long)p, src, kWave);
                ScanState w;
                w.c = (uint64_t)__shfl((long long)st.c, src, kWave);
                w.t = (uint64_t)__shfl((long long)st.t, src, kWave);
                w.lvl = (uint32_t)__shfl((int)st.lvl, src, kWave);
                w.j = (uint32_t)__shfl((int)st.j, src, kWave);
                const uint64_t wo = (uint64_t)__shfl((long long)scan_o, src, kWave);
                const uint64_t wcnt = (uint64_t)__shfl((long long)scan_cnt, src, kWave);
                const Desc dw = descs[wi];
                Load<K, false> Lw{};
                Lw.k = (const K *)dw.keys;
                Lw.r = dw.rows;
                Lw.node = 1;
                eyt_scan_wave(Lw, geos[wi], dw.form == F_EBS ? 1 : 0, lo[wp], hi[wp], (uint64_t)first[wp], wcnt,
                              rows_out + wo, w);
            }
            // wave-cooperative copy of the lanes' runs: every element finds
            // its run by a binary search over the runs' starts (per wave, in
            // LDS), so the wave copies 64 elements per step with CU
            // independent loads per lane in flight
            {
                const uint32_t w = threadIdx.x / kWave;
                uint32_t len32 = (uint32_t)run_len, incl = len32;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const uint32_t x = (uint32_t)__shfl_up((int)incl, off, kWave);
                    if (lane >= (uint32_t)off) incl += x;
                }
                const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
                if (total > 0) {
                    const uint32_t start = incl - len32;
                    s_start[w][lane] = start;
                    if (lane == kWave - 1) s_start[w][kWave] = total;
                    s_rows[w][lane] = run_rows;
                    s_rank0[w][lane] = (int64_t)run_first - (int64_t)start;
                    s_dst[w][lane] = rows_out + run_out - start;
                    s_geo[w][lane] = run_geo;
                    s_kinv[w][lane] = run_kinv;
                    s_mode[w][lane] = run_mode;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    constexpr int CU = 4;
                    for (uint32_t t0 = lane; t0 < total; t0 += kWave * CU) {
                        uint32_t v[CU], q[CU];
#pragma unroll
                        for (int u = 0; u < CU; ++u) {
                            const uint32_t t = t0 + (uint32_t)u * kWave;
                            uint32_t lo = 0;
#pragma unroll
                            for (uint32_t step = kWave / 2; step > 0; step >>= 1)
                                if (s_start[w][lo + step] <= t) lo += step;
                            q[u] = lo;
                            if (t < total) {
                                const uint64_t rank = (uint64_t)(s_rank0[w][lo] + (int64_t)t);
                                uint64_t slot = rank;
                                if (EYT && s_mode[w][lo] == MAP_BINARY) slot = 1 + rank_slot_binary(*s_geo[w][lo], rank);
                                else if (EYT && s_mode[w][lo] == MAP_KARY)
                                    slot = rank_slot_general(*s_geo[w][lo], rank, s_kinv[w][lo]);
                                v[u] = s_rows[w][lo][slot];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < CU; ++u) {
                            const uint32_t t = t0 + (uint32_t)u * kWave;
                            if (t < total) s_dst[w][q[u]][t] = v[u];
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
        }
    }
}

}  // namespace
}  // namespace idx

struct idx_batch {
    std::vector<idx_index *> members;  // each holds one batch reference for this batch
    idx::Desc *descs = nullptr;  // device
    idx::Geo *geos = nullptr;    // device, one per index (tree geometry for range lookups)
    uint32_t count = 0;
    bool u64 = false;
    bool has_sorted = false;  // holds BS or learned indexes
    bool has_eyt = false;     // holds EBS or EKS indexes
    size_t pin_bytes = 0;     // LDS of the largest member pin table (point launch)
    int cu_count = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_q = nullptr;
    const uint64_t *g_off = nullptr;
    uint32_t *g_out = nullptr;
    hipStream_t g_stream = nullptr;
};

using namespace idx;

namespace {

int launch_batch(idx_batch *b, const void *q, const uint64_t *off, uint32_t *out, hipStream_t s) {
    // persistent grid: 8 workgroups of 4 waves per CU
    const uint32_t grid = (uint32_t)b->cu_count * 8;
    const size_t lds = (b->pin_bytes + 15) & ~(size_t)15;
    if (b->u64)
        hipLaunchKernelGGL(k_batch_point<uint64_t>, dim3(grid), dim3(BT), lds, s, b->descs, b->count, off,
                           (const uint64_t *)q, out);
    else
        hipLaunchKernelGGL(k_batch_point<uint32_t>, dim3(grid), dim3(BT), lds, s, b->descs, b->count, off,
                           (const uint32_t *)q, out);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

void drop_graph(idx_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_q = nullptr;
    b->g_off = nullptr;
    b->g_out = nullptr;
}

}  // namespace

extern "C" {

int idx_batch_create(const idx_handle *indexes, uint32_t count, idx_stream stream, idx_batch_t *out) {
    if (!out) return IDX_ERR_ARG;
    *out = nullptr;
    if (!indexes || count == 0) return IDX_ERR_ARG;
    const bool u64 = indexes[0] && indexes[0]->u64;
    std::vector<Desc> host;
    try {
        host.resize(count);
    } catch (...) {
        return IDX_ERR_NOMEM;
    }
    for (uint32_t i = 0; i < count; ++i) {
        idx_index *h = indexes[i];
        if (!h || h->u64 != u64 || h->aos) return IDX_ERR_ARG;
        Desc d{};
        d.keys = h->keys;
        d.rows = h->rowids;
        d.n = h->n;
        d.k = h->geo.k;
        d.g = h->geo.g;
        d.levels = h->geo.levels;
        d.m_full = h->geo.m;
        d.gshift = (uint32_t)h->geo.gshift;
        d.early = (h->unique && h->params.early_exit == 1) ? 1u : 0u;
        // lookup parameters the batch takes from the member: EKS lanes per
        // lookup, and the top levels pinned in LDS (its pin table)
        d.lanes = h->layout == IDX_EKS ? h->params.group : 1u;
        d.vec = (h->layout == IDX_EKS && scan_vec_ok(h->geo, 0, h->u64 ? 8 : 4, false)) ? 1u : 0u;
        d.rscan = h->params.range_scan;
        d.kinv = h->geo.k > 2 ? ~0ull / h->geo.k + 1 : 0;  // ceil(2^64 / k)
        if (h->params.lds_levels && !(h->learned && h->params.model != 2)) {
            const int rc = build_pin(h, h->params.lds_levels, (hipStream_t)stream);
            if (rc != IDX_OK) return rc;
            d.pin = h->pin;
            d.pin_levels = h->params.lds_levels;
            d.pin_keys = h->pin_keys;
        }
        if (h->layout == IDX_BS) {
            d.form = F_BS;
            if (h->learned && h->params.model != 2) {
                d.form = F_LEARNED;
                d.leaves = model_leaves(h);
                d.root = model_root(h);
            }
        } else if (h->layout == IDX_EBS) {
            d.form = F_EBS;
        } else {
            d.form = F_EKS;
        }
        host[i] = d;
    }
    idx_batch *b = new (std::nothrow) idx_batch();
    if (!b) return IDX_ERR_NOMEM;
    b->count = count;
    b->u64 = u64;
    for (uint32_t i = 0; i < count; ++i) {
        if (host[i].form == F_EBS || host[i].form == F_EKS) b->has_eyt = true;
        else b->has_sorted = true;
        const size_t pb = (size_t)host[i].pin_keys * (u64 ? 8 : 4);
        if (pb > b->pin_bytes) b->pin_bytes = pb;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->cu_count = cus;
    (void)hipGetLastError();
    std::vector<Geo> geos;
    try {
        geos.resize(count);
    } catch (...) {
        delete b;
        return IDX_ERR_NOMEM;
    }
    for (uint32_t i = 0; i < count; ++i) geos[i] = indexes[i]->geo;
    if (hipMalloc((void **)&b->descs, sizeof(Desc) * count) != hipSuccess ||
        hipMalloc((void **)&b->geos, sizeof(Geo) * count) != hipSuccess) {
        (void)hipGetLastError();
        if (b->descs) (void)hipFree(b->descs);
        delete b;
        return IDX_ERR_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(b->descs, host.data(), sizeof(Desc) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->geos, geos.data(), sizeof(Geo) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        try {
            b->members.assign(indexes, indexes + count);
        } catch (...) {
            e = hipErrorOutOfMemory;
        }
    }
    if (e == hipSuccess) {
        // the descriptors point at the members' buffers: pin them
        for (idx_index *h : b->members) ++h->batch_refs;
        *out = b;
        return IDX_OK;
    }
    (void)hipFree(b->descs);
    (void)hipFree(b->geos);
    delete b;
    return hip_fail(e);
}

int idx_batch_point(idx_batch_t b, const void *queries, const uint64_t *offsets, uint32_t *out_rowid, uint32_t flags,
                    idx_stream stream) {
    if (!b || !offsets || (flags & ~IDX_BATCH_GRAPH)) return IDX_ERR_ARG;
    if (!queries || !out_rowid) return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (!(flags & IDX_BATCH_GRAPH)) return launch_batch(b, queries, offsets, out_rowid, s);
    if (!b->exec || b->g_q != queries || b->g_off != offsets || b->g_out != out_rowid || b->g_stream != s) {
        drop_graph(b);
        hipStream_t cs = nullptr;
        IDX_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        int rc = IDX_OK;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = launch_batch(b, queries, offsets, out_rowid, cs);
            e = hipStreamEndCapture(cs, &b->graph);
        }
        if (e == hipSuccess && rc == IDX_OK) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess || rc != IDX_OK) {
            drop_graph(b);
            return rc != IDX_OK ? rc : hip_fail(e);
        }
        b->g_q = queries;
        b->g_off = offsets;
        b->g_out = out_rowid;
        b->g_stream = s;
    }
    IDX_HIP(hipGraphLaunch(b->exec, s));
    return IDX_OK;
}

int idx_batch_mixed(idx_batch_t b, uint64_t m, const void *lo, const void *hi, const uint8_t *kind,
                    const uint64_t *offsets, uint32_t *out_rowid, uint64_t *range_offsets, uint32_t *range_rowids,
                    uint64_t capacity, uint64_t *total, idx_stream stream) {
    if (!b || !offsets || !range_offsets) return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (m == 0) {
        IDX_HIP(hipMemsetAsync(range_offsets, 0, sizeof(uint64_t), s));
        if (total) *total = 0;
        return IDX_OK;
    }
    if (!lo || !hi || !kind || !out_rowid || m > 0xFFFFFFFFull) return IDX_ERR_ARG;
    const uint64_t parts = scan_partials_for(m);
    char *tmp = nullptr;
    const size_t first_b = ((size_t)m * 4 + 255) & ~(size_t)255;
    IDX_HIP(hipMallocAsync((void **)&tmp, first_b + parts * 8, s));
    uint32_t *first = (uint32_t *)tmp;
    uint64_t *partial = (uint64_t *)(tmp + first_b);
    const uint32_t grid = (uint32_t)b->cu_count * 8;
    int rc = IDX_OK;
    do {
        for (int e = 0; e < 2; ++e) {
            if (!(e ? b->has_eyt : b->has_sorted)) continue;
            if (b->u64) {
                const auto kern = e ? k_batch_mixed_count<uint64_t, true> : k_batch_mixed_count<uint64_t, false>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(BT), 0, s, b->descs, b->geos, b->count, offsets, m,
                                   (const uint64_t *)lo, (const uint64_t *)hi, kind, out_rowid, first, range_offsets);
            } else {
                const auto kern = e ? k_batch_mixed_count<uint32_t, true> : k_batch_mixed_count<uint32_t, false>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(BT), 0, s, b->descs, b->geos, b->count, offsets, m,
                                   (const uint32_t *)lo, (const uint32_t *)hi, kind, out_rowid, first, range_offsets);
            }
        }
        if (hipGetLastError() != hipSuccess) {
            rc = IDX_ERR_HIP;
            break;
        }
        rc = exclusive_scan_u64(range_offsets, m, partial, s);
        if (rc != IDX_OK) break;
        uint64_t tot = 0;
        if (hipMemcpyAsync(&tot, range_offsets + m, sizeof(tot), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = IDX_ERR_HIP;
            break;
        }
        if (total) *total = tot;
        if (tot == 0 || !range_rowids) break;  // nothing to write, or counts only
        if (tot > capacity) {
            rc = IDX_ERR_CAPACITY;
            break;
        }
        for (int e = 0; e < 2; ++e) {
            if (!(e ? b->has_eyt : b->has_sorted)) continue;
            if (b->u64) {
                const auto kern = e ? k_batch_mixed_fill<uint64_t, true> : k_batch_mixed_fill<uint64_t, false>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(BT), 0, s, b->descs, b->geos, b->count, offsets, m,
                                   (const uint64_t *)lo, (const uint64_t *)hi, kind, first, range_offsets, range_rowids);
            } else {
                const auto kern = e ? k_batch_mixed_fill<uint32_t, true> : k_batch_mixed_fill<uint32_t, false>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(BT), 0, s, b->descs, b->geos, b->count, offsets, m,
                                   (const uint32_t *)lo, (const uint32_t *)hi, kind, first, range_offsets, range_rowids);
            }
        }
        if (hipGetLastError() != hipSuccess) rc = IDX_ERR_HIP;
    } while (0);
    (void)hipFreeAsync(tmp, s);
    return rc;
}

int idx_batch_destroy(idx_batch_t b) {
    if (!b) return IDX_OK;
    (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->geos) (void)hipFree(b->geos);
    if (b->descs) (void)hipFree(b->descs);
    (void)hipGetLastError();
    for (idx_index *h : b->members) --h->batch_refs;
    delete b;
    return IDX_OK;
}

}  // extern "C"
