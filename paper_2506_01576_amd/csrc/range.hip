// Batched range lookups [lo, hi] returning row IDs in key order.
//
// Three phases:
//  1. count: per query, the sorted rank of the first key >= lo and of the
//     first key > hi (a lower-bound descent for each; on the Eytzinger
//     layouts the rank of the descent's slot t is slot_rank(t)), giving the
//     match count; the first rank is kept in a scratch array;
//  2. exclusive scan of the counts into the caller's offsets (u64);
//  3. fill: BS copies the contiguous rowid run.  EBS/EKS either gather by
//     rank (default): the matches are the ranks [first, first + count), and
//     rank r sits at the level-order slot the layout build wrote it to (the
//     inverse of slot_rank, evaluated in closed form), so each row ID is read
//     from that slot without reading a key; or run the level scan of
//     Section 5: follow the lower-bound path of lo and, on every level, scan
//     right from the path position while keys are <= hi and the level has not
//     ended (qualifying entries of a level are contiguous, and at most two
//     extra entries per level are read).  The scan meets the matches in level
//     order; each is written at offset + slot_rank(t) - first rank, which puts
//     the query's rowids in key order.
// The count searches both bounds of a range in lockstep: the two descents
// read the same nodes (or keys) until their paths part, near the bottom.
// EBS is handled as the k = 2 level-order tree shifted by its empty slot.
#include "internal.hpp"
#include "access.hpp"
#include "range_scan.hpp"
#include "search.hpp"
#include "qio.hpp"

namespace idx {
namespace {

template <typename K, bool AOS>
struct RangeArgs {
    Load<K, AOS> L;
    Geo G;
    uint32_t off;  // layout slot of level-order slot 0 (1 for EBS)
    int layout;
    const K *__restrict__ lo;
    const K *__restrict__ hi;
    uint64_t m;
    uint64_t *__restrict__ offsets;
    uint32_t *__restrict__ first_rank;
    uint32_t *__restrict__ out;
    uint32_t handover;  // level matches after which a lane hands its scan to the wave
    uint64_t kinv;      // ceil(2^64 / k) for the rank-to-slot map (k > 2)
};

// Sorted array: lower-bound ranks of x0 and x1 >= x0 by two binary searches
// in lockstep; while their intervals coincide the second reads nothing of
// its own.  The SoA array stops at a window of at most 15 keys and reads it
// with independent 16-byte loads (the short-window scan).
// Both lower bounds are known to lie in [base, base + len] (base + len <= n).
template <typename K, bool AOS>
__device__ __forceinline__ void bs_ranks_in(const RangeArgs<K, AOS> &a, uint64_t base, uint64_t len, K x0, K x1,
                                            uint64_t &r0, uint64_t &r1) {
    const uint64_t n = a.G.n;
    uint64_t b0 = base, b1 = base;
    const uint64_t stop = AOS ? 1 : 15;
    while (len > stop) {
        const uint64_t half = len >> 1;
        const K k0 = a.L.key(b0 + half);
        const K k1 = b1 == b0 ? k0 : a.L.key(b1 + half);
        b0 = k0 < x0 ? b0 + half : b0;
        b1 = k1 < x1 ? b1 + half : b1;
        len -= half;
    }
    if constexpr (!AOS) {
        bool eq;
        const uint64_t s0 = (len + 1) < (n - b0) ? (len + 1) : (n - b0);
        const uint64_t s1 = (len + 1) < (n - b1) ? (len + 1) : (n - b1);
        r0 = b0 + count_below<K, 16>(a.L.k, b0, (uint32_t)s0, x0, eq);
        r1 = b1 + count_below<K, 16>(a.L.k, b1, (uint32_t)s1, x1, eq);
    } else {
        r0 = b0 + (b0 < n && a.L.key(b0) < x0 ? 1 : 0);
        r1 = b1 + (b1 < n && a.L.key(b1) < x1 ? 1 : 0);
    }
}

template <typename K, bool AOS>
__device__ __forceinline__ void bs_ranks(const RangeArgs<K, AOS> &a, K x0, K x1, uint64_t &r0, uint64_t &r1) {
    bs_ranks_in(a, 0, a.G.n, x0, x1, r0, r1);
}

// Eytzinger layouts: lower-bound ranks of x0 and of x1 >= x0 (when `two`),
// as the rank of the deepest path position whose pivot is >= the bound.  The
// two descents share each node until their paths part; a node is read once
// with 16-byte loads when the nodes allow it.
template <typename K, bool AOS>
__device__ __forceinline__ void eyt_ranks(const RangeArgs<K, AOS> &a, K x0, K x1, bool two, uint64_t &r0,
                                          uint64_t &r1) {
    const uint64_t n = a.G.n;
    const uint32_t g = a.G.g, kf = a.G.k;
    uint64_t c0 = 0, c1 = 0, cand0 = ~0ull, cand1 = ~0ull;
    if constexpr (!AOS) {
        if (scan_vec_ok(a.G, a.off, sizeof(K), false)) {  // whole nodes in registers
            constexpr int NK = kScanNodeBytes / sizeof(K);
            K kk0[NK], kk1[NK];
            for (;;) {
                const uint64_t i0 = c0 * g, i1 = c1 * g;
                const bool l0 = i0 < n, l1 = two && i1 < n;
                if (!l0 && !l1) break;
                if (l0) node_keys(a.L.k, i0, g, kk0);
                if (l1 && c1 != c0) node_keys(a.L.k, i1, g, kk1);
                if (l0) {
                    const uint32_t nv = (n - i0) < g ? (uint32_t)(n - i0) : g;
                    const uint32_t j = node_below(kk0, nv, x0);
                    if (l1 && c1 == c0) {
                        const uint32_t j1 = node_below(kk0, nv, x1);
                        if (j1 < nv) cand1 = i1 + j1;
                        c1 = c1 * kf + 1 + j1;
                    }
                    if (j < nv) cand0 = i0 + j;
                    c0 = c0 * kf + 1 + j;
                    if (l1 && i1 != i0) {
                        const uint32_t nv1 = (n - i1) < g ? (uint32_t)(n - i1) : g;
                        const uint32_t j1 = node_below(kk1, nv1, x1);
                        if (j1 < nv1) cand1 = i1 + j1;
                        c1 = c1 * kf + 1 + j1;
                    }
                } else {
                    const uint32_t nv1 = (n - i1) < g ? (uint32_t)(n - i1) : g;
                    const uint32_t j1 = node_below(kk1, nv1, x1);
                    if (j1 < nv1) cand1 = i1 + j1;
                    c1 = c1 * kf + 1 + j1;
                }
            }
            r0 = cand0 == ~0ull ? n : slot_rank(a.G, cand0);
            r1 = cand1 == ~0ull ? n : slot_rank(a.G, cand1);
            return;
        }
    }
    for (;;) {
        const uint64_t i0 = c0 * g, i1 = c1 * g;
        const bool l0 = i0 < n, l1 = two && i1 < n;
        if (!l0 && !l1) break;
        const uint64_t nv0 = l0 ? ((n - i0) < g ? (n - i0) : g) : 0;
        const uint64_t nv1 = l1 ? ((n - i1) < g ? (n - i1) : g) : 0;
        const bool same = l1 && c1 == c0;
        uint32_t j0 = 0, j1 = 0;
        for (uint32_t e = 0; e < g; ++e) {
            if (e < nv0) {
                const K k = a.L.key(a.off + i0 + e);
                j0 += k < x0 ? 1u : 0u;
                if (same) j1 += k < x1 ? 1u : 0u;
            }
            if (!same && e < nv1) j1 += a.L.key(a.off + i1 + e) < x1 ? 1u : 0u;
        }
        if (l0) {
            if (j0 < nv0) cand0 = i0 + j0;
            c0 = c0 * kf + 1 + j0;
        }
        if (l1) {
            if (j1 < nv1) cand1 = i1 + j1;
            c1 = c1 * kf + 1 + j1;
        }
    }
    r0 = cand0 == ~0ull ? n : slot_rank(a.G, cand0);
    r1 = cand1 == ~0ull ? n : slot_rank(a.G, cand1);
}

// First rank r0 of the range [L, U] and the rank r1 past its last match
// (r0 = r1 = 0 when L > U).
template <typename K, bool AOS>
__device__ __forceinline__ void range_ranks(const RangeArgs<K, AOS> &a, K L, K U, uint64_t &r0, uint64_t &r1) {
    r0 = 0;
    r1 = 0;
    if (L > U || a.G.n == 0) return;
    const bool top = U == key_max<K>();  // nothing is above U: r1 = n
    const K x1 = top ? U : (K)(U + 1);
    if (a.layout == IDX_BS) bs_ranks(a, L, x1, r0, r1);
    else eyt_ranks(a, L, x1, !top, r0, r1);
    if (top) r1 = a.G.n;
}

template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_range_count(RangeArgs<K, AOS> a) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.m) return;
    uint64_t r0, r1;
    range_ranks(a, a.lo[q], a.hi[q], r0, r1);
    a.first_rank[q] = (uint32_t)r0;
    a.offsets[q] = r1 > r0 ? r1 - r0 : 0;
}

// The same on a batch of ranges partitioned by the rank bucket of their
// lower bounds (lookup parameter reorder = 2): entry j holds lower bound
// q2[j] of the range at batch position pos[j], whose upper bound is read
// there (reading the upper bounds into partitioned order first, in a kernel
// of their own, cost more).  The tiles are walked XCD by XCD, so the ranges one XCD has in
// flight fall in a few buckets whose slice of the index stays in its L2.
// Both ranks go out in partitioned order, one 8-byte pair per range;
// k_range_put then writes each range's first rank and count at its position
// (random writes in a kernel of their own cost less than inside this one,
// where they slow the searches, or than two placement passes).
// On the sorted array the lower bound's bucket bounds its rank (see
// bucket_start): both searches start inside that interval, and the upper
// bound's search widens to the rest of the array only when its answer is
// past the interval (a range that leaves the bucket).
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_range_count_part(RangeArgs<K, AOS> a, const K *__restrict__ q2,
                                                          const uint32_t *__restrict__ pos,
                                                          const uint16_t *__restrict__ bkt, uint64_t bstep,
                                                          uint64_t bspan, uint64_t ntiles, uint64_t iters,
                                                          uint2 *__restrict__ ranks) {
    for (uint64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, ntiles, 1);
        if (tl >= ntiles) continue;
        const uint64_t j = tl * 256 + threadIdx.x;
        if (j >= a.m) continue;
        const K L = q2[j], U = a.hi[pos[j]];
        uint64_t r0 = 0, r1 = 0;
        if (a.layout == IDX_BS && L <= U) {
            const bool top = U == key_max<K>();
            const K x1 = top ? U : (K)(U + 1);
            const uint64_t base = bucket_start(bkt[j], bstep);
            bs_ranks_in(a, base, bspan, L, x1, r0, r1);
            // the window scan may also count the key at base + bspan, so an
            // answer past the interval shows as end or end + 1
            const uint64_t end = base + bspan;
            if (r1 >= end && end < a.G.n) {
                uint64_t unused;
                bs_ranks_in(a, end, a.G.n - end, x1, x1, r1, unused);
            }
            if (top) r1 = a.G.n;
        } else {
            range_ranks(a, L, U, r0, r1);
        }
        ranks[j] = make_uint2((uint32_t)r0, (uint32_t)r1);
    }
}

// Each range's first rank and count at its position, packed into one 8-byte
// word (first rank << 32 | count; both are below 2^32): one random write per
// range instead of two.  The scan that follows unpacks them.
__global__ __launch_bounds__(256) void k_range_put(const uint2 *__restrict__ ranks, const uint32_t *__restrict__ pos,
                                                   uint64_t m, uint64_t *__restrict__ packed) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint2 r = ranks[j];
    const uint32_t cnt = r.y > r.x ? r.y - r.x : 0u;
    packed[pos[j]] = ((uint64_t)r.x << 32) | cnt;
}

// Counts through the partition: per chunk of at most 2^31 ranges, partition
// the lower bounds, count in partitioned order, then write each range's
// packed first rank and count at its position (the scan unpacks them).
template <typename K, bool AOS>
int range_count_partitioned(idx_index *h, const RangeArgs<K, AOS> &a, hipStream_t s) {
    const uint64_t m = a.m;
    const uint64_t chunk = m < kPartChunk ? m : kPartChunk;
    const size_t pb = (partition_scratch_bytes(h, chunk) + 255) & ~(size_t)255;
    char *t = (char *)h->alloc.get(pb + (size_t)chunk * 8, s);
    if (!t) return IDX_ERR_NOMEM;
    uint2 *ranks = (uint2 *)(t + pb);  // both ranks of every range, partitioned order
    int rc = IDX_OK;
    for (uint64_t c0 = 0; c0 < m && rc == IDX_OK; c0 += chunk) {
        const uint64_t mc = (m - c0) < chunk ? (m - c0) : chunk;
        PartView v{};
        rc = partition_forward(h, a.lo + c0, mc, t, &v, s);
        if (rc != IDX_OK) break;
        RangeArgs<K, AOS> b = a;
        b.hi = a.hi + c0;
        b.m = mc;
        const uint64_t tiles = (mc + 255) / 256;
        const uint64_t iters = ((tiles + kXcds - 1) / kXcds) * kXcds;
        hipLaunchKernelGGL((k_range_count_part<K, AOS>), dim3((uint32_t)iters), dim3(256), 0, s, b, (const K *)v.q,
                           v.pos, v.bkt, v.bstep, v.bspan, tiles, iters, ranks);
        hipLaunchKernelGGL(k_range_put, dim3((uint32_t)tiles), dim3(256), 0, s, (const uint2 *)ranks, v.pos, mc,
                           a.offsets + c0);
        if (hipGetLastError() != hipSuccess) rc = IDX_ERR_HIP;
    }
    h->alloc.put(t, s);
    return rc;
}

// Where the entry of sorted rank r sits: the sorted array itself (BS and the
// learned form), or the level-order slot the layout build wrote it to.
enum : int { MAP_SORTED = 0, MAP_BINARY = 1, MAP_KARY = 2 };

template <int MAP, typename K, bool AOS>
__device__ __forceinline__ uint64_t slot_of_rank(const RangeArgs<K, AOS> &a, uint64_t r) {
    if constexpr (MAP == MAP_SORTED) return r;
    else if constexpr (MAP == MAP_BINARY) return a.off + rank_slot_binary(a.G, r);
    else return a.off + rank_slot_general(a.G, r, a.kinv);
}

// Each wave takes 64 consecutive queries, whose row-ID runs are consecutive
// in the output, and copies their concatenation: every element finds its run
// by a binary search over the runs' starts (per wave, in LDS), so stores are
// coalesced and each lane has several loads in flight.  The run of a range
// is its ranks [first, first + count); MAP says where each rank is stored.
template <typename K, bool AOS, int MAP>
__global__ __launch_bounds__(256) void k_range_fill_rank(RangeArgs<K, AOS> a) {
    constexpr int WPB = 256 / kWave;
    __shared__ uint64_t s_start[WPB][kWave + 1];
    __shared__ uint64_t s_src[WPB][kWave];  // first rank of the run minus its start
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t q0 = ((uint64_t)blockIdx.x * WPB + w) * kWave;
    if (q0 >= a.m) return;  // whole wave: q0 is wave-uniform
    const uint64_t q = q0 + lane;
    uint64_t len = 0, r0 = 0;
    if (q < a.m) {
        len = a.offsets[q + 1] - a.offsets[q];
        r0 = a.first_rank[q];
    }
    uint64_t incl = len;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t x = (uint64_t)__shfl_up((long long)incl, off, kWave);
        if (lane >= (uint32_t)off) incl += x;
    }
    const uint64_t total = (uint64_t)__shfl((long long)incl, kWave - 1, kWave);
    if (total == 0) return;
    const uint64_t start = incl - len;
    s_start[w][lane] = start;
    if (lane == kWave - 1) s_start[w][kWave] = total;
    s_src[w][lane] = r0 - start;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t *out = a.out + a.offsets[q0];
    constexpr int CU = 4;
    for (uint64_t t0 = lane; t0 < total; t0 += (uint64_t)kWave * CU) {
        uint32_t v[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const uint64_t t = t0 + (uint64_t)u * kWave;
            if (t >= total) continue;
            uint32_t lo = 0;
#pragma unroll
            for (uint32_t step = kWave / 2; step > 0; step >>= 1)
                if (s_start[w][lo + step] <= t) lo += step;
            v[u] = a.L.row(slot_of_rank<MAP>(a, s_src[w][lo] + t));
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const uint64_t t = t0 + (uint64_t)u * kWave;
            if (t < total) out[t] = v[u];
        }
    }
}

// EBS/EKS: level scan along the lower-bound path of lo, one lane per range,
// switching to the whole wave for ranges with many matches per level
// (hybrid coalesced scanning, range_scan.hpp).
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_range_fill_eyt(RangeArgs<K, AOS> a) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t o = 0, cnt = 0, r0 = 0;
    K L = 0, U = 0;
    if (q < a.m) {
        o = a.offsets[q];
        cnt = a.offsets[q + 1] - o;
        L = a.lo[q];
        U = a.hi[q];
        r0 = a.first_rank[q];
    }
    ScanState st{};
    bool paused = false;
    if (cnt > 0) {
        if constexpr (!AOS) {
            if (scan_vec_ok(a.G, a.off, sizeof(K), false))
                paused = eyt_scan_lane_vec(a.L.k, a.L.r, a.G, L, U, r0, cnt, a.out + o, st, a.handover);
            else
                paused = eyt_scan_lane(a.L, a.G, a.off, L, U, r0, cnt, a.out + o, st, a.handover);
        } else {
            paused = eyt_scan_lane(a.L, a.G, a.off, L, U, r0, cnt, a.out + o, st, a.handover);
        }
    }
    // every lane of the wave reaches this point: continue paused scans together
    uint64_t pend = __ballot(paused);
    while (pend) {
        const int src = __builtin_ctzll(pend);
        pend &= pend - 1;
        ScanState w;
        w.c = (uint64_t)__shfl((long long)st.c, src, kWave);
        w.t = (uint64_t)__shfl((long long)st.t, src, kWave);
        w.lvl = (uint32_t)__shfl((int)st.lvl, src, kWave);
        w.j = (uint32_t)__shfl((int)st.j, src, kWave);
        const K wl = (K)__shfl((long long)(uint64_t)L, src, kWave);
        const K wu = (K)__shfl((long long)(uint64_t)U, src, kWave);
        const uint64_t wr0 = (uint64_t)__shfl((long long)r0, src, kWave);
        const uint64_t wcnt = (uint64_t)__shfl((long long)cnt, src, kWave);
        const uint64_t wo = (uint64_t)__shfl((long long)o, src, kWave);
        eyt_scan_wave(a.L, a.G, a.off, wl, wu, wr0, wcnt, a.out + wo, w);
    }
}

// ------------------------------------------------------------- u64 scan

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;
static_assert(SC_TILE == kScanTile, "range_scratch_bytes sizes the scan partials by this tile");

__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t *s_wave, uint64_t *total) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    uint64_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t t = __shfl_up(incl, off, kWave);
        if (lane >= (uint32_t)off) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint64_t before = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < SC_THREADS / kWave; ++w) {
        const uint64_t c = s_wave[w];
        before += (w < (int)wave) ? c : 0;
        sum += c;
    }
    __syncthreads();
    *total = sum;
    return before + incl - v;
}

// PACKED: each value is (first rank << 32 | count) and only the count is
// summed (k_range_put's words).
template <bool PACKED>
__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const uint64_t *__restrict__ v, uint64_t m,
                                                            uint64_t *__restrict__ partial) {
    __shared__ uint64_t s_wave[SC_THREADS / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * SC_THREADS + threadIdx.x;
        const uint64_t x = i < m ? v[i] : 0;
        sum += PACKED ? (x & 0xFFFFFFFFull) : x;
    }
    uint64_t total;
    block_scan_u64(sum, s_wave, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the per-tile partial sums in place.
__global__ __launch_bounds__(SC_THREADS) void k_scan_partials(uint64_t *__restrict__ partial, uint64_t tiles) {
    __shared__ uint64_t s_wave[SC_THREADS / kWave];
    uint64_t running = 0;
    for (uint64_t chunk = 0; chunk < tiles; chunk += SC_TILE) {
        uint64_t v[SC_ITEMS], sum = 0;
        const uint64_t first = chunk + (uint64_t)threadIdx.x * SC_ITEMS;
#pragma unroll
        for (int j = 0; j < SC_ITEMS; ++j) {
            v[j] = first + j < tiles ? partial[first + j] : 0;
            sum += v[j];
        }
        uint64_t total;
        uint64_t acc = running + block_scan_u64(sum, s_wave, &total);
#pragma unroll
        for (int j = 0; j < SC_ITEMS; ++j) {
            if (first + j < tiles) partial[first + j] = acc;
            acc += v[j];
        }
        running += total;
    }
}

// Tile-local exclusive scan plus the tile's prefix; writes offsets[m] = total.
// PACKED: the values are k_range_put's words; the counts are scanned and the
// first ranks written to `first`.
template <bool PACKED>
__global__ __launch_bounds__(SC_THREADS) void k_scan_apply(uint64_t *__restrict__ v, uint64_t m,
                                                           const uint64_t *__restrict__ partial,
                                                           uint32_t *__restrict__ first) {
    __shared__ uint64_t s_wave[SC_THREADS / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    // a thread's items are consecutive: whole ones move as 16-byte loads and
    // stores (a per-element store is one memory request each)
    const bool vec = base + SC_ITEMS <= m && ((uintptr_t)v & 15) == 0;
    uint64_t x[SC_ITEMS], sum = 0;
    if (vec) {
        const uint4 *p = (const uint4 *)(v + base);
#pragma unroll
        for (int c = 0; c < SC_ITEMS / 2; ++c) {
            const uint4 w = p[c];
            x[2 * c] = ((uint64_t)w.y << 32) | w.x;
            x[2 * c + 1] = ((uint64_t)w.w << 32) | w.z;
        }
    } else {
#pragma unroll
        for (int j = 0; j < SC_ITEMS; ++j) x[j] = base + j < m ? v[base + j] : 0;
    }
    if constexpr (PACKED) {
        uint32_t f[SC_ITEMS];
#pragma unroll
        for (int j = 0; j < SC_ITEMS; ++j) {
            f[j] = (uint32_t)(x[j] >> 32);
            x[j] &= 0xFFFFFFFFull;
        }
        if (vec) {  // `first` is 256-byte aligned and base a multiple of 16
            uint4 *q = (uint4 *)(first + base);
#pragma unroll
            for (int c = 0; c < SC_ITEMS / 4; ++c) q[c] = make_uint4(f[4 * c], f[4 * c + 1], f[4 * c + 2], f[4 * c + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < SC_ITEMS; ++j)
                if (base + j < m) first[base + j] = f[j];
        }
    }
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) sum += x[j];
    uint64_t total;
    uint64_t acc = partial[blockIdx.x] + block_scan_u64(sum, s_wave, &total);
    uint64_t o[SC_ITEMS];
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
        o[j] = acc;
        acc += x[j];
    }
    if (vec) {
        uint4 *p = (uint4 *)(v + base);
#pragma unroll
        for (int c = 0; c < SC_ITEMS / 2; ++c)
            p[c] = make_uint4((uint32_t)o[2 * c], (uint32_t)(o[2 * c] >> 32), (uint32_t)o[2 * c + 1],
                              (uint32_t)(o[2 * c + 1] >> 32));
    } else {
#pragma unroll
        for (int j = 0; j < SC_ITEMS; ++j)
            if (base + j < m) v[base + j] = o[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SC_THREADS - 1) v[m] = acc;
}

// Exclusive scan of v[0, m) in place, v[m] = total.  With `first`, v holds
// k_range_put's packed words: the counts are scanned and the first ranks go
// to first[0, m).
int exclusive_scan(uint64_t *v, uint64_t m, uint64_t *partial, hipStream_t s, uint32_t *first = nullptr) {
    const uint64_t tiles = (m + SC_TILE - 1) / SC_TILE;
    if (first)
        hipLaunchKernelGGL(k_scan_reduce<true>, dim3((uint32_t)tiles), dim3(SC_THREADS), 0, s, v, m, partial);
    else
        hipLaunchKernelGGL(k_scan_reduce<false>, dim3((uint32_t)tiles), dim3(SC_THREADS), 0, s, v, m, partial);
    IDX_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SC_THREADS), 0, s, partial, tiles);
    IDX_LAUNCH_CHECK();
    if (first)
        hipLaunchKernelGGL(k_scan_apply<true>, dim3((uint32_t)tiles), dim3(SC_THREADS), 0, s, v, m, partial, first);
    else
        hipLaunchKernelGGL(k_scan_apply<false>, dim3((uint32_t)tiles), dim3(SC_THREADS), 0, s, v, m, partial,
                           (uint32_t *)nullptr);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS>
int range_t(idx_index *h, const void *lo, const void *hi, uint64_t m, uint64_t *offsets, uint32_t *out,
            uint64_t capacity, uint64_t *total, char *given, hipStream_t s) {
    RangeArgs<K, AOS> a{};
    a.L = make_load<K, AOS>(h);
    a.G = h->geo;
    a.off = h->layout == IDX_EBS ? 1u : 0u;
    a.layout = h->layout;
    a.lo = (const K *)lo;
    a.hi = (const K *)hi;
    a.m = m;
    a.offsets = offsets;
    a.out = out;
    a.handover = h->params.range_scan == 2 ? kNoHandover : kHandover;
    a.kinv = h->geo.k > 2 ? ~0ull / h->geo.k + 1 : 0;  // ceil(2^64 / k)
    const size_t rank_bytes = ((m * 4 + 255) / 256) * 256;
    char *scratch = given ? given : (char *)h->alloc.get(range_scratch_bytes(m), s);
    if (!scratch) return IDX_ERR_NOMEM;
    a.first_rank = (uint32_t *)scratch;
    uint64_t *partial = (uint64_t *)(scratch + rank_bytes);
    int rc = IDX_OK;
    uint64_t tot = 0;
    bool packed = false;  // offsets hold k_range_put's packed words
    const uint32_t blocks = (uint32_t)((m + 255) / 256);
    do {
        if (h->learned && h->params.model != 2) {
            // the no-allocation entry point uses leaf lines only when they
            // exist already (writing them would allocate)
            rc = range_count_learned(h, lo, hi, m, a.first_rank, offsets, given == nullptr, s);
            if (rc != IDX_OK) break;
        } else if (h->params.reorder >= 2 && !given && h->n >= 4) {
            // the caller-given scratch (no-allocation entry point) has no room
            // for the partition: those calls count unpartitioned
            rc = range_count_partitioned(h, a, s);
            if (rc != IDX_OK) break;
            packed = true;
        } else {
            hipLaunchKernelGGL((k_range_count<K, AOS>), dim3(blocks), dim3(256), 0, s, a);
            if (hipGetLastError() != hipSuccess) {
                rc = IDX_ERR_HIP;
                break;
            }
        }
        rc = exclusive_scan(offsets, m, partial, s, packed ? a.first_rank : nullptr);
        if (rc != IDX_OK) break;
        hipError_t e = hipMemcpyAsync(&tot, offsets + m, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e);
            break;
        }
        if (total) *total = tot;
        if (!out || tot == 0) break;
        if (tot > capacity) {
            rc = IDX_ERR_CAPACITY;
            break;
        }
        const uint32_t wblocks = (uint32_t)(((m + kWave - 1) / kWave + 3) / 4);
        if (h->layout == IDX_BS) {
            hipLaunchKernelGGL((k_range_fill_rank<K, AOS, MAP_SORTED>), dim3(wblocks), dim3(256), 0, s, a);
        } else if (h->params.range_scan == 3) {
            if (h->geo.k == 2)
                hipLaunchKernelGGL((k_range_fill_rank<K, AOS, MAP_BINARY>), dim3(wblocks), dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_range_fill_rank<K, AOS, MAP_KARY>), dim3(wblocks), dim3(256), 0, s, a);
        } else {
            hipLaunchKernelGGL((k_range_fill_eyt<K, AOS>), dim3(blocks), dim3(256), 0, s, a);
        }
        if (hipGetLastError() != hipSuccess) rc = IDX_ERR_HIP;
    } while (0);
    if (!given) h->alloc.put(scratch, s);
    return rc;
}

__global__ void k_zero_u64(uint64_t *p) { *p = 0; }

}  // namespace

int range_lookup_in(idx_index *h, const void *lo, const void *hi, uint64_t m, uint64_t *offsets, uint32_t *out,
                    uint64_t capacity, uint64_t *total, void *scratch, hipStream_t s) {
    if (m == 0) {
        // offsets[0] = 0 (a kernel, not a memset node, so the call stays capturable)
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, offsets);
        IDX_LAUNCH_CHECK();
        if (total) *total = 0;
        return IDX_OK;
    }
    char *sc = (char *)scratch;
    if (h->u64)
        return h->aos ? range_t<uint64_t, true>(h, lo, hi, m, offsets, out, capacity, total, sc, s)
                      : range_t<uint64_t, false>(h, lo, hi, m, offsets, out, capacity, total, sc, s);
    return h->aos ? range_t<uint32_t, true>(h, lo, hi, m, offsets, out, capacity, total, sc, s)
                  : range_t<uint32_t, false>(h, lo, hi, m, offsets, out, capacity, total, sc, s);
}

int range_lookup(idx_index *h, const void *lo, const void *hi, uint64_t m, uint64_t *offsets, uint32_t *out,
                 uint64_t capacity, uint64_t *total, hipStream_t s) {
    return range_lookup_in(h, lo, hi, m, offsets, out, capacity, total, nullptr, s);
}

int exclusive_scan_u64(uint64_t *v, uint64_t m, uint64_t *partial, hipStream_t s) {
    return exclusive_scan(v, m, partial, s);
}

uint64_t scan_partials_for(uint64_t m) { return (m + SC_TILE - 1) / SC_TILE; }

}  // namespace idx
