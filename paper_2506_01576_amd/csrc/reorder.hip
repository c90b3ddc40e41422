// Point lookups on a batch partitioned by rank bucket.
//
// Section 7.4 observes that neighbouring lookups with close keys share their
// search paths, that globally sorting the batch gives this best, and that a
// block-local sort is the cheap approximation (the local form lives in
// qio.hpp).  On MI355X the global form pays at scale: a lookup into a
// 768 MiB index costs three to four 128-byte lines that miss L2 (random
// requests that miss L2 run at ~55 G/s whether the Infinity Cache or HBM
// serves them), while one XCD's 4 MiB L2 can hold the whole slice of the
// index that a narrow key range touches.  So the batch is partitioned --
// counting passes, not a sort -- into B buckets of equal index rank range
// (about 512 KiB of index each), the lookups walk the partitioned batch XCD
// by XCD so the buckets one XCD has in flight are few and their lines are
// reused from its L2, and the answers are carried back to the caller's order.
//
// Every scatter below keeps the number of partially written 128-byte lines
// in flight per XCD well under its L2 (a few dozen output runs per
// workgroup): an evicted partial line costs HBM a read-modify-write.
//
//  forward
//   1. splitters: B - 1 index keys at ranks step, 2 step, ... (step = n / B),
//      built once per handle and cached;
//   2. count: every query's fine bucket (a table of key cells in LDS, then
//      a search of the few splitters in the query's cell), kept as u16, and
//      per-bucket totals;
//   3. bucket starts (one workgroup);
//   4. scatter to B1 coarse buckets (query, batch position, fine bucket);
//   5. scatter within each coarse bucket to its B2 fine buckets;
//  lookup
//   6. the handle's lookup kernel over the partitioned batch, tiles walked
//      XCD by XCD, answers written in partitioned order;
//  backward
//   7. scatter (position, answer) pairs to D output windows of 2 MiB (counts
//      are known: window d holds positions [d 2^S, (d+1) 2^S));
//   8. write every answer to its position, windows walked XCD by XCD, so the
//      writes of one window merge into whole lines in one L2.
// Within a run, entries land in the order workgroup threads claim them, so
// the partitioned order is not deterministic; answers never depend on it,
// and the bucket function only has to be monotone for locality.
#include <type_traits>

#include "internal.hpp"
#include "access.hpp"
#include "qio.hpp"

namespace idx {
namespace {

constexpr uint32_t kPartThreads = 1024;
constexpr uint64_t kPartTile = 65536;          // entries per partition workgroup
constexpr uint32_t kMaxBuckets = 4096;          // bucket ids fit u16
constexpr uint32_t kCoarse = 64;                // first-pass bucket count (at most)
constexpr uint64_t kBucketBytes = 512 * 1024;   // target index bytes per bucket
constexpr uint32_t kWindowShift = 19;           // at least 2^19 answers (2 MiB) per output window
constexpr uint32_t kMaxWindows = 256;
constexpr uint64_t kChunk = 1ull << 31;         // batch positions fit u32
constexpr int kLoadAhead = 8;                   // entries a thread loads before using them

// Splitters from the sorted array: split[j] = key at rank (j + 1) * step.
template <typename K, bool AOS>
__global__ void k_split_sorted(Load<K, AOS> L, uint64_t step, uint32_t B, K *__restrict__ split) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B) return;
    split[j] = (j + 1 < B) ? L.key((uint64_t)(j + 1) * step) : key_max_v<K>();
}

// Splitters from an Eytzinger layout: every slot whose sorted rank is a
// multiple of step writes itself.  first = 1 for EBS (1-based slots).
template <typename K, bool AOS>
__global__ void k_split_eyt(Load<K, AOS> L, Geo G, uint64_t first, uint64_t step, uint32_t B, K *__restrict__ split) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G.n) return;
    if (t == 0) split[B - 1] = key_max_v<K>();
    const uint64_t r = slot_rank(G, t);
    if (r == 0 || r % step != 0) return;
    const uint64_t j = r / step;
    if (j < B) split[j - 1] = L.key(t + first);
}

// Bucket table: the key range from the first splitter to the second-largest
// one is cut into kCells cells of 2^sh keys (the last cell also takes every
// larger key, the first every smaller one).  Cell h's keys lie between the
// splitters cell_first[h] and cell_first[h + 1], so a lookup searches only
// those: none or one for uniform keys, never more than all B.
constexpr uint32_t kCellBits = 12;
constexpr uint32_t kCells = 1u << kCellBits;

template <typename K>
__device__ __forceinline__ uint32_t cell_of(K x, K base, uint32_t sh) {
    if (x < base) return 0;
    const uint64_t c = (uint64_t)(x - base) >> sh;
    return c < kCells - 1 ? (uint32_t)c : kCells - 1;
}

// Cell width: the smallest 2^sh for which the span from split[0] to
// split[B - 2] fits kCells cells.
template <typename K>
__device__ __forceinline__ uint32_t cell_shift(const K *s_split, uint32_t B) {
    const uint64_t span = B >= 2 ? (uint64_t)(s_split[B - 2] - s_split[0]) : 0;
    const uint32_t bits = span ? 64u - (uint32_t)__clzll((long long)span) : 0u;
    return bits > kCellBits ? bits - kCellBits : 0u;
}

// Fills cell_first[0, kCells]: the number of splitters whose cell is below h.
template <typename K>
__device__ __forceinline__ void build_cells(const K *s_split, uint32_t B, K base, uint32_t sh, uint16_t *cell_first) {
    for (uint32_t h = threadIdx.x; h <= kCells; h += blockDim.x) {
        uint32_t lo = 0, n = B;  // first splitter j with cell_of(split[j]) >= h
        while (n) {
            const uint32_t half = n >> 1;
            if (cell_of(s_split[lo + half], base, sh) < h) {
                lo += half + 1;
                n -= half + 1;
            } else {
                n = half;
            }
        }
        cell_first[h] = (uint16_t)lo;
    }
}

// Bucket of x = the number of splitters below x (splitters ascend, the last
// is the largest key): all those of lower cells plus those of x's own cell
// that are below x.
template <typename K>
__device__ __forceinline__ uint32_t bucket_of_cells(const K *s_split, const uint16_t *cell_first, K base, uint32_t sh,
                                                    K x) {
    const uint32_t h = cell_of(x, base, sh);
    uint32_t b = cell_first[h], n = (uint32_t)cell_first[h + 1] - b;
    while (n) {
        const uint32_t half = n >> 1;
        if (s_split[b + half] < x) {
            b += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return b;
}

__global__ void k_zero_u32(uint32_t *p, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

__device__ __forceinline__ uint64_t tile_end(uint64_t lo, uint64_t m) {
    return lo + kPartTile < m ? lo + kPartTile : m;
}

// 2. Fine bucket of every query and per-bucket totals.
template <typename K>
__global__ __launch_bounds__(kPartThreads) void k_fwd_count(const K *__restrict__ q, uint64_t m,
                                                            const K *__restrict__ split, uint32_t B,
                                                            uint16_t *__restrict__ bkt,
                                                            uint32_t *__restrict__ total) {
    extern __shared__ __align__(16) char smem[];
    K *s_split = (K *)smem;
    uint32_t *s_hist = (uint32_t *)(s_split + B);
    uint16_t *s_cell = (uint16_t *)(s_hist + B);  // kCells + 1 entries
    for (uint32_t i = threadIdx.x; i < B; i += blockDim.x) {
        s_split[i] = split[i];
        s_hist[i] = 0;
    }
    __syncthreads();
    const K base = s_split[0];
    const uint32_t sh = cell_shift(s_split, B);
    build_cells(s_split, B, base, sh, s_cell);
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * kPartTile, hi = tile_end(lo, m);
    // kLoadAhead queries per thread are loaded before any is placed, so
    // their loads are in flight together
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)kLoadAhead * blockDim.x) {
        K v[kLoadAhead];
#pragma unroll
        for (int u = 0; u < kLoadAhead; ++u) {
            const uint64_t i = i0 + (uint64_t)u * blockDim.x;
            v[u] = i < hi ? q[i] : K(0);
        }
#pragma unroll
        for (int u = 0; u < kLoadAhead; ++u) {
            const uint64_t i = i0 + (uint64_t)u * blockDim.x;
            if (i >= hi) continue;
            const uint32_t b = bucket_of_cells(s_split, s_cell, base, sh, v[u]);
            bkt[i] = (uint16_t)b;
            atomicAdd(&s_hist[b], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += blockDim.x)
        if (s_hist[b]) atomicAdd(&total[b], s_hist[b]);
}

// 3. Bucket starts from the totals; coarse and window cursors.  One
// workgroup of kPartThreads threads; B <= kMaxBuckets.
__global__ __launch_bounds__(kPartThreads) void k_starts(const uint32_t *__restrict__ total, uint32_t B, uint32_t B2,
                                                         uint32_t *__restrict__ fcur, uint32_t *__restrict__ ccur,
                                                         uint32_t D, uint32_t shift, uint32_t *__restrict__ dcur) {
    __shared__ uint32_t s_sum[kPartThreads];
    constexpr uint32_t PER = kMaxBuckets / kPartThreads;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        const uint32_t b = threadIdx.x * PER + j;
        v[j] = b < B ? total[b] : 0;
        sum += v[j];
    }
    s_sum[threadIdx.x] = sum;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (uint32_t off = 1; off < kPartThreads; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0;
        __syncthreads();
        s_sum[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s_sum[threadIdx.x] - sum;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        const uint32_t b = threadIdx.x * PER + j;
        if (b < B) {
            fcur[b] = run;
            if (b % B2 == 0) ccur[b / B2] = run;
        }
        run += v[j];
    }
    for (uint32_t d = threadIdx.x; d < D; d += blockDim.x) dcur[d] = d << shift;
}

// Window cursors of the backward scatter (also set by k_starts): window d
// starts at position d << shift.
__global__ void k_window_cursors(uint32_t *__restrict__ dcur, uint32_t D, uint32_t shift) {
    const uint32_t d = threadIdx.x;
    if (d < D) dcur[d] = d << shift;
}

// 4./5./7. One scatter pass: entry i goes to run run_of(i) of NB runs.  Per
// tile a workgroup reserves one contiguous piece of every run the tile feeds
// (one global atomic per run), then fills the pieces front to back in rounds
// of kSub entries sorted by run in LDS, so consecutive lanes write
// consecutive addresses.  The grid is one workgroup per compute
// unit, each walking its own tiles, which bounds the partially written lines
// in flight per XCD to about 32 workgroups x NB runs x 2 per output array.
struct FwdCoarse {};
struct FwdFine {};
struct Bwd {};

template <typename K, typename Pass>
struct ScatterArgs {
    const K *__restrict__ q_in;
    const uint32_t *__restrict__ p_in;   // batch positions (fine pass, backward pass)
    const uint16_t *__restrict__ b_in;   // fine bucket ids
    const uint32_t *__restrict__ r_in;   // answers (backward pass)
    K *__restrict__ q_out;
    uint32_t *__restrict__ p_out;
    uint16_t *__restrict__ b_out;
    uint64_t *__restrict__ pk_out;       // backward: position << 32 | answer
    uint32_t *__restrict__ cur;          // run cursors
    uint64_t m;
    uint64_t ntiles;
    uint32_t B2;                         // fine buckets per coarse bucket
    uint32_t NB;                         // runs this pass feeds
    uint32_t shift;                      // backward: log2 of the output window
};

template <typename K, typename Pass>
__device__ __forceinline__ uint32_t run_of(const ScatterArgs<K, Pass> &a, uint64_t i) {
    if constexpr (std::is_same_v<Pass, FwdCoarse>) return a.b_in[i] / a.B2;
    else if constexpr (std::is_same_v<Pass, FwdFine>) return a.b_in[i];
    else return a.p_in[i] >> a.shift;
}

// Entries of one staged round: each thread loads kSubPer of them, they are
// sorted by run in LDS, and every run's piece leaves with consecutive lanes
// writing consecutive addresses.  A tile whose runs span more than kSpan run
// ids (a fine pass over a small batch) places entries directly instead.
constexpr uint32_t kSubPer = 4;
constexpr uint32_t kSub = kPartThreads * kSubPer;
constexpr uint32_t kSpan = 256;

template <typename K, typename Pass>
struct Staged {
    static constexpr bool bwd = std::is_same_v<Pass, Bwd>;
    // per entry: query key, batch position, fine bucket (forward) or the
    // (position, answer) pair (backward); and its run relative to the tile's
    // smallest run
    static constexpr size_t entry_bytes = (bwd ? 8 : sizeof(K) + 4 + 2) + 2;
};

template <typename K, typename Pass>
size_t scatter_lds_bytes(uint32_t NB) {
    return (((size_t)NB * 4 + 15) & ~(size_t)15) + (size_t)kSub * Staged<K, Pass>::entry_bytes;
}

template <typename K, typename Pass>
__global__ __launch_bounds__(kPartThreads) void k_scatter(ScatterArgs<K, Pass> a) {
    constexpr bool BWD = std::is_same_v<Pass, Bwd>;
    constexpr bool COARSE = std::is_same_v<Pass, FwdCoarse>;
    extern __shared__ __align__(16) char smem[];
    uint32_t *s_cnt = (uint32_t *)smem;  // per run: count, then cursor
    char *st = smem + (((size_t)a.NB * 4 + 15) & ~(size_t)15);
    uint64_t *st_pk = (uint64_t *)st;               // backward
    K *st_q = (K *)st;                              // forward
    uint32_t *st_p = (uint32_t *)(st + (size_t)kSub * sizeof(K));
    uint16_t *st_b = (uint16_t *)((char *)st_p + (size_t)kSub * 4);
    uint16_t *st_r = BWD ? (uint16_t *)(st + (size_t)kSub * 8) : (uint16_t *)((char *)st_b + (size_t)kSub * 2);
    __shared__ uint32_t s_sub[kSpan], s_off[kSpan], s_wsum[kSpan / kWave];
    __shared__ uint32_t s_lo, s_hi;
    for (uint64_t tl = blockIdx.x; tl < a.ntiles; tl += gridDim.x) {
        for (uint32_t b = threadIdx.x; b < a.NB; b += blockDim.x) s_cnt[b] = 0;
        if (threadIdx.x == 0) {
            s_lo = 0xFFFFFFFFu;
            s_hi = 0;
        }
        __syncthreads();
        const uint64_t lo = tl * kPartTile, hi = tile_end(lo, a.m);
        uint32_t rmin = 0xFFFFFFFFu, rmax = 0;
        for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)kLoadAhead * blockDim.x) {
            uint32_t rv[kLoadAhead];
#pragma unroll
            for (int u = 0; u < kLoadAhead; ++u) {
                const uint64_t i = i0 + (uint64_t)u * blockDim.x;
                rv[u] = i < hi ? run_of(a, i) : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int u = 0; u < kLoadAhead; ++u) {
                if (rv[u] == 0xFFFFFFFFu) continue;
                atomicAdd(&s_cnt[rv[u]], 1u);
                rmin = rv[u] < rmin ? rv[u] : rmin;
                rmax = rv[u] > rmax ? rv[u] : rmax;
            }
        }
        if (rmin != 0xFFFFFFFFu) {
            atomicMin(&s_lo, rmin);
            atomicMax(&s_hi, rmax);
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < a.NB; b += blockDim.x) {
            const uint32_t c = s_cnt[b];
            s_cnt[b] = c ? atomicAdd(&a.cur[b], c) : 0u;
        }
        __syncthreads();
        const uint32_t r_lo = s_lo;
        if (s_hi - r_lo >= kSpan) {
            // direct placement: four entries per thread per round, so their loads overlap
            for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * (uint64_t)blockDim.x) {
                uint32_t d[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t i = i0 + (uint64_t)u * blockDim.x;
                    d[u] = i < hi ? atomicAdd(&s_cnt[run_of(a, i)], 1u) : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t i = i0 + (uint64_t)u * blockDim.x;
                    if (i >= hi) continue;
                    if constexpr (COARSE) {
                        a.q_out[d[u]] = a.q_in[i];
                        a.p_out[d[u]] = (uint32_t)i;
                        a.b_out[d[u]] = a.b_in[i];
                    } else if constexpr (!BWD) {
                        a.q_out[d[u]] = a.q_in[i];
                        a.p_out[d[u]] = a.p_in[i];
                        a.b_out[d[u]] = a.b_in[i];
                    } else {
                        a.pk_out[d[u]] = ((uint64_t)a.p_in[i] << 32) | a.r_in[i];
                    }
                }
            }
            __syncthreads();  // before the next tile clears the counters
            continue;
        }
        // staged rounds of kSub entries
        for (uint64_t s0 = lo; s0 < hi; s0 += kSub) {
            const uint32_t ns = hi - s0 < kSub ? (uint32_t)(hi - s0) : kSub;
            if (threadIdx.x < kSpan) s_sub[threadIdx.x] = 0;
            __syncthreads();
            uint32_t rr[kSubPer], rk[kSubPer], pp[kSubPer];
            K qq[kSubPer];
            uint16_t bb[kSubPer];
            uint64_t pk[kSubPer];
#pragma unroll
            for (uint32_t u = 0; u < kSubPer; ++u) {
                const uint32_t j = u * kPartThreads + threadIdx.x;
                rr[u] = kSpan;
                if (j >= ns) continue;
                const uint64_t i = s0 + j;
                rr[u] = run_of(a, i) - r_lo;
                rk[u] = atomicAdd(&s_sub[rr[u]], 1u);
                if constexpr (BWD) {
                    pk[u] = ((uint64_t)a.p_in[i] << 32) | a.r_in[i];
                } else {
                    qq[u] = a.q_in[i];
                    pp[u] = COARSE ? (uint32_t)i : a.p_in[i];
                    bb[u] = a.b_in[i];
                }
            }
            __syncthreads();
            // exclusive scan of the run counts of this round
            if (threadIdx.x < kSpan) {
                const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
                const uint32_t v = s_sub[threadIdx.x];
                uint32_t inc = v;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const uint32_t x = (uint32_t)__shfl_up((int)inc, off, kWave);
                    if (lane >= (uint32_t)off) inc += x;
                }
                if (lane == kWave - 1) s_wsum[w] = inc;
                s_off[threadIdx.x] = inc - v;
            }
            __syncthreads();
            if (threadIdx.x < kSpan) {
                uint32_t add = 0;
                for (uint32_t w = 0; w < threadIdx.x / kWave; ++w) add += s_wsum[w];
                s_off[threadIdx.x] += add;
            }
            __syncthreads();
            // entries into the staging area, sorted by run
#pragma unroll
            for (uint32_t u = 0; u < kSubPer; ++u) {
                if (rr[u] >= kSpan) continue;
                const uint32_t j = s_off[rr[u]] + rk[u];
                st_r[j] = (uint16_t)rr[u];
                if constexpr (BWD) {
                    st_pk[j] = pk[u];
                } else {
                    st_q[j] = qq[u];
                    st_p[j] = pp[u];
                    st_b[j] = bb[u];
                }
            }
            __syncthreads();
            // every run's piece: consecutive staged entries to consecutive addresses
#pragma unroll
            for (uint32_t u = 0; u < kSubPer; ++u) {
                const uint32_t j = u * kPartThreads + threadIdx.x;
                if (j >= ns) continue;
                const uint32_t r = st_r[j];
                const uint32_t d = s_cnt[r_lo + r] + (j - s_off[r]);
                if constexpr (BWD) {
                    a.pk_out[d] = st_pk[j];
                } else {
                    a.q_out[d] = st_q[j];
                    a.p_out[d] = st_p[j];
                    a.b_out[d] = st_b[j];
                }
            }
            __syncthreads();
            if (threadIdx.x < kSpan && r_lo + threadIdx.x < a.NB) s_cnt[r_lo + threadIdx.x] += s_sub[threadIdx.x];
            __syncthreads();
        }
    }
}

// 8. Answers to their positions.  One workgroup per compute unit walking
// its XCD's share of the tiles in order, so the entries one XCD has in
// flight stay within about one output window, whose lines fill in its L2.
constexpr uint32_t kPlaceThreads = 1024;
constexpr uint32_t kPlacePer = 4;

__global__ __launch_bounds__(kPlaceThreads) void k_place(const uint64_t *__restrict__ pk, uint64_t m, uint64_t ntiles,
                                                         uint64_t iters, uint32_t *__restrict__ out) {
    constexpr uint64_t TILE = (uint64_t)kPlaceThreads * kPlacePer;
    for (uint64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, ntiles, 1);
        if (tl >= ntiles) continue;
        const uint64_t t0 = tl * TILE;
        uint64_t v[kPlacePer];
#pragma unroll
        for (uint32_t r = 0; r < kPlacePer; ++r) {
            const uint64_t i = t0 + (uint64_t)r * kPlaceThreads + threadIdx.x;
            v[r] = i < m ? pk[i] : ~0ull;
        }
#pragma unroll
        for (uint32_t r = 0; r < kPlacePer; ++r)
            if (v[r] != ~0ull) out[v[r] >> 32] = (uint32_t)v[r];
    }
}

// Length of the rank interval [bucket_start(b), that + span] holding the
// lower bound of any key of bucket b: splitter b - 1 (rank b * step) is below
// the key and splitter b (rank (b + 1) * step) is not, so the lower bound is
// in [b * step + 1, (b + 1) * step] (from 0 for b = 0, up to n for the last
// bucket); the largest such interval serves every bucket and never reaches
// past n.
uint64_t bucket_span(uint64_t n, uint32_t B) {
    const uint64_t step = n / B;
    const uint64_t last = n - (B - 1) * step - 1;
    return step > last ? step : last;
}

// Bucket count for the handle: a power of two giving about kBucketBytes of
// index per bucket, at most kMaxBuckets and at most n.
uint32_t buckets_for(const idx_index *h) {
    const uint64_t bytes = h->n * ((h->u64 ? 8 : 4) + 4);
    uint32_t B = 2;
    while (B < kMaxBuckets && (uint64_t)B * kBucketBytes < bytes) B <<= 1;
    while (B > 2 && B > h->n) B >>= 1;
    return B;
}

template <typename K, bool AOS>
int build_splitters_t(idx_index *h, uint32_t B, hipStream_t s) {
    const uint64_t step = h->n / B;
    const Load<K, AOS> L = make_load<K, AOS>(h);
    if (h->layout == IDX_BS) {
        hipLaunchKernelGGL((k_split_sorted<K, AOS>), dim3((B + 255) / 256), dim3(256), 0, s, L, step, B, (K *)h->split);
    } else {
        const uint64_t first = h->layout == IDX_EBS ? 1 : 0;
        hipLaunchKernelGGL((k_split_eyt<K, AOS>), dim3((uint32_t)((h->n + 255) / 256)), dim3(256), 0, s, L, h->geo,
                           first, step, B, (K *)h->split);
    }
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

int build_splitters(idx_index *h, uint32_t B, hipStream_t s) {
    if (h->split && h->split_buckets == B) return IDX_OK;
    drop_splitters(h, s);
    h->split = h->alloc.get((size_t)B * (h->u64 ? 8 : 4), s);
    if (!h->split) return IDX_ERR_NOMEM;
    int rc;
    if (h->u64) rc = h->aos ? build_splitters_t<uint64_t, true>(h, B, s) : build_splitters_t<uint64_t, false>(h, B, s);
    else rc = h->aos ? build_splitters_t<uint32_t, true>(h, B, s) : build_splitters_t<uint32_t, false>(h, B, s);
    if (rc != IDX_OK) {
        drop_splitters(h, s);
        return rc;
    }
    h->split_buckets = B;
    return IDX_OK;
}

// Scratch of one chunk of m queries (256-byte aligned regions).
struct PartBufs {
    void *q1;         // coarse-partitioned queries; later the (position, answer) pairs
    uint32_t *p1;     // coarse-partitioned positions; later the answers in partitioned order
    uint16_t *b1;     // coarse-partitioned fine bucket ids
    uint16_t *bkt;    // fine bucket id of every query; after the fine pass, in partitioned order
    void *q2;         // fine-partitioned queries
    uint32_t *p2;     // fine-partitioned positions
    uint32_t *total;  // kMaxBuckets per-bucket totals
    uint32_t *fcur;   // kMaxBuckets
    uint32_t *ccur;   // kCoarse
    uint32_t *dcur;   // kMaxWindows
};

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t part_bytes(uint64_t m, size_t kb) {
    return up256(m * 8 > m * kb ? m * 8 : m * kb) + up256(m * 4) + 2 * up256(m * 2) + up256(m * kb) + up256(m * 4) +
           up256((size_t)(2 * kMaxBuckets + kCoarse + kMaxWindows) * 4);
}

PartBufs carve(char *t, uint64_t m, size_t kb) {
    PartBufs p{};
    p.q1 = t;
    t += up256(m * 8 > m * kb ? m * 8 : m * kb);
    p.p1 = (uint32_t *)t;
    t += up256(m * 4);
    p.b1 = (uint16_t *)t;
    t += up256(m * 2);
    p.bkt = (uint16_t *)t;
    t += up256(m * 2);
    p.q2 = t;
    t += up256(m * kb);
    p.p2 = (uint32_t *)t;
    t += up256(m * 4);
    p.total = (uint32_t *)t;
    p.fcur = p.total + kMaxBuckets;
    p.ccur = p.fcur + kMaxBuckets;
    p.dcur = p.ccur + kCoarse;
    return p;
}

// Forward passes (steps 2-5): fine buckets, their starts, then the coarse
// and fine scatters; the partitioned queries land in P.q2 with their batch
// positions in P.p2.
template <typename K>
int partition_fwd(idx_index *h, const K *q, uint64_t m, uint32_t B, const PartBufs &P, hipStream_t s) {
    const uint32_t B1 = B < kCoarse ? B : kCoarse;
    const uint32_t B2 = B / B1;
    const uint64_t tiles = (m + kPartTile - 1) / kPartTile;
    const uint32_t sgrid = (uint32_t)(tiles < (uint64_t)h->cu_count ? tiles : (uint64_t)h->cu_count);
    uint32_t shift = kWindowShift;
    while (((m - 1) >> shift) + 1 > kMaxWindows) ++shift;
    const uint32_t D = (uint32_t)(((m - 1) >> shift) + 1);
    // totals start at zero (a fill kernel, not a memset node, so the
    // sequence can be captured in a graph)
    hipLaunchKernelGGL(k_zero_u32, dim3(kMaxBuckets / 256), dim3(256), 0, s, P.total, kMaxBuckets);
    IDX_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_fwd_count<K>), dim3((uint32_t)tiles), dim3(kPartThreads),
                       (size_t)B * (sizeof(K) + 4) + (kCells + 1) * 2, s, q,
                       m, (const K *)h->split, B, P.bkt, P.total);
    IDX_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_starts, dim3(1), dim3(kPartThreads), 0, s, P.total, B, B2, P.fcur, P.ccur, D, shift, P.dcur);
    IDX_LAUNCH_CHECK();
    {
        ScatterArgs<K, FwdCoarse> a{};
        a.q_in = q;
        a.b_in = P.bkt;
        a.q_out = (K *)P.q1;
        a.p_out = P.p1;
        a.b_out = P.b1;
        a.cur = P.ccur;
        a.m = m;
        a.ntiles = tiles;
        a.B2 = B2;
        a.NB = B1;
        const size_t lds = scatter_lds_bytes<K, FwdCoarse>(B1);
        hipLaunchKernelGGL((k_scatter<K, FwdCoarse>), dim3(sgrid), dim3(kPartThreads), lds, s, a);
        IDX_LAUNCH_CHECK();
    }
    {
        ScatterArgs<K, FwdFine> a{};
        a.q_in = (const K *)P.q1;
        a.p_in = P.p1;
        a.b_in = P.b1;
        a.q_out = (K *)P.q2;
        a.p_out = P.p2;
        a.b_out = P.bkt;  // caller-order bucket ids are no longer needed
        a.cur = P.fcur;
        a.m = m;
        a.ntiles = tiles;
        a.B2 = B2;
        a.NB = B;
        const size_t lds = scatter_lds_bytes<K, FwdFine>(B);
        hipLaunchKernelGGL((k_scatter<K, FwdFine>), dim3(sgrid), dim3(kPartThreads), lds, s, a);
        IDX_LAUNCH_CHECK();
    }
    return IDX_OK;
}

// Backward passes (steps 7-8): answers `ans` in partitioned order (positions
// P.p2) to out[position].  Uses P.q1 for the (position, answer) pairs and
// the window cursors P.dcur, which k_starts set; a second placement over the
// same partition resets them first.
int place_back(idx_index *h, const PartBufs &P, uint64_t m, const uint32_t *ans, uint32_t *out, hipStream_t s) {
    const uint64_t tiles = (m + kPartTile - 1) / kPartTile;
    const uint32_t sgrid = (uint32_t)(tiles < (uint64_t)h->cu_count ? tiles : (uint64_t)h->cu_count);
    uint32_t shift = kWindowShift;
    while (((m - 1) >> shift) + 1 > kMaxWindows) ++shift;
    const uint32_t D = (uint32_t)(((m - 1) >> shift) + 1);
    hipLaunchKernelGGL(k_window_cursors, dim3(1), dim3(kMaxWindows), 0, s, P.dcur, D, shift);
    IDX_LAUNCH_CHECK();
    {
        ScatterArgs<uint32_t, Bwd> a{};
        a.p_in = P.p2;
        a.r_in = ans;
        a.pk_out = (uint64_t *)P.q1;
        a.cur = P.dcur;
        a.m = m;
        a.ntiles = tiles;
        a.NB = D;
        a.shift = shift;
        const size_t lds = scatter_lds_bytes<uint32_t, Bwd>(D);
        hipLaunchKernelGGL((k_scatter<uint32_t, Bwd>), dim3(sgrid), dim3(kPartThreads), lds, s, a);
        IDX_LAUNCH_CHECK();
    }
    const uint64_t ptile = (uint64_t)kPlaceThreads * kPlacePer;
    const uint64_t ptiles = (m + ptile - 1) / ptile;
    const uint64_t piters = ((ptiles + kXcds - 1) / kXcds) * kXcds;
    uint64_t pgrid = (uint64_t)h->cu_count - (uint64_t)h->cu_count % kXcds;
    if (pgrid == 0) pgrid = kXcds;
    if (pgrid > piters) pgrid = piters;
    hipLaunchKernelGGL(k_place, dim3((uint32_t)pgrid), dim3(kPlaceThreads), 0, s, (const uint64_t *)P.q1, m, ptiles,
                       piters, out);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K>
int partition_chunk(idx_index *h, const K *q, uint64_t m, uint32_t *out, uint32_t B, const PartBufs &P,
                    hipStream_t s) {
    int rc = partition_fwd<K>(h, q, m, B, P, s);
    if (rc != IDX_OK) return rc;
    // answers in partitioned order go to p1 (free after the fine pass), or
    // (reorder = 3) straight to their positions in out; the sorted array's
    // search starts inside each lookup's bucket
    const bool direct = h->params.reorder == 3;
    PointIO io{P.q2, m, direct ? out : P.p1, false, true};
    if (direct) io.pos = P.p2;
    if (h->layout == IDX_BS && !(h->learned && h->params.model != 2)) {
        io.bkt = P.bkt;
        io.bstep = h->n / B;
        io.bspan = bucket_span(h->n, B);
    }
    rc = point_run(h, io, s);
    if (rc != IDX_OK || direct) return rc;
    return place_back(h, P, m, P.p1, out, s);
}

}  // namespace

// ---- the partition as a service for other lookups (range counts): the
// forward passes and the answer placement of one chunk, on scratch the
// caller provides.
size_t partition_scratch_bytes(const idx_index *h, uint64_t m) { return part_bytes(m, h->u64 ? 8 : 4); }

int partition_forward(idx_index *h, const void *q, uint64_t m, void *scratch, PartView *out, hipStream_t s) {
    if (m == 0 || m > kChunk) return IDX_ERR_ARG;
    const uint32_t B = buckets_for(h);
    int rc = build_splitters(h, B, s);
    if (rc != IDX_OK) return rc;
    const size_t kb = h->u64 ? 8 : 4;
    const PartBufs P = carve((char *)scratch, m, kb);
    rc = h->u64 ? partition_fwd<uint64_t>(h, (const uint64_t *)q, m, B, P, s)
                : partition_fwd<uint32_t>(h, (const uint32_t *)q, m, B, P, s);
    if (rc != IDX_OK) return rc;
    out->q = P.q2;
    out->pos = P.p2;
    out->m = m;
    out->scratch = scratch;
    out->bkt = P.bkt;
    out->bstep = h->n / B;
    out->bspan = bucket_span(h->n, B);
    return IDX_OK;
}

void drop_splitters(idx_index *h, hipStream_t s) {
    if (h->split) h->alloc.put(h->split, s);
    h->split = nullptr;
    h->split_buckets = 0;
}

int point_partitioned(idx_index *h, const void *q, uint64_t m, uint32_t *out, hipStream_t s) {
    if (h->n < 4) {
        PointIO io{q, m, out, false, false};
        return point_run(h, io, s);
    }
    const uint32_t B = buckets_for(h);
    int rc = build_splitters(h, B, s);
    if (rc != IDX_OK) return rc;
    const size_t kb = h->u64 ? 8 : 4;
    const uint64_t chunk = m < kChunk ? m : kChunk;
    char *tmp = (char *)h->alloc.get(part_bytes(chunk, kb), s);
    if (!tmp) return IDX_ERR_NOMEM;
    const PartBufs P = carve(tmp, chunk, kb);
    for (uint64_t c0 = 0; c0 < m && rc == IDX_OK; c0 += chunk) {
        const uint64_t mc = (m - c0) < chunk ? (m - c0) : chunk;
        // positions of this chunk are relative to its own start
        if (h->u64)
            rc = partition_chunk<uint64_t>(h, (const uint64_t *)q + c0, mc, out + c0, B, P, s);
        else
            rc = partition_chunk<uint32_t>(h, (const uint32_t *)q + c0, mc, out + c0, B, P, s);
    }
    h->alloc.put(tmp, s);
    return rc;
}

}  // namespace idx
