// Query input and answer output of a point-lookup launch, shared by the
// one-lookup-per-lane kernels (BS, EBS, EKS single, learned); the lane-group
// kernels use only its tile walk.
//
// Two ways a tile of T = blockDim * R lookups meets memory:
//  plain        lookup i reads q[i] and writes out[i];
//  local sort   (Section 7.4) the tile's queries are sorted by key in LDS, so
//               neighbouring lanes search neighbouring keys and share their
//               search paths for longer; the answers are put back in input
//               order in LDS and leave with one coalesced write.
// Lane t's r-th lookup is tile element r * blockDim + t, so in the sorted
// tile adjacent lanes of a wave hold adjacent keys.
//
// Tiles can be walked XCD by XCD: MI355X dispatches workgroup w to XCD w % 8,
// and the remap hands each XCD a contiguous eighth of the tiles, so on a
// batch partitioned by rank bucket (reorder.hip) the lookups one XCD has in
// flight cover a few buckets whose slice of the index fits that XCD's L2.
#pragma once

#include "internal.hpp"

namespace idx {

constexpr uint32_t kXcds = 8;
constexpr uint32_t kMaxSortTile = 8192;  // T = blockDim * R elements sorted in LDS

template <typename K>
__host__ __device__ constexpr K key_max_v() {
    return (K)~(K)0;
}

template <typename K>
struct QueryIO {
    const K *__restrict__ q;
    uint32_t *__restrict__ out;
    uint64_t m;
    uint64_t ntiles;      // tiles of the launch's tile size
    uint64_t iters;       // loop bound over tile slots (>= ntiles when remapped)
    uint32_t local_sort;  // 1: sort each tile in LDS first
    uint32_t xcd;         // 1: XCD-contiguous tile order
    uint32_t sort_off;    // byte offset of the sort buffer in dynamic LDS
    uint32_t rounds;      // short-window scan: 1 = whole window at once, 2 = first line first
    const uint32_t *__restrict__ pos;  // answer of lookup i goes to out[pos[i]] (null: out[i])
    const uint16_t *__restrict__ bkt;  // partitioned batch: bucket of every lookup, or null
    uint64_t bstep;       // its lower bound lies in [bucket_start(b, bstep), that + bspan]
    uint64_t bspan;
};

// Tile of loop slot `it`; >= ntiles for the padding slots of the remap.
__device__ __forceinline__ uint64_t tile_of(uint64_t it, uint64_t ntiles, uint32_t xcd) {
    if (!xcd) return it;
    const uint64_t per = (ntiles + kXcds - 1) / kXcds;
    return (it % kXcds) * per + it / kXcds;
}

template <typename K>
inline void set_tiles(QueryIO<K> &io, uint64_t tile) {
    io.ntiles = (io.m + tile - 1) / tile;
    io.iters = io.xcd ? ((io.ntiles + kXcds - 1) / kXcds) * kXcds : io.ntiles;
}

// Bitonic sort of T = blockDim * R (key, index) pairs in LDS, ascending by key
// then index (a strict order, so the result is unique).  T is a power of two.
template <typename K>
__device__ void bitonic_sort_lds(K *sk, uint16_t *si, uint32_t T) {
    const uint32_t half = T >> 1;
    for (uint32_t size = 2; size <= T; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t p = threadIdx.x; p < half; p += blockDim.x) {
                const uint32_t i = 2 * stride * (p / stride) + (p % stride);
                const uint32_t j = i + stride;
                const bool up = (i & size) == 0;
                const K a = sk[i], b = sk[j];
                const uint16_t ia = si[i], ib = si[j];
                const bool a_gt = (a > b) || (a == b && ia > ib);
                if (a_gt == up) {
                    sk[i] = b;
                    sk[j] = a;
                    si[i] = ib;
                    si[j] = ia;
                }
            }
            __syncthreads();
        }
    }
}

// Loads the R queries of this lane for the tile at t0; src[r] is the
// element's index within the tile (its answer's slot).
template <typename K, int R, bool SORT>
__device__ __forceinline__ void tile_load(const QueryIO<K> &io, char *smem, uint64_t t0, K (&x)[R],
                                          uint32_t (&src)[R]) {
    const uint32_t B = blockDim.x;
    if constexpr (!SORT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            src[r] = (uint32_t)r * B + threadIdx.x;
            const uint64_t qi = t0 + src[r];
            x[r] = qi < io.m ? io.q[qi] : K(0);
        }
        return;
    }
    const uint32_t T = B * R;
    K *sk = (K *)(smem + io.sort_off);
    uint16_t *si = (uint16_t *)(sk + T);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * B + threadIdx.x;
        const uint64_t qi = t0 + i;
        sk[i] = qi < io.m ? io.q[qi] : key_max_v<K>();
        si[i] = (uint16_t)i;
    }
    __syncthreads();
    bitonic_sort_lds(sk, si, T);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = (uint32_t)r * B + threadIdx.x;
        x[r] = sk[e];
        src[r] = si[e];
    }
    __syncthreads();  // the buffer is reused for the answers
}

// Tile element held in the lane's r-th slot: fixed for a plain tile (so the
// src array is never kept live), the sort's permutation otherwise.
template <int R, bool SORT>
__device__ __forceinline__ uint32_t src_of(const uint32_t (&src)[R], int r) {
    if constexpr (SORT) return src[r];
    return (uint32_t)r * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ bool tile_valid(uint64_t m, uint64_t t0, uint32_t src) { return t0 + src < m; }

// Puts the answer of tile element `src` (ignored when its query lies beyond m).
template <typename K, bool SORT>
__device__ __forceinline__ void tile_put(const QueryIO<K> &io, char *smem, uint64_t t0, uint32_t src, uint32_t v) {
    if constexpr (SORT) {
        ((uint32_t *)(smem + io.sort_off))[src] = v;
    } else {
        const uint64_t qi = t0 + src;
        if (qi < io.m) io.out[io.pos ? io.pos[qi] : qi] = v;
    }
}

// After every lane's tile_put: the sorted tile's answers leave in input
// order with one coalesced write.
template <typename K, int R, bool SORT>
__device__ __forceinline__ void tile_flush(const QueryIO<K> &io, char *smem, uint64_t t0) {
    if constexpr (SORT) {
        const uint32_t B = blockDim.x;
        const uint32_t *sres = (const uint32_t *)(smem + io.sort_off);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = (uint32_t)r * B + threadIdx.x;
            const uint64_t qi = t0 + i;
            if (qi < io.m) io.out[qi] = sres[i];
        }
        __syncthreads();  // before the next tile overwrites the buffer
    }
}

// LDS bytes the local sort of T elements needs.
inline size_t sort_lds_bytes(uint32_t T, size_t key_bytes) { return (size_t)T * (key_bytes + 2); }

}  // namespace idx
