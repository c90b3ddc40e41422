// Layout construction: the parallel Eytzinger permutation (Sections 4 and
// 6.1), AoS interleaving (Section 7.1), the post-sort checks, layout export
// and the LDS pin tables used by cache pinning (Section 7.3).
#include "internal.hpp"
#include "access.hpp"

namespace idx {

Geo make_geo(uint64_t n, uint32_t k) {
    Geo G{};
    G.n = n;
    G.k = k < 2 ? 2 : k;
    G.g = G.k - 1;
    G.gshift = -1;
    for (int s = 0; s < 32; ++s)
        if ((1u << s) == G.g) G.gshift = s;
    // start[l] = k^l - 1, saturated far above any n
    const uint64_t cap = 1ull << 62;
    uint64_t p = 1;
    for (int l = 0; l < kMaxLevels; ++l) {
        G.start[l] = p - 1;
        if (p > cap / G.k) p = cap;
        else p *= G.k;
    }
    uint32_t m = 0;
    while (m + 1 < (uint32_t)kMaxLevels && G.start[m + 1] <= n) ++m;
    G.m = m;
    G.b = n - G.start[m];
    G.levels = m + (G.b > 0 ? 1u : 0u);
    return G;
}

namespace {

// The sorted-array layout: entry t to slot t (a copy, or the interleaving
// of keys and row IDs for the array of structures).
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_copy_sorted(const K *__restrict__ sk, const uint32_t *__restrict__ sr,
                                                     uint64_t n, Store<K, AOS> dst) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    dst.put(t, sk[t], sr[t]);
}

// The Eytzinger layouts, built in rank order: thread r loads sorted entry r
// (the read is consecutive per wave, each line of the sorted arrays fetched
// once) and stores it at its level-order slot, + off (off = 1 for the binary
// layout's empty slot 0).  A wave's 64 ranks land on runs of consecutive
// slots, one per level (32, 16, 8, ... slots for k = 2); the workgroups of
// one XCD take a contiguous share of the ranks, so the short runs of the
// upper levels from neighbouring waves complete their lines in one L2.  A
// gather in slot order would fetch every line of the sorted arrays once per
// level wherever a level's stride is below a line.
constexpr uint32_t kPermXcds = 8;  // workgroups are dealt round-robin over the 8 XCDs

template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_permute_rank2(const K *__restrict__ sk, const uint32_t *__restrict__ sr,
                                                       Geo G, uint32_t off, Store<K, AOS> dst) {
    const uint32_t per = gridDim.x / kPermXcds, rem = gridDim.x % kPermXcds;
    const uint32_t x = blockIdx.x % kPermXcds, i = blockIdx.x / kPermXcds;
    const uint32_t blk = x * per + (x < rem ? x : rem) + i;  // a bijection of [0, gridDim.x)
    const uint64_t r = (uint64_t)blk * blockDim.x + threadIdx.x;
    if (r >= G.n) return;
    dst.put(rank_slot_binary(G, r) + off, sk[r], sr[r]);
}

// The same for any k (the k-ary layout, no empty slot): slot
// rank_slot_general(r).  k - 1 of every k ranks go to consecutive slots of
// the lowest level while it lasts.
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_permute_rank(const K *__restrict__ sk, const uint32_t *__restrict__ sr, Geo G,
                                                      uint64_t kinv, Store<K, AOS> dst) {
    const uint32_t per = gridDim.x / kPermXcds, rem = gridDim.x % kPermXcds;
    const uint32_t x = blockIdx.x % kPermXcds, i = blockIdx.x / kPermXcds;
    const uint32_t blk = x * per + (x < rem ? x : rem) + i;  // a bijection of [0, gridDim.x)
    const uint64_t r = (uint64_t)blk * blockDim.x + threadIdx.x;
    if (r >= G.n) return;
    dst.put(rank_slot_general(G, r, kinv), sk[r], sr[r]);
}

template <typename K, bool AOS>
__global__ void k_empty_slot0(Store<K, AOS> dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst.put(0, K(0), kMiss);
}

template <typename K>
__global__ __launch_bounds__(256) void k_check(const K *__restrict__ sk, const uint32_t *__restrict__ sr, uint64_t n,
                                               uint32_t *flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool dup = false, res = false;
    if (i < n) {
        dup = i > 0 && sk[i] == sk[i - 1];
        res = sr[i] == kMiss;
    }
    const uint64_t bd = __ballot(dup), br = __ballot(res);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bd) atomicOr(&flags[0], 1u);
        if (br) atomicOr(&flags[1], 1u);
    }
}

template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_export(Load<K, AOS> src, uint64_t slots, K *__restrict__ ko,
                                                uint32_t *__restrict__ ro) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= slots) return;
    if (ko) ko[s] = src.key(s);
    if (ro) ro[s] = src.row(s);
}

// Pin table of the binary search on the sorted array: entry v (heap
// numbering, v in [1, 2^L)) is the key the branchless lower-bound search
// probes at the tree node v, found by replaying the path encoded by v's bits.
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_pin_bs(Load<K, AOS> src, uint64_t n, uint32_t count, K *__restrict__ pin) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= count) return;
    if (v == 0) {
        pin[0] = K(0);
        return;
    }
    const int depth = 31 - __clz((int)v);
    uint64_t base = 0, len = n;
    for (int d = depth - 1; d >= 0; --d) {
        const uint64_t half = len >> 1;
        if ((v >> d) & 1u) base += half;
        len -= half;
    }
    pin[v] = src.key(base + (len >> 1));
}

// Pin table of an Eytzinger layout: its first `count` slots.
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_pin_prefix(Load<K, AOS> src, uint64_t slots, uint32_t count,
                                                    K *__restrict__ pin) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= count) return;
    pin[v] = v < slots ? src.key(v) : ~K(0);
}

template <typename K, bool AOS>
int build_layout_t(idx_index *h, const K *sk, const uint32_t *sr, hipStream_t s) {
    Store<K, AOS> dst = make_store<K, AOS>(h);
    const uint64_t n = h->n;
    const uint32_t off = h->layout == IDX_EBS ? 1u : 0u;
    if (h->layout == IDX_EBS) {
        hipLaunchKernelGGL((k_empty_slot0<K, AOS>), dim3(1), dim3(64), 0, s, dst);
        IDX_LAUNCH_CHECK();
    }
    if (n == 0) return IDX_OK;
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    if (h->layout == IDX_BS) {
        hipLaunchKernelGGL((k_copy_sorted<K, AOS>), dim3(blocks), dim3(256), 0, s, sk, sr, n, dst);
    } else if (h->geo.k == 2) {  // EBS (k = 2 always, off = 1) or EKS with k = 2
        hipLaunchKernelGGL((k_permute_rank2<K, AOS>), dim3(blocks), dim3(256), 0, s, sk, sr, h->geo, off, dst);
    } else {  // EKS, k in [3, IDX_MAX_FANOUT], off = 0
        // ceil(2^64 / k) for the exact divisions of the inverse slot map
        const uint64_t k = h->geo.k;
        const uint64_t kinv = ~0ull / k + 1;
        hipLaunchKernelGGL((k_permute_rank<K, AOS>), dim3(blocks), dim3(256), 0, s, sk, sr, h->geo, kinv, dst);
    }
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

}  // namespace

int build_layout(idx_index *h, const void *sorted_keys, const uint32_t *sorted_rows, hipStream_t s) {
    if (h->u64)
        return h->aos ? build_layout_t<uint64_t, true>(h, (const uint64_t *)sorted_keys, sorted_rows, s)
                      : build_layout_t<uint64_t, false>(h, (const uint64_t *)sorted_keys, sorted_rows, s);
    return h->aos ? build_layout_t<uint32_t, true>(h, (const uint32_t *)sorted_keys, sorted_rows, s)
                  : build_layout_t<uint32_t, false>(h, (const uint32_t *)sorted_keys, sorted_rows, s);
}

int check_sorted(const void *sorted_keys, const uint32_t *sorted_rows, uint64_t n, bool u64, uint32_t *flags,
                 hipStream_t s) {
    if (n == 0) return IDX_OK;
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    if (u64)
        hipLaunchKernelGGL(k_check<uint64_t>, dim3(blocks), dim3(256), 0, s, (const uint64_t *)sorted_keys,
                           sorted_rows, n, flags);
    else
        hipLaunchKernelGGL(k_check<uint32_t>, dim3(blocks), dim3(256), 0, s, (const uint32_t *)sorted_keys,
                           sorted_rows, n, flags);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

namespace {
template <typename K, bool AOS>
int export_t(const idx_index *h, void *ko, uint32_t *ro, hipStream_t s) {
    if (h->slots == 0) return IDX_OK;
    const uint32_t blocks = (uint32_t)((h->slots + 255) / 256);
    hipLaunchKernelGGL((k_export<K, AOS>), dim3(blocks), dim3(256), 0, s, make_load<K, AOS>(h), h->slots, (K *)ko,
                       ro);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS>
int pin_t(idx_index *h, uint32_t count, hipStream_t s) {
    const uint32_t blocks = (count + 255) / 256;
    if (h->layout == IDX_BS)
        hipLaunchKernelGGL((k_pin_bs<K, AOS>), dim3(blocks), dim3(256), 0, s, make_load<K, AOS>(h), h->n, count,
                           (K *)h->pin);
    else
        hipLaunchKernelGGL((k_pin_prefix<K, AOS>), dim3(blocks), dim3(256), 0, s, make_load<K, AOS>(h), h->slots,
                           count, (K *)h->pin);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}
}  // namespace

int export_layout(const idx_index *h, void *ko, uint32_t *ro, hipStream_t s) {
    if (h->u64) return h->aos ? export_t<uint64_t, true>(h, ko, ro, s) : export_t<uint64_t, false>(h, ko, ro, s);
    return h->aos ? export_t<uint32_t, true>(h, ko, ro, s) : export_t<uint32_t, false>(h, ko, ro, s);
}

// Number of pin-table entries for `levels` top levels.  BS and EBS use heap
// numbering with an unused entry 0 (2^L entries); EKS uses slots
// [0, k^L - 1).
uint32_t pin_entries_for(const idx_index *h, uint32_t levels) {
    if (levels == 0) return 0;
    if (h->layout == IDX_EKS) return (uint32_t)h->geo.start[levels];
    return 1u << levels;
}

uint32_t pin_levels_for(const idx_index *h, size_t bytes) {
    const size_t kb = h->u64 ? 8 : 4;
    uint32_t best = 0;
    uint32_t maxl = h->geo.m;
    if (h->layout == IDX_BS) {
        // binary-search steps over n keys: the pinned levels must all be steps
        uint64_t len = h->n;
        maxl = 0;
        while (len > 1) {
            len -= len >> 1;
            ++maxl;
        }
    }
    for (uint32_t l = 1; l <= maxl && l < 24; ++l)
        if ((size_t)pin_entries_for(h, l) * kb <= bytes) best = l;
    return best;
}

int build_pin(idx_index *h, uint32_t levels, hipStream_t s) {
    if (levels == h->pin_levels_built && (levels == 0 || h->pin)) return IDX_OK;
    if (h->pin) {
        h->alloc.put(h->pin, s);
        h->pin = nullptr;
        h->pin_keys = 0;
        h->pin_levels_built = 0;
    }
    if (levels == 0) return IDX_OK;
    const uint32_t count = pin_entries_for(h, levels);
    h->pin = h->alloc.get((size_t)count * (h->u64 ? 8 : 4), s);
    if (!h->pin) return IDX_ERR_NOMEM;
    int rc;
    if (h->u64) rc = h->aos ? pin_t<uint64_t, true>(h, count, s) : pin_t<uint64_t, false>(h, count, s);
    else rc = h->aos ? pin_t<uint32_t, true>(h, count, s) : pin_t<uint32_t, false>(h, count, s);
    if (rc != IDX_OK) return rc;
    h->pin_keys = count;
    h->pin_levels_built = levels;
    return IDX_OK;
}

}  // namespace idx
