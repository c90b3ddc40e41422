// Internal declarations of libidx: the handle, the tree geometry and the
// host-side launchers each kernel file provides.  gfx950 (MI355X) only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/idx.h"

namespace idx {

constexpr uint32_t kMiss = IDX_MISS;
constexpr int kWave = 64;
constexpr int kMaxLevels = 40;

// Shape of the complete k-ary search tree over n keys stored in level order
// (Sections 4 and 6.1).  Level l holds (k-1)*k^l slots starting at slot
// k^l - 1; the first m levels are full (k^m - 1 <= n), the b = n - (k^m - 1)
// remaining keys sit left-aligned on level m.
struct Geo {
    uint64_t n;
    uint32_t k;      // fan-out
    uint32_t g;      // k - 1 keys per node
    uint32_t m;      // full levels
    uint32_t levels; // m + (b > 0)
    int32_t gshift;  // log2(g) when g is a power of two, else -1
    uint32_t pad;
    uint64_t b;                  // keys on the partial level
    uint64_t start[kMaxLevels];  // start[l] = k^l - 1 (saturated), l <= levels
};

Geo make_geo(uint64_t n, uint32_t k);

// Default-stream-ordered device memory through the handle's allocator.
struct Alloc {
    idx_allocator a{};
    bool custom = false;
    void *get(size_t bytes, hipStream_t s) const;
    void put(void *p, hipStream_t s) const;
};

struct LearnedModel;  // learned rank model (learned.hip)

}  // namespace idx

struct idx_index {
    uint64_t n = 0;
    uint64_t slots = 0;
    int layout = IDX_BS;
    uint32_t k = 1;
    uint32_t flags = 0;
    bool u64 = false;
    bool aos = false;
    bool unique = true;
    uint32_t node = 1;  // keys per AoS block (k - 1 for EKS, 1 otherwise)
    uint32_t stride = 0;  // bytes per AoS block
    void *keys = nullptr;       // SoA keys or AoS blocks
    uint32_t *rowids = nullptr; // SoA rowids (nullptr for AoS)
    size_t key_bytes = 0, row_bytes = 0;
    void *pin = nullptr;        // top of the search tree, ready to copy to LDS
    uint32_t pin_keys = 0;      // keys in `pin`
    uint32_t pin_levels_built = 0;
    idx::Geo geo{};
    idx::Alloc alloc;
    idx_lookup_params params{};
    float ms_sort = 0.f, ms_permute = 0.f;
    hipStream_t last_stream = nullptr;
    int cu_count = 256;
    size_t lds_max = 64 * 1024;  // LDS bytes one workgroup may use on this device
    idx::LearnedModel *learned = nullptr;  // attached rank model (BS layout only)
    void *split = nullptr;       // rank-bucket splitter keys for partitioned lookups
    uint32_t split_buckets = 0;  // buckets those splitters define (0 = none built)
    // Leaf-line buffer of the model a re-training replaced, kept for the new
    // model's lines when the leaf count is the same (a fresh buffer of that
    // size costs a mapping of device memory on every re-training).
    void *spare_lines = nullptr;
    size_t spare_lines_bytes = 0;
    // Batches (idx_batch_create) holding this handle: their descriptors point
    // at its layout and model buffers, so while any holds it the handle may
    // not be destroyed, retrained or have its model dropped.
    uint32_t batch_refs = 0;
};

namespace idx {

// ---- sort.hip ---------------------------------------------------------------
// Bytes of temporary device memory sort_pairs needs for n keys.
size_t sort_temp_bytes(uint64_t n, bool u64);
// Stable LSD radix sort of (key, rowid) by key.  in_* are read only; the
// result is written to out_*; temp holds sort_temp_bytes(n, u64) bytes.
// Synchronises `s` once (to decide which digit passes can be skipped).
int sort_pairs(const void *keys_in, const uint32_t *rows_in, uint64_t n, bool u64, void *keys_out,
               uint32_t *rows_out, void *temp, hipStream_t s);

// ---- layout.hip -------------------------------------------------------------
// Fills the layout buffers of h from the sorted arrays (permutation for
// EBS/EKS, copy or interleave for BS).
int build_layout(idx_index *h, const void *sorted_keys, const uint32_t *sorted_rows, hipStream_t s);
// flags[0] |= 1 when two adjacent sorted keys are equal, flags[1] |= 1 when a
// rowid equals IDX_MISS.
int check_sorted(const void *sorted_keys, const uint32_t *sorted_rows, uint64_t n, bool u64, uint32_t *flags,
                 hipStream_t s);
// Copies the layout into SoA caller buffers.
int export_layout(const idx_index *h, void *keys_out, uint32_t *rows_out, hipStream_t s);
// (Re)builds the LDS pin table of the top `levels` tree levels.
int build_pin(idx_index *h, uint32_t levels, hipStream_t s);
// Sorted rank of level-order slot t (0-based) -- Sections 4 and 6.1.
__host__ __device__ inline uint64_t slot_rank(const Geo &G, uint64_t t);

// ---- point.hip --------------------------------------------------------------
// Where one point-lookup launch reads its queries and writes its answers.
struct PointIO {
    const void *q;
    uint64_t m;
    uint32_t *out;
    bool local_sort;       // sort each tile of lookups in LDS first (Section 7.4)
    bool xcd;              // walk tiles XCD by XCD
    // a batch partitioned by rank bucket: the bucket of every lookup, and the
    // rank interval [start(b), start(b) + span] that holds the lower bound of
    // a key of bucket b, start(b) = b * step + (b > 0) (sorted array only)
    const uint16_t *bkt = nullptr;
    uint64_t bstep = 0;
    uint64_t bspan = 0;
    // answer of lookup i goes to out[pos[i]] (nullptr: out[i])
    const uint32_t *pos = nullptr;
};
int point_lookup(idx_index *h, const void *q, uint64_t m, uint32_t *out, hipStream_t s);
// One launch of the handle's point-lookup form over `io`.
int point_run(idx_index *h, const PointIO &io, hipStream_t s);
// Resolve defaults and validate a parameter set for h.
int resolve_params(const idx_index *h, const idx_lookup_params *in, idx_lookup_params *out);
// Largest number of top levels whose keys fit in `bytes` of LDS.
uint32_t pin_levels_for(const idx_index *h, size_t bytes);
// Pin-table entries (keys) for `levels` top levels.
uint32_t pin_entries_for(const idx_index *h, uint32_t levels);

// ---- reorder.hip ------------------------------------------------------------
// Point lookups on a batch partitioned by rank bucket first.
int point_partitioned(idx_index *h, const void *q, uint64_t m, uint32_t *out, hipStream_t s);
void drop_splitters(idx_index *h, hipStream_t s);
// The partition for other lookups: one chunk of m <= 2^31 query keys
// partitioned by rank bucket (keys q and batch positions pos, both in
// partitioned order); the caller writes each answer at its position.
struct PartView {
    const void *q;
    const uint32_t *pos;
    uint64_t m;
    void *scratch;
    const uint16_t *bkt;  // bucket of every entry (partitioned order)
    uint64_t bstep;       // ranks per bucket; lower bounds of bucket b lie in
    uint64_t bspan;       // [b * bstep + (b > 0), that + bspan]
};
// Rank interval that holds the lower bound of a key of bucket b.
__host__ __device__ inline uint64_t bucket_start(uint64_t b, uint64_t step) { return b ? b * step + 1 : 0; }
constexpr uint64_t kPartChunk = 1ull << 31;
size_t partition_scratch_bytes(const idx_index *h, uint64_t m);
int partition_forward(idx_index *h, const void *q, uint64_t m, void *scratch, PartView *out, hipStream_t s);

// ---- range.hip --------------------------------------------------------------
// Exclusive scan of v[0..m) in place, v[m] = total; partial holds
// ceil(m / 4096) entries.
int exclusive_scan_u64(uint64_t *v, uint64_t m, uint64_t *partial, hipStream_t s);
uint64_t scan_partials_for(uint64_t m);
int range_lookup(idx_index *h, const void *lo, const void *hi, uint64_t m, uint64_t *offsets, uint32_t *out,
                 uint64_t capacity, uint64_t *total, hipStream_t s);
// The same with the call's scratch (range_scratch_bytes(m) bytes, 256-byte
// aligned) given by the caller; nullptr = from the handle's allocator.
int range_lookup_in(idx_index *h, const void *lo, const void *hi, uint64_t m, uint64_t *offsets, uint32_t *out,
                    uint64_t capacity, uint64_t *total, void *scratch, hipStream_t s);
// Queries per tile of the u64 exclusive scan (one partial sum per tile).
constexpr uint64_t kScanTile = 4096;
// Scratch of one range call over m ranges: the first matching rank of every
// range (u32, rounded up to 256 bytes), then one u64 partial per scan tile.
constexpr size_t range_scratch_bytes(uint64_t m) {
    return (size_t)(((m * 4 + 255) / 256) * 256 + ((m + kScanTile - 1) / kScanTile) * 8 + 256);
}

// ---- learned.hip ------------------------------------------------------------
int learn(idx_index *h, uint32_t leaves, uint32_t epochs, uint32_t feature, hipStream_t s);
// learn_batch.hip: models of many indexes trained by one launch sequence.
int learn_batch(idx_index *const *hs, uint32_t count, const uint32_t *leaves, uint32_t epochs, uint32_t feature,
                hipStream_t s);
// Frees the attached model (and any spare leaf-line buffer).  keep_lines: the
// model's leaf lines become the handle's spare buffer instead.
void drop_model(idx_index *h, hipStream_t s, bool keep_lines = false);
int learn_stats(const idx_index *h, idx_learn_stats *out);
int learn_export(const idx_index *h, void *leaves_out, hipStream_t s);
int learn_eval(idx_index *h, uint32_t feature, const float *root_ab, uint32_t leaves, const float *leaf_ab,
               double *root_acc, double *leaf_acc, hipStream_t s);
int point_learned(idx_index *h, const PointIO &io, hipStream_t s);
// The attached model's leaf lines, written unless they are there.
int ensure_lines(idx_index *h, hipStream_t s);
// first-match ranks and counts of ranges through the model
// may_alloc: the leaf lines may be written here (else they are used only if
// they exist).
int range_count_learned(idx_index *h, const void *lo, const void *hi, uint64_t m, uint32_t *first, uint64_t *count,
                        bool may_alloc, hipStream_t s);

// ---- abi.hip: handle life cycle ----------------------------------------------
// A handle with its layout buffers allocated (validates layout, k, flags).
int handle_new(uint64_t n, int layout, uint32_t k, uint32_t flags, const idx_allocator *alloc, hipStream_t s,
               idx_index **out);
// Resolves the default lookup parameters and hands the handle out.
int handle_finish(idx_index *h, hipStream_t s, idx_handle *out);
// Frees a handle that is not handed out (waits for its stream first).
void handle_discard(idx_index *h, hipStream_t s);

// ---- error plumbing ----------------------------------------------------------
int hip_fail(hipError_t e);

}  // namespace idx

#define IDX_HIP(call)                                 \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return idx::hip_fail(e_); \
    } while (0)

#define IDX_LAUNCH_CHECK() IDX_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Inline device helpers shared by the kernel files.
// ---------------------------------------------------------------------------
namespace idx {

// Sorted rank of level-order slot t (0-based), t < n.  Bottom (partial) level
// entries: rank i + floor(i/(k-1)) with i the position within the level;
// upper-level entries: the rank p in the perfect tree of m levels,
// p = k^(m-l-1) * (1 + i + floor(i/(k-1))) - 1, shifted right by the number
// of bottom-level keys that precede it, min(b, (k-1)(p+1)).  This is the
// reading of Sections 4 and 6.1 with the two cases assigned to the bottom and
// upper levels respectively and m = floor(log_k(n+1)), l(t) = floor(log_k(t+1)).
__host__ __device__ inline uint64_t div_g(const Geo &G, uint64_t v) {
    return G.gshift >= 0 ? (v >> G.gshift) : v / G.g;
}

__host__ __device__ inline uint64_t slot_rank(const Geo &G, uint64_t t) {
    const uint64_t bottom_start = G.start[G.m];
    if (t >= bottom_start) {
        const uint64_t i = t - bottom_start;
        return i + div_g(G, i);
    }
    uint32_t l = 0;
    if (G.k == 2) {
        l = 63u - (uint32_t)__builtin_clzll(t + 1);
    } else {
        while (G.start[l + 1] <= t) ++l;
    }
    const uint64_t i = t - G.start[l];
    // k^(m-l-1) = start[m-l-1] + 1
    const uint64_t p = (G.start[G.m - l - 1] + 1) * (1 + i + div_g(G, i)) - 1;
    const uint64_t skip = G.g * (p + 1);
    return p + (skip < G.b ? skip : G.b);
}

// Level-order slot of sorted rank r < n, the inverse of slot_rank, for the
// binary layout (k = 2).  The first 2b ranks alternate: even ranks are the b
// bottom-level entries (slot start[m] + r/2), odd ranks upper-level keys of
// perfect-tree rank p = (r - 1)/2; later ranks are upper-level keys with
// p = r - b.  In the perfect tree of m levels, p + 1 = 2^e * u with u odd
// puts the key on level m - 1 - e at position (u - 1)/2.
__host__ __device__ inline uint64_t rank_slot_binary(const Geo &G, uint64_t r) {
    uint64_t p;
    if (r < 2 * G.b) {
        if ((r & 1) == 0) return G.start[G.m] + (r >> 1);
        p = r >> 1;
    } else {
        p = r - G.b;
    }
    const uint64_t v = p + 1;
    const uint32_t e = (uint32_t)__builtin_ctzll(v);
    const uint32_t l = G.m - 1 - e;
    return G.start[l] + ((v >> e) >> 1);
}

// floor(x / k) for x < 2^32 and 2 <= k < 2^32, given kinv = ceil(2^64 / k):
// the high half of x * kinv (exact, since x * (kinv * k - 2^64) < 2^64).
__host__ __device__ inline uint64_t div_small(uint64_t x, uint64_t kinv) {
    return (uint64_t)(((unsigned __int128)x * kinv) >> 64);
}

// The inverse of slot_rank for any k (n < 2^32).  Ranks come in groups of k
// while bottom-level keys last: k - 1 bottom entries, then one upper-level
// key.  An upper-level key has perfect-tree rank p (p = r / k in a group,
// p = r - b after the groups); p + 1 = k^e * u with u not a multiple of k
// puts it on level m - 1 - e at position (u - 1) - (u - 1) / k.
__host__ __device__ inline uint64_t rank_slot_general(const Geo &G, uint64_t r, uint64_t kinv) {
    const uint64_t q = div_small(r, kinv);
    const uint64_t j = r - q * G.k;
    if (j < G.g && q * G.g + j < G.b) return G.start[G.m] + q * G.g + j;
    const uint64_t p = (j == G.g && G.g * (q + 1) <= G.b) ? q : r - G.b;
    uint64_t v = p + 1;
    uint32_t e = 0;
    for (;;) {
        const uint64_t w = div_small(v, kinv);
        if (w * G.k != v) break;
        v = w;
        ++e;
    }
    const uint32_t l = G.m - 1 - e;
    return G.start[l] + (v - 1) - div_small(v - 1, kinv);
}

}  // namespace idx
