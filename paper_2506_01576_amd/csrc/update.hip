// The read-mostly update path: a new index over an existing sorted array
// plus a batch of new pairs (Section 8.5 rebuilds the whole structure for a
// batch of updates; here only the batch is sorted and then merged), and
// saving / loading a handle as one host byte blob.
//
// Merge: the batch is radix-sorted, then merged with the index's sorted
// array by merge path: each workgroup takes a tile of output positions, finds
// by binary search on the tile's first and last diagonal how many of them
// come from the old array, stages both input pieces in LDS and merges there.
// Old keys go first on equal keys, so the result is the stable sort of (old
// pairs in their order, new pairs in theirs) -- exactly what building from
// the concatenation gives.
// The merged array is then checked and laid out like a fresh build.
#include <cstring>
#include <new>

#include "internal.hpp"
#include "learned_model.hpp"

namespace idx {
namespace {

constexpr int MT = 256;            // threads per merge workgroup
constexpr int MPER = 8;            // outputs per thread
constexpr int MTILE = MT * MPER;   // outputs per workgroup

// Old elements among the first d outputs: the first i with A[i] > B[d - i - 1]
// (A wins ties), i in [max(0, d - nb), min(d, na)].
template <typename K>
__device__ __forceinline__ uint64_t merge_split(const K *a, uint64_t na, const K *b, uint64_t nb, uint64_t d) {
    uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= b[d - mid - 1]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One output tile per workgroup: the tile's two input pieces come into LDS
// with coalesced loads, each thread merges MPER outputs from there into an
// LDS output tile, which leaves with coalesced stores.
template <typename K>
__global__ __launch_bounds__(MT) void k_merge(const K *__restrict__ ak, const uint32_t *__restrict__ ar, uint64_t na,
                                              const K *__restrict__ bk, const uint32_t *__restrict__ br, uint64_t nb,
                                              K *__restrict__ ok, uint32_t *__restrict__ orow) {
    __shared__ K s_in[MTILE];
    __shared__ uint32_t s_inr[MTILE];
    __shared__ K s_out[MTILE];
    __shared__ uint32_t s_outr[MTILE];
    __shared__ uint64_t s_split[2];
    const uint64_t total = na + nb;
    const uint64_t d0 = (uint64_t)blockIdx.x * MTILE;
    const uint64_t d1 = d0 + MTILE < total ? d0 + MTILE : total;
    if (threadIdx.x == 0) s_split[0] = merge_split(ak, na, bk, nb, d0);
    if (threadIdx.x == 1) s_split[1] = merge_split(ak, na, bk, nb, d1);
    __syncthreads();
    const uint64_t ia = s_split[0], ib = s_split[1];
    const uint64_t ja = d0 - ia, jb = d1 - ib;
    const uint32_t la = (uint32_t)(ib - ia), lb = (uint32_t)(jb - ja);
    for (uint32_t e = threadIdx.x; e < la; e += MT) {
        s_in[e] = ak[ia + e];
        s_inr[e] = ar[ia + e];
    }
    for (uint32_t e = threadIdx.x; e < lb; e += MT) {
        s_in[la + e] = bk[ja + e];
        s_inr[la + e] = br[ja + e];
    }
    __syncthreads();
    const K *A = s_in;
    const K *B = s_in + la;
    const uint32_t dl = threadIdx.x * MPER;
    if (dl < la + lb) {
        uint32_t i = (uint32_t)merge_split(A, la, B, lb, dl), j = dl - i;
        const uint32_t end = dl + MPER < la + lb ? dl + MPER : la + lb;
        for (uint32_t d = dl; d < end; ++d) {
            const bool take_a = j >= lb || (i < la && A[i] <= B[j]);
            if (take_a) {
                s_out[d] = A[i];
                s_outr[d] = s_inr[i];
                ++i;
            } else {
                s_out[d] = B[j];
                s_outr[d] = s_inr[la + j];
                ++j;
            }
        }
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < la + lb; e += MT) {
        ok[d0 + e] = s_out[e];
        orow[d0 + e] = s_outr[e];
    }
}

uint32_t merge_grid(uint64_t total) {
    const uint64_t g = (total + MTILE - 1) / MTILE;
    return (uint32_t)(g ? g : 1);
}

// ---- blob format (host, little endian)
constexpr char kMagic[8] = {'I', 'D', 'X', 'B', 'L', 'O', 'B', '2'};  // 2: spline bins with 26-bit first leaves

struct BlobHeader {
    char magic[8];
    uint64_t n;
    int32_t layout;
    uint32_t k;
    uint32_t flags;
    uint32_t unique;
    uint64_t key_bytes;
    uint64_t row_bytes;
    uint32_t has_model;
    uint32_t leaves;
    RootRec root;
    idx_learn_stats stats;
};

// Bytes of a spline root's bin records; 0 for a linear root.
uint64_t spline_bytes(const RootRec &R) {
    return R.mode == IDX_FEATURE_SPLINE ? (uint64_t)R.nb * sizeof(SplineBin) : 0;
}

uint64_t blob_size(const idx_index *h) {
    uint64_t s = sizeof(BlobHeader) + h->key_bytes + h->row_bytes;
    if (h->learned) s += (uint64_t)h->learned->root.L * sizeof(LeafRec) + spline_bytes(h->learned->root);
    return s;
}

}  // namespace
}  // namespace idx

using namespace idx;

extern "C" {

int idx_merge(idx_handle src, const void *keys, const uint32_t *rowids, uint64_t m, int layout, uint32_t k,
              uint32_t flags, const idx_allocator *alloc, idx_stream stream, idx_handle *out) {
    if (!out) return IDX_ERR_ARG;
    *out = nullptr;
    if (!src || src->layout != IDX_BS || src->aos) return IDX_ERR_ARG;
    if (((flags & IDX_KEY_U64) != 0) != src->u64) return IDX_ERR_ARG;
    if (m > 0 && (!keys || !rowids)) return IDX_ERR_ARG;
    if (m > IDX_MAX_KEYS || src->n + m > IDX_MAX_KEYS) return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    src->last_stream = s;
    const uint64_t n = src->n + m;
    idx_index *h = nullptr;
    int rc = handle_new(n, layout, k, flags, alloc, s, &h);
    if (rc != IDX_OK) return rc;
    const size_t kb = h->u64 ? 8 : 4;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const bool direct = layout == IDX_BS && !h->aos;
    const size_t merged_kb = direct ? 0 : up(n * kb), merged_rb = direct ? 0 : up(n * 4);
    const size_t delta_kb = up(m * kb), delta_rb = up(m * 4), sort_b = sort_temp_bytes(m, h->u64);
    char *tmp = (char *)h->alloc.get(merged_kb + merged_rb + delta_kb + delta_rb + sort_b + 256, s);
    if (!tmp) {
        handle_discard(h, s);
        return IDX_ERR_NOMEM;
    }
    void *mk = direct ? h->keys : (void *)tmp;
    uint32_t *mr = direct ? h->rowids : (uint32_t *)(tmp + merged_kb);
    void *dk = tmp + merged_kb + merged_rb;
    uint32_t *dr = (uint32_t *)((char *)dk + delta_kb);
    void *sort_tmp = (char *)dr + delta_rb;
    uint32_t *dflags = (uint32_t *)((char *)sort_tmp + sort_b);
    uint32_t hflags[2] = {0, 0};
    do {
        hipError_t e = hipMemsetAsync(dflags, 0, 2 * sizeof(uint32_t), s);
        if (e != hipSuccess) { rc = hip_fail(e); break; }
        rc = sort_pairs(keys, rowids, m, h->u64, dk, dr, sort_tmp, s);
        if (rc != IDX_OK) break;
        if (n > 0) {
            if (h->u64)
                hipLaunchKernelGGL(k_merge<uint64_t>, dim3(merge_grid(n)), dim3(MT), 0, s,
                                   (const uint64_t *)src->keys, src->rowids, src->n, (const uint64_t *)dk, dr, m,
                                   (uint64_t *)mk, mr);
            else
                hipLaunchKernelGGL(k_merge<uint32_t>, dim3(merge_grid(n)), dim3(MT), 0, s,
                                   (const uint32_t *)src->keys, src->rowids, src->n, (const uint32_t *)dk, dr, m,
                                   (uint32_t *)mk, mr);
            e = hipGetLastError();
            if (e != hipSuccess) { rc = hip_fail(e); break; }
        }
        rc = check_sorted(mk, mr, n, h->u64, dflags, s);
        if (rc != IDX_OK) break;
        if (!direct) {
            rc = build_layout(h, mk, mr, s);
            if (rc != IDX_OK) break;
        }
        e = hipMemcpyAsync(hflags, dflags, sizeof(hflags), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e); break; }
    } while (0);
    h->alloc.put(tmp, s);
    if (rc == IDX_OK && hflags[1]) rc = IDX_ERR_RESERVED_ROWID;
    if (rc != IDX_OK) {
        handle_discard(h, s);
        return rc;
    }
    h->unique = hflags[0] == 0;
    return handle_finish(h, s, out);
}

int idx_save(idx_handle h, void *blob, uint64_t capacity, uint64_t *size, idx_stream stream) {
    if (!h || !size) return IDX_ERR_ARG;
    const uint64_t need = blob_size(h);
    *size = need;
    if (!blob) return IDX_OK;
    if (capacity < need) return IDX_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    BlobHeader hd{};
    std::memcpy(hd.magic, kMagic, sizeof(kMagic));
    hd.n = h->n;
    hd.layout = h->layout;
    hd.k = h->k;
    hd.flags = h->flags;
    hd.unique = h->unique ? 1u : 0u;
    hd.key_bytes = h->key_bytes;
    hd.row_bytes = h->row_bytes;
    if (h->learned) {
        hd.has_model = 1;
        hd.leaves = h->learned->root.L;
        hd.root = h->learned->root;
        hd.stats = h->learned->stats;
    }
    char *p = (char *)blob;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    IDX_HIP(hipMemcpyAsync(p, h->keys, h->key_bytes, hipMemcpyDeviceToHost, s));
    p += h->key_bytes;
    if (h->row_bytes) IDX_HIP(hipMemcpyAsync(p, h->rowids, h->row_bytes, hipMemcpyDeviceToHost, s));
    p += h->row_bytes;
    if (h->learned) {
        IDX_HIP(hipMemcpyAsync(p, h->learned->leaves, (size_t)hd.leaves * sizeof(LeafRec), hipMemcpyDeviceToHost, s));
        p += (size_t)hd.leaves * sizeof(LeafRec);
        if (spline_bytes(hd.root))
            IDX_HIP(hipMemcpyAsync(p, h->learned->spline, spline_bytes(hd.root), hipMemcpyDeviceToHost, s));
    }
    IDX_HIP(hipStreamSynchronize(s));
    return IDX_OK;
}

int idx_load(const void *blob, uint64_t size, const idx_allocator *alloc, idx_stream stream, idx_handle *out) {
    if (!out) return IDX_ERR_ARG;
    *out = nullptr;
    if (!blob || size < sizeof(BlobHeader)) return IDX_ERR_ARG;
    BlobHeader hd;
    std::memcpy(&hd, blob, sizeof(hd));
    if (std::memcmp(hd.magic, kMagic, sizeof(kMagic)) != 0) return IDX_ERR_ARG;
    if (hd.has_model > 1 || (hd.has_model && (hd.layout != IDX_BS || hd.leaves == 0 || hd.leaves > (1u << 26) ||
                                              hd.root.L != hd.leaves || hd.root.mode == 0 ||
                                              hd.root.mode > IDX_FEATURE_SPLINE ||
                                              (hd.root.mode == IDX_FEATURE_SPLINE &&
                                               (hd.root.nb == 0 || hd.root.nb > spline_bins(hd.n) ||
                                                hd.root.shift > 64 || (hd.root.shift == 64 && hd.root.nb != 1) ||
                                                (hd.root.bfeat != IDX_FEATURE_LINEAR &&
                                                 hd.root.bfeat != IDX_FEATURE_LOG))))))
        return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    idx_index *h = nullptr;
    int rc = handle_new(hd.n, hd.layout, hd.k, hd.flags, alloc, s, &h);
    if (rc != IDX_OK) return rc;
    const uint64_t leaf_b = hd.has_model ? (uint64_t)hd.leaves * sizeof(LeafRec) : 0;
    const uint64_t spl_b = hd.has_model ? spline_bytes(hd.root) : 0;
    if (h->key_bytes != hd.key_bytes || h->row_bytes != hd.row_bytes ||
        size != sizeof(BlobHeader) + hd.key_bytes + hd.row_bytes + leaf_b + spl_b) {
        handle_discard(h, s);
        return IDX_ERR_ARG;
    }
    const char *p = (const char *)blob + sizeof(BlobHeader);
    hipError_t e = hipMemcpyAsync(h->keys, p, h->key_bytes, hipMemcpyHostToDevice, s);
    p += h->key_bytes;
    if (e == hipSuccess && h->row_bytes) e = hipMemcpyAsync(h->rowids, p, h->row_bytes, hipMemcpyHostToDevice, s);
    p += h->row_bytes;
    if (e == hipSuccess && hd.has_model) {
        LearnedModel *M = new (std::nothrow) LearnedModel();
        if (M) M->leaves = (LeafRec *)h->alloc.get(leaf_b, s);
        if (M && M->leaves && spl_b) M->spline = (SplineBin *)h->alloc.get(spl_b, s);
        if (!M || !M->leaves || (spl_b && !M->spline)) {
            if (M && M->leaves) h->alloc.put(M->leaves, s);
            delete M;
            handle_discard(h, s);
            return IDX_ERR_NOMEM;
        }
        M->root = hd.root;
        M->root.bins = spl_b ? M->spline : nullptr;
        M->stats = hd.stats;
        h->learned = M;
        e = hipMemcpyAsync(M->leaves, p, leaf_b, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && spl_b) e = hipMemcpyAsync(M->spline, p + leaf_b, spl_b, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e);
        handle_discard(h, s);
        return rc;
    }
    h->unique = hd.unique != 0;
    return handle_finish(h, s, out);
}

}  // extern "C"
