// The C ABI of libidx (include/idx.h): argument validation, ownership,
// allocation and dispatch to the kernel files.  No C++ exception leaves here.
#include <new>

#include "internal.hpp"

namespace idx {

static thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? IDX_ERR_NOMEM : IDX_ERR_HIP;
}

void *Alloc::get(size_t bytes, hipStream_t s) const {
    if (bytes == 0) bytes = 256;
    if (custom) return a.alloc(a.ctx, bytes, (idx_stream)s);
    void *p = nullptr;
    const hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Alloc::put(void *p, hipStream_t s) const {
    if (!p) return;
    if (custom) a.release(a.ctx, p, (idx_stream)s);
    else (void)hipFreeAsync(p, s);
}

namespace {

// Keep freed stream-ordered memory in the device pool instead of returning it
// to the driver, so repeated builds and range calls do not pay for mapping.
void tune_pool_once() {
    static thread_local int done_dev = -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (done_dev == dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
    done_dev = dev;
}

int cu_count_of_current_device() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 256;
    }
    return cus > 0 ? cus : 256;
}

size_t lds_max_of_current_device() {
    int dev = 0, bytes = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 64 * 1024;
    }
    return bytes > 0 ? (size_t)bytes : 64 * 1024;
}

// Layout allocations are padded so that a full-node vector read at the last
// (partial) node stays inside the buffer.
uint64_t padded_slots(uint64_t slots) { return ((slots + 63) / 64) * 64 + 64; }

void free_handle_buffers(idx_index *h, hipStream_t s) {
    drop_model(h, s);  // also frees a spare leaf-line buffer
    drop_splitters(h, s);
    h->alloc.put(h->keys, s);
    h->alloc.put(h->rowids, s);
    h->alloc.put(h->pin, s);
    h->keys = nullptr;
    h->rowids = nullptr;
    h->pin = nullptr;
}

}  // namespace
}  // namespace idx

using namespace idx;

extern "C" {

const char *idx_strerror(int status) {
    switch (status) {
        case IDX_OK: return "ok";
        case IDX_ERR_ARG: return "invalid argument";
        case IDX_ERR_RESERVED_ROWID: return "a row ID equals the reserved miss sentinel 0xFFFFFFFF";
        case IDX_ERR_NOMEM: return "device memory allocation failed";
        case IDX_ERR_HIP: return "HIP runtime or kernel launch error";
        case IDX_ERR_CAPACITY: return "range output exceeds the given capacity";
        case IDX_ERR_SCRATCH: return "request exceeds the library's fixed scratch (IDX_NOALLOC_MAX_RANGES ranges)";
        default: return "unknown status";
    }
}

int idx_last_hip_error(void) { return g_last_hip; }

}  // extern "C"

namespace {

// Validates (layout, k, flags, alloc) and creates a handle with its layout
// buffers allocated.  The first allocation precedes every other HIP call, so
// an allocator failure is reported without touching the device.
int new_handle(uint64_t n, int layout, uint32_t k, uint32_t flags, const idx_allocator *alloc, hipStream_t s,
               idx_index **out) {
    *out = nullptr;
    if (n > IDX_MAX_KEYS) return IDX_ERR_ARG;
    if (flags & ~(IDX_KEY_U64 | IDX_AOS | IDX_AOS_PADDED)) return IDX_ERR_ARG;
    if ((flags & IDX_AOS_PADDED) && !(flags & IDX_AOS)) return IDX_ERR_ARG;
    if (layout == IDX_BS) k = 1;
    else if (layout == IDX_EBS) {
        if (k != 2) return IDX_ERR_ARG;
    } else if (layout == IDX_EKS) {
        if (k < 2 || k > IDX_MAX_FANOUT) return IDX_ERR_ARG;
    } else {
        return IDX_ERR_ARG;
    }
    if (alloc && (!alloc->alloc || !alloc->release)) return IDX_ERR_ARG;

    idx_index *h = new (std::nothrow) idx_index();
    if (!h) return IDX_ERR_NOMEM;
    h->n = n;
    h->layout = layout;
    h->k = k;
    h->flags = flags;
    h->u64 = (flags & IDX_KEY_U64) != 0;
    h->aos = (flags & IDX_AOS) != 0;
    h->slots = n + (layout == IDX_EBS ? 1 : 0);
    h->geo = make_geo(n, layout == IDX_EKS ? k : 2);
    h->node = layout == IDX_EKS ? h->geo.g : 1;
    h->last_stream = s;
    if (alloc) {
        h->alloc.a = *alloc;
        h->alloc.custom = true;
    }
    const size_t kb = h->u64 ? 8 : 4;
    const uint64_t ps = padded_slots(h->slots);
    if (h->aos) {
        const uint64_t blocks = (ps + h->node - 1) / h->node;
        uint32_t stride = h->node * (uint32_t)(kb + 4);
        if (flags & IDX_AOS_PADDED) {
            uint32_t p2 = 16;
            while (p2 < stride) p2 <<= 1;
            stride = p2;
        }
        h->stride = stride;
        h->key_bytes = blocks * stride;
        h->row_bytes = 0;
    } else {
        h->key_bytes = ps * kb;
        h->row_bytes = ps * 4;
    }
    h->keys = h->alloc.get(h->key_bytes, s);
    if (!h->keys) {
        delete h;
        return alloc ? IDX_ERR_NOMEM : hip_fail((hipError_t)g_last_hip);
    }
    if (!alloc) tune_pool_once();
    if (h->row_bytes) {
        h->rowids = (uint32_t *)h->alloc.get(h->row_bytes, s);
        if (!h->rowids) {
            free_handle_buffers(h, s);
            delete h;
            return IDX_ERR_NOMEM;
        }
    }
    h->cu_count = cu_count_of_current_device();
    h->lds_max = lds_max_of_current_device();
    *out = h;
    return IDX_OK;
}

int finish_handle(idx_index *h, hipStream_t s, idx_handle *out) {
    if (resolve_params(h, nullptr, &h->params) != IDX_OK) {
        free_handle_buffers(h, s);
        delete h;
        return IDX_ERR_ARG;
    }
    *out = h;
    return IDX_OK;
}

}  // namespace

namespace idx {

// Handle life cycle for the other entry-point files (update.hip).
int handle_new(uint64_t n, int layout, uint32_t k, uint32_t flags, const idx_allocator *alloc, hipStream_t s,
               idx_index **out) {
    return new_handle(n, layout, k, flags, alloc, s, out);
}

int handle_finish(idx_index *h, hipStream_t s, idx_handle *out) { return finish_handle(h, s, out); }

void handle_discard(idx_index *h, hipStream_t s) {
    (void)hipStreamSynchronize(s);
    free_handle_buffers(h, s);
    delete h;
}

}  // namespace idx

extern "C" {

int idx_build(const void *keys, const uint32_t *rowids, uint64_t n, int layout, uint32_t k, uint32_t flags,
              const idx_allocator *alloc, idx_stream stream, idx_handle *out) {
    if (!out) return IDX_ERR_ARG;
    *out = nullptr;
    if (n > 0 && (!keys || !rowids)) return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    idx_index *h = nullptr;
    int rc = new_handle(n, layout, k, flags, alloc, s, &h);
    if (rc != IDX_OK) return rc;
    const size_t kb = h->u64 ? 8 : 4;

    // Temporaries: sorted SoA copy (unless the layout is BS/SoA, which the
    // sort writes directly), sort scratch, check flags.
    const bool direct = layout == IDX_BS && !h->aos;
    const size_t sorted_kb = direct ? 0 : ((n * kb + 255) / 256) * 256;
    const size_t sorted_rb = direct ? 0 : ((n * 4 + 255) / 256) * 256;
    const size_t sort_b = sort_temp_bytes(n, h->u64);
    char *tmp = (char *)h->alloc.get(sorted_kb + sorted_rb + sort_b + 256, s);
    if (!tmp) {
        free_handle_buffers(h, s);
        delete h;
        return IDX_ERR_NOMEM;
    }
    void *sk = direct ? h->keys : (void *)tmp;
    uint32_t *sr = direct ? h->rowids : (uint32_t *)(tmp + sorted_kb);
    void *sort_tmp = tmp + sorted_kb + sorted_rb;
    uint32_t *dflags = (uint32_t *)(tmp + sorted_kb + sorted_rb + sort_b);

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    uint32_t hflags[2] = {0, 0};
    do {
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) {
                rc = hip_fail(hipGetLastError());
                break;
            }
        if (rc != IDX_OK) break;
        hipError_t e = hipMemsetAsync(dflags, 0, 2 * sizeof(uint32_t), s);
        if (e != hipSuccess) { rc = hip_fail(e); break; }
        (void)hipEventRecord(ev[0], s);
        rc = sort_pairs(keys, rowids, n, h->u64, sk, sr, sort_tmp, s);
        if (rc != IDX_OK) break;
        (void)hipEventRecord(ev[1], s);
        rc = check_sorted(sk, sr, n, h->u64, dflags, s);
        if (rc != IDX_OK) break;
        if (!direct) {
            rc = build_layout(h, sk, sr, s);
            if (rc != IDX_OK) break;
        }
        (void)hipEventRecord(ev[2], s);
        e = hipMemcpyAsync(hflags, dflags, sizeof(hflags), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e); break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) h->ms_sort = ms;
        if (hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) h->ms_permute = direct ? 0.f : ms;
        (void)hipGetLastError();
    } while (0);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    h->alloc.put(tmp, s);
    if (rc == IDX_OK && hflags[1]) rc = IDX_ERR_RESERVED_ROWID;
    if (rc != IDX_OK) {
        (void)hipStreamSynchronize(s);
        free_handle_buffers(h, s);
        delete h;
        return rc;
    }
    h->unique = hflags[0] == 0;
    return finish_handle(h, s, out);
}

int idx_relayout(idx_handle src, int layout, uint32_t k, uint32_t flags, const idx_allocator *alloc,
                 idx_stream stream, idx_handle *out) {
    if (!out) return IDX_ERR_ARG;
    *out = nullptr;
    if (!src || src->layout != IDX_BS || src->aos) return IDX_ERR_ARG;
    if (((flags & IDX_KEY_U64) != 0) != src->u64) return IDX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    idx_index *h = nullptr;
    int rc = new_handle(src->n, layout, k, flags, alloc, s, &h);
    if (rc != IDX_OK) return rc;
    h->unique = src->unique;
    src->last_stream = s;
    if (layout == IDX_BS && !h->aos) {
        hipError_t e = hipMemcpyAsync(h->keys, src->keys, src->n * (h->u64 ? 8 : 4), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h->rowids, src->rowids, src->n * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = hip_fail(e);
    } else {
        rc = build_layout(h, src->keys, src->rowids, s);
    }
    if (rc != IDX_OK) {
        (void)hipStreamSynchronize(s);
        free_handle_buffers(h, s);
        delete h;
        return rc;
    }
    return finish_handle(h, s, out);
}

int idx_point(idx_handle h, const void *queries, uint64_t m, uint32_t *out_rowid, idx_stream stream) {
    if (!h) return IDX_ERR_ARG;
    if (m > 0 && (!queries || !out_rowid)) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return point_lookup(h, queries, m, out_rowid, (hipStream_t)stream);
}

int idx_range(idx_handle h, const void *lo, const void *hi, uint64_t m, uint64_t *out_offsets, uint32_t *out_rowids,
              uint64_t capacity, uint64_t *total, idx_stream stream) {
    if (!h || !out_offsets) return IDX_ERR_ARG;
    if (m > 0 && (!lo || !hi)) return IDX_ERR_ARG;
    if (m > 0xFFFFFFFFull * 256ull) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return range_lookup(h, lo, hi, m, out_offsets, out_rowids, capacity, total, (hipStream_t)stream);
}

int idx_destroy(idx_handle h) {
    if (!h) return IDX_OK;
    if (h->batch_refs) return IDX_ERR_ARG;  // a batch still reads its buffers
    // Work still queued on the last stream may read the buffers.
    (void)hipStreamSynchronize(h->last_stream);
    (void)hipGetLastError();
    free_handle_buffers(h, h->last_stream);
    (void)hipStreamSynchronize(h->last_stream);
    (void)hipGetLastError();
    delete h;
    return IDX_OK;
}

int idx_get_info(idx_handle h, idx_info *o) {
    if (!h || !o) return IDX_ERR_ARG;
    idx_info i{};
    i.n = h->n;
    i.slots = h->slots;
    i.footprint_bytes = h->aos ? ((h->slots + h->node - 1) / h->node) * h->stride
                               : h->slots * ((h->u64 ? 8 : 4) + 4);
    i.layout = h->layout;
    i.k = h->k;
    i.flags = h->flags;
    i.unique = h->unique ? 1u : 0u;
    i.levels = h->geo.levels;
    i.full_levels = h->geo.m;
    i.bottom_keys = h->geo.b;
    i.build_ms_sort = h->ms_sort;
    i.build_ms_permute = h->ms_permute;
    *o = i;
    return IDX_OK;
}

int idx_export(idx_handle h, void *keys_out, uint32_t *rowids_out, idx_stream stream) {
    if (!h) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return export_layout(h, keys_out, rowids_out, (hipStream_t)stream);
}

int idx_learn(idx_handle h, uint32_t leaves, uint32_t epochs, uint32_t feature, idx_stream stream) {
    if (!h || h->batch_refs) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return learn(h, leaves, epochs, feature, (hipStream_t)stream);
}

int idx_learn_batch(const idx_handle *indexes, uint32_t count, const uint32_t *leaves, uint32_t epochs,
                    uint32_t feature, idx_stream stream) {
    if (!indexes || count == 0) return IDX_ERR_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (!indexes[i] || indexes[i]->batch_refs) return IDX_ERR_ARG;
    for (uint32_t i = 0; i < count; ++i) indexes[i]->last_stream = (hipStream_t)stream;
    return learn_batch(indexes, count, leaves, epochs, feature, (hipStream_t)stream);
}

int idx_learn_stats_get(idx_handle h, idx_learn_stats *out) {
    if (!h || !out) return IDX_ERR_ARG;
    return learn_stats(h, out);
}

int idx_learn_export(idx_handle h, void *leaves_out, idx_stream stream) {
    if (!h) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return learn_export(h, leaves_out, (hipStream_t)stream);
}

int idx_unlearn(idx_handle h) {
    if (!h || h->batch_refs) return IDX_ERR_ARG;
    drop_model(h, h->last_stream);
    return IDX_OK;
}

int idx_learn_eval(idx_handle h, uint32_t feature, const float *root_ab, uint32_t leaves, const float *leaf_ab,
                   double *root_acc, double *leaf_acc, idx_stream stream) {
    if (!h) return IDX_ERR_ARG;
    h->last_stream = (hipStream_t)stream;
    return learn_eval(h, feature, root_ab, leaves, leaf_ab, root_acc, leaf_acc, (hipStream_t)stream);
}

uint64_t idx_slot_rank(uint64_t n, uint32_t k, uint64_t slot) {
    if (k < 2 || slot >= n) return ~0ull;
    const Geo G = make_geo(n, k);
    return slot_rank(G, slot);
}

uint64_t idx_rank_slot(uint64_t n, uint32_t k, uint64_t rank) {
    if (k < 2 || k > IDX_MAX_FANOUT || n > IDX_MAX_KEYS || rank >= n) return ~0ull;
    const Geo G = make_geo(n, k);
    if (k == 2) return rank_slot_binary(G, rank);
    return rank_slot_general(G, rank, ~0ull / k + 1);
}

int idx_set_params(idx_handle h, const idx_lookup_params *p) {
    if (!h) return IDX_ERR_ARG;
    idx_lookup_params r{};
    const int rc = resolve_params(h, p, &r);
    if (rc != IDX_OK) return rc;
    // the batch descriptors holding h copied its use of the model, its early
    // exit, its EKS lanes per lookup, its pinned levels (and point at its pin
    // table) and its range fill
    if (h->batch_refs && (r.model != h->params.model || r.early_exit != h->params.early_exit ||
                          r.group != h->params.group || r.lds_levels != h->params.lds_levels ||
                          r.range_scan != h->params.range_scan))
        return IDX_ERR_ARG;
    h->params = r;
    return IDX_OK;
}

int idx_get_params(idx_handle h, idx_lookup_params *out) {
    if (!h || !out) return IDX_ERR_ARG;
    *out = h->params;
    return IDX_OK;
}

}  // extern "C"
