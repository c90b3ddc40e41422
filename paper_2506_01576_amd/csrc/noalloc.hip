// Range lookups with no device allocation: idx_range_noalloc.
//
// idx_range needs scratch beside its outputs (the first matching rank of
// every range and the partial sums of the offsets scan) and takes it from the
// handle's allocator on every call.  This entry point takes it from one
// statically sized device array instead, so a caller that may not allocate
// (graph capture, a serving loop, a harness that forbids allocation) can run
// range lookups.  The kernels are those of idx_range.
//
// Each device holds its own copy of the array, at its own address, until the
// process ends.  In host code the array's name is only a host-side stand-in,
// so its device address is looked up once per device (hipGetSymbolAddress,
// with that device current) and only that address is handed to kernels.
// Every call on one device shares the array, which keeps the last call's
// contents: calls that overlap on one device race.  Nothing in it needs to
// start at zero: the count kernel writes every range's first rank and the
// scan writes every partial before either is read.
#include <mutex>

#include "internal.hpp"

namespace idx {
namespace {

constexpr size_t kScratchBytes = range_scratch_bytes(IDX_NOALLOC_MAX_RANGES);
static_assert(kScratchBytes % 256 == 0, "scratch is handed out in 256-byte units");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// Device address of this device's copy of the array (looked up once per
// device, with that device current); nullptr and the error when it fails.
void *scratch_on(int dev, hipError_t *err) {
    std::call_once(g_once[dev], [dev] {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[dev] = e;
        g_ptr[dev] = e == hipSuccess ? p : nullptr;
    });
    *err = g_err[dev];
    return g_ptr[dev];
}

}  // namespace
}  // namespace idx

using namespace idx;

extern "C" {

int idx_range_noalloc(idx_handle h, const void *lo, const void *hi, uint64_t m, uint64_t *out_offsets,
                      uint32_t *out_rowids, uint64_t capacity, uint64_t *total, idx_stream stream) {
    if (!h || !out_offsets || (m > 0 && (!lo || !hi))) return IDX_ERR_ARG;
    if (m > IDX_NOALLOC_MAX_RANGES) return IDX_ERR_SCRATCH;
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return hip_fail(de);
    if (dev < 0 || dev >= kMaxDevices) return IDX_ERR_ARG;
    hipError_t e = hipSuccess;
    void *p = scratch_on(dev, &e);
    if (!p) return hip_fail(e);
    h->last_stream = (hipStream_t)stream;
    return range_lookup_in(h, lo, hi, m, out_offsets, out_rowids, capacity, total, p, (hipStream_t)stream);
}

}  // extern "C"
