// Learned rank model on a sorted-array index (BS layout): a two-stage FP32
// model -- a linear root over a monotone key feature selects one of L leaves,
// each leaf a line over the leaf-local key offset -- trained on the GPU on the
// index's own (key, rank) pairs, then used to narrow every lookup to a window
// bounded by the leaf's measured error (the window-then-search idea of the
// PGM index the paper compares with, Section 8; the last-mile search is the
// expensive step, Section 9).
//
// Exactness does not depend on the model.  The root is non-decreasing in the
// key (non-negative slope over a non-decreasing feature, round-to-nearest
// arithmetic without contraction), so the keys of a leaf form one contiguous
// rank interval [base, base + size) and every key that maps to a leaf has its
// lower bound inside that interval (or at its end).  Inside a leaf the
// prediction is non-decreasing too, and the error bounds are measured with the
// same device function over all of the leaf's keys; a window
// [pred + elo, pred + ehi + 1] clamped to the leaf interval therefore contains
// the lower bound of any query, member or not.
//
// Training (per stage, `epochs` times): a forward/backward kernel evaluates
// the FP32 prediction and accumulates, in FP64, the loss sum, the gradient
// sums (residual * feature, residual) and the Hessian sums (feature^2,
// feature, count); an update kernel takes the Newton step
// theta -= H^-1 g, which for this quadratic loss reaches the least-squares
// fit in one step from zero, the second step correcting FP32 rounding.
#include <climits>

#include <new>

#include "internal.hpp"
#include "access.hpp"
#include "learned_model.hpp"
#include "qio.hpp"

namespace idx {

namespace {

constexpr int LT = 256;  // threads per block in the training kernels
constexpr int CHUNK = 32;  // consecutive keys per thread in the per-leaf passes

template <typename K, bool AOS>
__global__ __launch_bounds__(LT) void k_root_accum(Load<K, AOS> keys, uint64_t n, const RootRec *Rp,
                                                   double *__restrict__ acc) {
    __shared__ double s[LT / kWave][NACC];
    const RootRec R = *Rp;
    double a[NACC] = {0, 0, 0, 0, 0, 0};
    const double scale = (double)R.L / (double)n;
    for (uint64_t i = (uint64_t)blockIdx.x * LT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * LT) {
        const uint64_t key = (uint64_t)keys.key(i);
        const float t = (float)((double)i * scale);
        float x, pred;
        if (R.mode == IDX_FEATURE_SPLINE) {
            x = 0.f;  // no parameters to fit: only the loss is wanted
            (void)spline_leaf(R, key, &pred);
        } else {
            x = key_feature(key, R.mode);
            pred = __fadd_rn(__fmul_rn(R.a1, x), R.a0);
        }
        const float r = __fsub_rn(pred, t);  // forward residual
        a[0] += 1.0;
        a[1] += x;
        a[2] += (double)x * x;
        a[3] += r;
        a[4] += (double)r * x;
        a[5] += (double)r * r;
    }
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
        const double v = wave_sum(a[j]);
        if (lane == 0) s[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        double v = 0;
        for (int w = 0; w < LT / kWave; ++w) v += s[w][threadIdx.x];
        atomicAdd(&acc[threadIdx.x], v);
    }
}

__global__ void k_root_update(RootRec *R, const double *acc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) newton_linear(acc, R->a0, R->a1);
}

__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_fill_f64(double *p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Keys per leaf: each wave counts the leaf runs of its 64 * CHUNK
// consecutive keys, one atomic per run and step.
template <typename K, bool AOS>
__global__ __launch_bounds__(LT) void k_leaf_count(Load<K, AOS> keys, uint64_t n, const RootRec *Rp,
                                                   unsigned long long *__restrict__ count) {
    const RootRec R = *Rp;
    const uint64_t b = ((uint64_t)blockIdx.x * LT + (threadIdx.x & ~(uint32_t)(kWave - 1))) * CHUNK;
    const uint64_t e = b + (uint64_t)kWave * CHUNK < n ? b + (uint64_t)kWave * CHUNK : n;
    wave_leaf_counts(
        b, e, [&](uint64_t i) { return leaf_of(R, (uint64_t)keys.key(i)); },
        [&](uint32_t l, uint32_t c) { atomicAdd(&count[l], (unsigned long long)c); });
}

// Leaf records from the exclusive scan of the per-leaf counts (base[l] =
// keys before leaf l, base[L] = n): base rank, size, first key; parameters
// start at zero and error bounds empty.
template <typename K, bool AOS>
__global__ void k_leaf_init(Load<K, AOS> keys, const unsigned long long *__restrict__ base, uint32_t L,
                            LeafRec *__restrict__ leaves) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    LeafRec r{};
    r.base = (uint32_t)base[l];
    r.size = (uint32_t)(base[l + 1] - base[l]);
    r.kmin = r.size ? (uint64_t)keys.key(r.base) : 0ull;
    r.b0 = 0.f;
    r.b1 = 0.f;
    r.elo = INT_MAX;
    r.ehi = INT_MIN;
    leaves[l] = r;
}

// The workgroup's leaves' keys into LDS (false: the range is too large).
template <typename K, bool AOS>
__device__ __forceinline__ bool stage_leaf_keys(Load<K, AOS> keys, const LeafRec *__restrict__ leaves, uint32_t L,
                                                K *s_key, uint32_t cap, uint64_t &kb) {
    const uint32_t l0 = blockIdx.x * kLeafBlock;
    if (l0 >= L) return false;  // workgroup-uniform (a launch over no leaves)
    const uint32_t l1 = l0 + kLeafBlock < L ? l0 + kLeafBlock : L;
    kb = leaves[l0].base;
    const uint64_t ke = (uint64_t)leaves[l1 - 1].base + leaves[l1 - 1].size;
    if (ke - kb > cap) return false;  // workgroup-uniform
    stage_keys<K>([&](uint64_t i) { return keys.key(i); }, kb, ke, s_key);
    return true;
}

// Per-leaf sums, one thread per leaf over its key range; a leaf of more than
// kLeafCap keys gets zero sums here and raises *big for k_leaf_accum_big.
// UPDATE (training): a leaf of at most kLeafCap keys takes its Newton step
// at once from the sums in registers, which are not stored; the large
// leaves' steps follow k_leaf_accum_big (k_leaf_update_big).
// The staging area holds `cap` keys (dynamic LDS, sized by stage_cap).
template <typename K, bool AOS, bool UPDATE = false>
__global__ __launch_bounds__(kLeafBlock) void k_leaf_accum_small(Load<K, AOS> keys, LeafRec *__restrict__ leaves,
                                                                 uint32_t L, double *__restrict__ acc, uint32_t *big,
                                                                 uint32_t cap) {
    extern __shared__ __align__(16) char smem_stage[];
    K *s_key = (K *)smem_stage;
    uint64_t kb;
    const bool staged = stage_leaf_keys(keys, leaves, L, s_key, cap, kb);
    const uint32_t l = blockIdx.x * kLeafBlock + threadIdx.x;
    if (l >= L) return;
    const LeafRec r = leaves[l];
    double a[NACC] = {0, 0, 0, 0, 0, 0};
    if (r.size > kLeafCap) *big = 1u;
    else if (staged) leaf_sums_thread([&](uint64_t i) { return (uint64_t)s_key[i - kb]; }, r, a);
    else leaf_sums_thread([&](uint64_t i) { return (uint64_t)keys.key(i); }, r, a);
    if (UPDATE && r.size <= kLeafCap) {
        float b0 = r.b0, b1 = r.b1;
        newton_linear(a, b0, b1);
        leaves[l].b0 = b0;
        leaves[l].b1 = b1;
        return;
    }
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[(uint64_t)l * NACC + j] = a[j];
}

// The keys of leaves larger than kLeafCap: the wave walk over all keys,
// skipping every step without such a key (nothing to do when *big is 0).
template <typename K, bool AOS>
__global__ __launch_bounds__(LT) void k_leaf_accum_big(Load<K, AOS> keys, uint64_t n, const RootRec *Rp,
                                                       const LeafRec *__restrict__ leaves, double *__restrict__ acc,
                                                       const uint32_t *big) {
    if (*big == 0u) return;
    const RootRec R = *Rp;
    // this wave's CHUNK * 64 consecutive keys
    const uint64_t b = ((uint64_t)blockIdx.x * LT + (threadIdx.x & ~(uint32_t)(kWave - 1))) * CHUNK;
    const uint64_t e = b + (uint64_t)kWave * CHUNK < n ? b + (uint64_t)kWave * CHUNK : n;
    wave_leaf_sums<NACC>(
        b, e,
        [&](uint64_t i, uint32_t &l, double *a) {
            const uint64_t key = (uint64_t)keys.key(i);
            l = leaf_of(R, key);
            const LeafRec L = leaves[l];
            if (L.size <= kLeafCap) return false;
            leaf_terms(L, i, key, a);
            return true;
        },
        [&](uint32_t l, const double *v) {
#pragma unroll
            for (int j = 0; j < NACC; ++j) atomicAdd(&acc[(uint64_t)l * NACC + j], v[j]);
        });
}

// The Newton step of the leaves larger than kLeafCap (nothing to do when
// *big is 0; the others stepped in k_leaf_accum_small).
__global__ void k_leaf_update_big(LeafRec *__restrict__ leaves, const double *__restrict__ acc, uint32_t L,
                                  const uint32_t *big) {
    if (*big == 0u) return;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    LeafRec r = leaves[l];
    if (r.size <= kLeafCap) return;
    newton_linear(acc + (uint64_t)l * NACC, r.b0, r.b1);
    leaves[l].b0 = r.b0;
    leaves[l].b1 = r.b1;
}

// Per-leaf error bounds, one thread per leaf of at most kLeafCap keys; each
// leaf's squared residuals go to loss[l] (0 for the large leaves, whose loss
// k_leaf_errors_big adds to the total itself).  `loss` is the start of the
// per-leaf accumulators, which training no longer needs: dense, so the
// writes here and the reads in k_leaf_finish move 8 bytes per leaf, not a
// strided line each.
template <typename K, bool AOS>
__global__ __launch_bounds__(kLeafBlock) void k_leaf_errors_small(Load<K, AOS> keys, LeafRec *__restrict__ leaves,
                                                                  uint32_t L, double *__restrict__ loss, uint32_t cap) {
    extern __shared__ __align__(16) char smem_stage[];
    K *s_key = (K *)smem_stage;
    uint64_t kb;
    const bool staged = stage_leaf_keys(keys, leaves, L, s_key, cap, kb);
    const uint32_t l = blockIdx.x * kLeafBlock + threadIdx.x;
    if (l >= L) return;
    const LeafRec r = leaves[l];
    double ls = 0.0;
    if (r.size != 0 && r.size <= kLeafCap) {
        long long lo, hi;
        if (staged) leaf_errs_thread([&](uint64_t i) { return (uint64_t)s_key[i - kb]; }, r, lo, hi, &ls);
        else leaf_errs_thread([&](uint64_t i) { return (uint64_t)keys.key(i); }, r, lo, hi, &ls);
        leaves[l].elo = (int32_t)lo;
        leaves[l].ehi = (int32_t)hi;
    }
    loss[l] = ls;
}

// Error bounds of the leaves larger than kLeafCap (the wave walk).
template <typename K, bool AOS>
__global__ __launch_bounds__(LT) void k_leaf_errors_big(Load<K, AOS> keys, uint64_t n, const RootRec *Rp,
                                                        LeafRec *__restrict__ leaves, const uint32_t *big,
                                                        double *__restrict__ loss) {
    if (*big == 0u) return;
    const RootRec R = *Rp;
    const uint64_t b = ((uint64_t)blockIdx.x * LT + (threadIdx.x & ~(uint32_t)(kWave - 1))) * CHUNK;
    const uint64_t e = b + (uint64_t)kWave * CHUNK < n ? b + (uint64_t)kWave * CHUNK : n;
    double ls = 0.0;  // this lane's squared residuals over the large leaves' keys
    wave_leaf_maxes(
        b, e,
        [&](uint64_t i, uint32_t &l, long long *a) {
            const uint64_t key = (uint64_t)keys.key(i);
            l = leaf_of(R, key);
            const LeafRec L = leaves[l];
            if (L.size <= kLeafCap) return false;
            const long long err = leaf_err(L, i, key);
            a[0] = -err;
            a[1] = err;
            ls += leaf_sq_residual(L, i, key);
            return true;
        },
        [&](uint32_t l, const long long *v) {
            atomicMin(&leaves[l].elo, (int32_t)(-v[0]));
            atomicMax(&leaves[l].ehi, (int32_t)v[1]);
        });
    ls = wave_sum(ls);
    if ((threadIdx.x & (kWave - 1)) == 0 && ls != 0.0) atomicAdd(loss, ls);
}

// Empty leaves get a zero window; statistics of the windows and the leaves'
// losses (loss[l], written by k_leaf_errors_small).
__global__ __launch_bounds__(256) void k_leaf_finish(LeafRec *__restrict__ leaves, uint32_t L,
                                                     const double *__restrict__ loss,
                                                     double *__restrict__ stats /* sum_w*size, max_w, sum loss */) {
    __shared__ double s_ws[256 / kWave], s_wm[256 / kWave], s_ls[256 / kWave];
    double ws = 0, wmax = 0, ls = 0;
    for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < L; l += gridDim.x * blockDim.x) {
        ls += loss[l];
        LeafRec r = leaves[l];
        if (r.size == 0 || r.elo > r.ehi) {
            leaves[l].elo = 0;
            leaves[l].ehi = -1;
        } else {
            const double w = (double)r.ehi - (double)r.elo + 2.0;  // window slots incl. one past
            ws += w * r.size;
            wmax = w > wmax ? w : wmax;
        }
    }
    ws = wave_sum(ws);
    ls = wave_sum(ls);
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(wmax, off, kWave);
        wmax = o > wmax ? o : wmax;
    }
    const uint32_t wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_ws[wave] = ws;
        s_wm[wave] = wmax;
        s_ls[wave] = ls;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / kWave; ++w) {
            ws += s_ws[w];
            wmax = s_wm[w] > wmax ? s_wm[w] : wmax;
            ls += s_ls[w];
        }
        atomicAdd(&stats[0], ws);
        atomicAdd(&stats[2], ls);
        // max via compare-and-swap on the bit pattern (values are >= 0)
        unsigned long long *p = (unsigned long long *)&stats[1];
        unsigned long long old = *p;
        while (__longlong_as_double(old) < wmax) {
            const unsigned long long prev = atomicCAS(p, old, __double_as_longlong(wmax));
            if (prev == old) break;
            old = prev;
        }
    }
}

// Spline root geometry from the smallest and largest build key (one thread).
template <typename K, bool AOS>
__global__ void k_spline_geometry(Load<K, AOS> keys, uint64_t n, RootRec *R) {
    if (blockIdx.x == 0 && threadIdx.x == 0) spline_geometry(*R, (uint64_t)keys.key(0), (uint64_t)keys.key(n - 1), n);
}

// Spline root bins, one thread per bin.
template <typename K, bool AOS>
__global__ void k_spline_bins(Load<K, AOS> keys, uint64_t n, const RootRec *Rp, SplineBin *__restrict__ bins) {
    const RootRec R = *Rp;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= R.nb) return;
    bins[b] = spline_bin([&](uint64_t i) { return (uint64_t)keys.key(i); }, n, R, b);
}

uint32_t grid_for(uint64_t threads, uint32_t block) {
    uint64_t b = (threads + block - 1) / block;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) b = 0x7FFFFFFFull;
    return (uint32_t)b;
}

// Per-leaf key counts, their exclusive scan and the leaf records.
template <typename K, bool AOS>
int leaf_layout(Load<K, AOS> keys, uint64_t n, const RootRec *d_root, uint32_t L, unsigned long long *count,
                uint64_t *partial, LeafRec *leaves, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((uint64_t)L + 1, 256)), dim3(256), 0, s, (uint64_t *)count,
                       (uint64_t)L + 1);
    hipLaunchKernelGGL((k_leaf_count<K, AOS>), dim3(grid_for((n + CHUNK - 1) / CHUNK, LT)), dim3(LT), 0, s, keys, n,
                       d_root, count);
    IDX_LAUNCH_CHECK();
    const int rc = exclusive_scan_u64((uint64_t *)count, L, partial, s);
    if (rc != IDX_OK) return rc;
    hipLaunchKernelGGL((k_leaf_init<K, AOS>), dim3(grid_for(L, 256)), dim3(256), 0, s, keys,
                       (const unsigned long long *)count, L, leaves);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

// Bytes of the leaf counters and scan partials for L leaves.
size_t layout_scratch_bytes(uint32_t L) {
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    return up256(((size_t)L + 1) * 8) + up256(scan_partials_for(L) * 8);
}

template <typename K, bool AOS>
int train_t(idx_index *h, uint32_t L, uint32_t epochs, uint32_t feature, hipStream_t s) {
    const uint64_t n = h->n;
    const Load<K, AOS> keys = make_load<K, AOS>(h);
    LearnedModel *M = h->learned;
    const bool want_lin = feature != IDX_FEATURE_SPLINE, want_sp = feature == IDX_FEATURE_AUTO ||
                                                                   feature == IDX_FEATURE_SPLINE;
    const bool both = want_lin && want_sp;
    // device scratch: root record, root acc, leaf acc, stats, counts and scan
    // partials, and (both root families) a second leaf table; every region
    // starts on a 256-byte boundary (FP64 atomics need 8-byte alignment)
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t leaf_acc_b = up256((size_t)L * NACC * sizeof(double));
    const size_t alt_b = both ? up256((size_t)L * sizeof(LeafRec)) : 0;
    char *tmp = (char *)h->alloc.get(256 + 256 + leaf_acc_b + 256 + layout_scratch_bytes(L) + alt_b, s);
    if (!tmp) return IDX_ERR_NOMEM;
    RootRec *d_root = (RootRec *)tmp;
    double *root_acc = (double *)(tmp + 256);
    double *leaf_acc = (double *)(tmp + 512);
    double *stats = (double *)(tmp + 512 + leaf_acc_b);
    unsigned long long *count = (unsigned long long *)(tmp + 512 + leaf_acc_b + 256);
    uint64_t *partial = (uint64_t *)((char *)count + up256(((size_t)L + 1) * 8));
    LeafRec *alt = both ? (LeafRec *)(tmp + 512 + leaf_acc_b + 256 + layout_scratch_bytes(L)) : nullptr;
    uint32_t *d_big = (uint32_t *)(stats + 8);  // a leaf larger than kLeafCap exists
    const uint32_t rblocks = (uint32_t)((n + LT * 8 - 1) / (LT * 8)) > 2048 ? 2048u
                                                                             : (uint32_t)((n + LT * 8 - 1) / (LT * 8));
    const uint32_t cblocks = grid_for((n + CHUNK - 1) / CHUNK, LT);

    // One root candidate: place R on the device (a spline candidate also gets
    // its geometry and bins), take `ep_n` Newton steps, measure the loss.
    auto candidate = [&](RootRec R, uint32_t ep_n, RootRec &out, double &loss) -> int {
        if (hipMemcpyAsync(d_root, &R, sizeof(R), hipMemcpyHostToDevice, s) != hipSuccess) return IDX_ERR_HIP;
        if (R.mode == IDX_FEATURE_SPLINE) {
            hipLaunchKernelGGL((k_spline_geometry<K, AOS>), dim3(1), dim3(64), 0, s, keys, n, d_root);
            hipLaunchKernelGGL((k_spline_bins<K, AOS>), dim3(grid_for(spline_bins(n), 256)), dim3(256), 0, s, keys, n,
                               d_root, M->spline);
        }
        for (uint32_t ep = 0; ep <= ep_n; ++ep) {
            hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, root_acc, (uint64_t)NACC);
            hipLaunchKernelGGL((k_root_accum<K, AOS>), dim3(rblocks ? rblocks : 1), dim3(LT), 0, s, keys, n, d_root,
                               root_acc);
            if (ep < ep_n) hipLaunchKernelGGL(k_root_update, dim3(1), dim3(64), 0, s, d_root, root_acc);
        }
        double acc[NACC];
        if (hipMemcpyAsync(acc, root_acc, sizeof(acc), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&out, d_root, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return IDX_ERR_HIP;
        loss = acc[5];
        return IDX_OK;
    };
    const uint32_t cap = stage_cap(n, L);  // keys staged per workgroup of the per-leaf passes
    // Leaves under root R into `leaves`: layout, Newton steps, error bounds;
    // st = {sum of window * size, max window, leaf loss}.
    auto leaves_for = [&](const RootRec &R, LeafRec *leaves, double st[4]) -> int {
        if (hipMemcpyAsync(d_root, &R, sizeof(R), hipMemcpyHostToDevice, s) != hipSuccess) return IDX_ERR_HIP;
        int rc = leaf_layout<K, AOS>(keys, n, d_root, L, count, partial, leaves, s);
        if (rc != IDX_OK) return rc;
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, d_big, (uint64_t)1, 0u);
        for (uint32_t ep = 0; ep < epochs; ++ep) {
            hipLaunchKernelGGL((k_leaf_accum_small<K, AOS, true>), dim3(grid_for(L, kLeafBlock)), dim3(kLeafBlock),
                               (size_t)cap * sizeof(K), s, keys, leaves, L, leaf_acc, d_big, cap);
            hipLaunchKernelGGL((k_leaf_accum_big<K, AOS>), dim3(cblocks), dim3(LT), 0, s, keys, n, d_root, leaves,
                               leaf_acc, d_big);
            hipLaunchKernelGGL(k_leaf_update_big, dim3(grid_for(L, 256)), dim3(256), 0, s, leaves, leaf_acc, L, d_big);
        }
        // the final leaf loss comes with the error bounds (same walk)
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, stats, (uint64_t)4);
        hipLaunchKernelGGL((k_leaf_errors_small<K, AOS>), dim3(grid_for(L, kLeafBlock)), dim3(kLeafBlock),
                           (size_t)cap * sizeof(K), s, keys, leaves, L, leaf_acc, cap);
        hipLaunchKernelGGL((k_leaf_errors_big<K, AOS>), dim3(cblocks), dim3(LT), 0, s, keys, n, d_root, leaves, d_big,
                           stats + 2);
        hipLaunchKernelGGL(k_leaf_finish, dim3(grid_for(L, 256) < 1024 ? grid_for(L, 256) : 1024), dim3(256), 0, s,
                           leaves, L, leaf_acc, stats);
        if (hipGetLastError() != hipSuccess) return IDX_ERR_HIP;
        if (hipMemcpyAsync(st, stats, 4 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return IDX_ERR_HIP;
        return IDX_OK;
    };

    int rc = IDX_OK;
    do {
        // ---- stage 1: roots.  A linear root takes `epochs` Newton steps over
        // either key feature; a spline root is built from the keys' ranks over
        // either bin feature.  Within each family the lower loss wins.
        RootRec best_lin{}, best_sp{};
        double loss_lin = -1.0, loss_sp = -1.0;
        for (uint32_t f = IDX_FEATURE_LINEAR; f <= IDX_FEATURE_LOG && rc == IDX_OK; ++f) {
            RootRec R{}, got;
            double loss;
            R.L = L;
            if (want_lin && (feature == IDX_FEATURE_AUTO || feature == f)) {
                R.mode = f;
                if ((rc = candidate(R, epochs, got, loss)) != IDX_OK) break;
                if (loss_lin < 0 || loss < loss_lin) { loss_lin = loss; best_lin = got; }
            }
            if (want_sp) {
                R.mode = IDX_FEATURE_SPLINE;
                R.bins = M->spline;
                R.bfeat = f;
                if ((rc = candidate(R, 0, got, loss)) != IDX_OK) break;
                if (loss_sp < 0 || loss < loss_sp) { loss_sp = loss; best_sp = got; }
            }
        }
        if (rc != IDX_OK) break;
        if (want_sp && best_sp.bfeat != IDX_FEATURE_LOG) {  // the table holds the last bins built: rebuild the winner
            if (hipMemcpyAsync(d_root, &best_sp, sizeof(best_sp), hipMemcpyHostToDevice, s) != hipSuccess) {
                rc = IDX_ERR_HIP;
                break;
            }
            hipLaunchKernelGGL((k_spline_bins<K, AOS>), dim3(grid_for(spline_bins(n), 256)), dim3(256), 0, s, keys, n,
                               d_root, M->spline);
        }

        // ---- stage 2: leaves under each family's root; with both, the lower
        // estimated lookup cost wins
        double st[4], st2[4];
        bool sp = !want_lin;
        if ((rc = leaves_for(want_lin ? best_lin : best_sp, M->leaves, st)) != IDX_OK) break;
        if (both) {
            if ((rc = leaves_for(best_sp, alt, st2)) != IDX_OK) break;
            if (window_cost(st2[0] / (double)n, true) < window_cost(st[0] / (double)n, false)) {
                sp = true;
                for (int j = 0; j < 4; ++j) st[j] = st2[j];
                if (hipMemcpyAsync(M->leaves, alt, (size_t)L * sizeof(LeafRec), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    rc = IDX_ERR_HIP;
                    break;
                }
            }
        }
        M->root = sp ? best_sp : best_lin;
        M->stats.root_loss = sp ? loss_sp : loss_lin;
        M->stats.leaf_loss = st[2];
        M->stats.mean_window = n ? st[0] / (double)n : 0.0;
        M->stats.max_window = st[1];
    } while (0);
    h->alloc.put(tmp, s);
    return rc;
}

}  // namespace

int learn(idx_index *h, uint32_t L, uint32_t epochs, uint32_t feature, hipStream_t s) {
    if (h->layout != IDX_BS || h->n == 0) return IDX_ERR_ARG;
    if (L == 0 || L > (1u << 26) || epochs == 0 || epochs > 16 || feature > IDX_FEATURE_SPLINE) return IDX_ERR_ARG;
    drop_model(h, s, h->params.leaf_lines == 1);
    LearnedModel *M = new (std::nothrow) LearnedModel();
    if (!M) return IDX_ERR_NOMEM;
    M->leaves = (LeafRec *)h->alloc.get((size_t)L * sizeof(LeafRec), s);
    if (M->leaves && (feature == IDX_FEATURE_AUTO || feature == IDX_FEATURE_SPLINE)) {
        M->spline = (SplineBin *)h->alloc.get((size_t)spline_bins(h->n) * sizeof(SplineBin), s);
        if (!M->spline) {
            h->alloc.put(M->leaves, s);
            M->leaves = nullptr;
        }
    }
    if (!M->leaves) {
        delete M;
        return IDX_ERR_NOMEM;
    }
    h->learned = M;
    M->stats.leaves = L;
    M->stats.epochs = epochs;
    int rc;
    if (h->u64) rc = h->aos ? train_t<uint64_t, true>(h, L, epochs, feature, s) : train_t<uint64_t, false>(h, L, epochs, feature, s);
    else rc = h->aos ? train_t<uint32_t, true>(h, L, epochs, feature, s) : train_t<uint32_t, false>(h, L, epochs, feature, s);
    if (rc != IDX_OK) {
        drop_model(h, s);
        return rc;
    }
    M->stats.feature = M->root.mode;
    M->stats.root_a0 = M->root.a0;
    M->stats.root_a1 = M->root.a1;
    M->stats.segments = M->root.mode == IDX_FEATURE_SPLINE ? M->root.nb : 0;
    M->stats.bin_feature = M->root.mode == IDX_FEATURE_SPLINE ? M->root.bfeat : 0;
    if (M->root.mode != IDX_FEATURE_SPLINE && M->spline) {
        h->alloc.put(M->spline, s);
        M->spline = nullptr;
    }
    if (h->params.leaf_lines == 1) {
        rc = ensure_lines(h, s);
        if (rc == IDX_OK && hipStreamSynchronize(s) != hipSuccess) rc = IDX_ERR_HIP;
        if (rc != IDX_OK) {
            drop_model(h, s);
            return rc;
        }
    }
    return IDX_OK;
}

void drop_model(idx_index *h, hipStream_t s, bool keep_lines) {
    void *lines = h->learned ? h->learned->lines : nullptr;
    if (h->spare_lines && (!keep_lines || lines)) {
        h->alloc.put(h->spare_lines, s);
        h->spare_lines = nullptr;
        h->spare_lines_bytes = 0;
    }
    if (!h->learned) return;
    h->alloc.put(h->learned->leaves, s);
    if (h->learned->spline) h->alloc.put(h->learned->spline, s);
    if (lines && keep_lines) {
        h->spare_lines = lines;
        h->spare_lines_bytes = (size_t)h->learned->root.L * kLineBytes;
    } else if (lines) {
        h->alloc.put(lines, s);
    }
    delete h->learned;
    h->learned = nullptr;
}

int learn_stats(const idx_index *h, idx_learn_stats *out) {
    if (!h->learned) return IDX_ERR_ARG;
    *out = h->learned->stats;
    return IDX_OK;
}

int learn_export(const idx_index *h, void *leaves_out, hipStream_t s) {
    if (!h->learned) return IDX_ERR_ARG;
    if (!leaves_out) return IDX_OK;
    IDX_HIP(hipMemcpyAsync(leaves_out, h->learned->leaves, (size_t)h->learned->root.L * sizeof(LeafRec),
                           hipMemcpyDeviceToDevice, s));
    return IDX_OK;
}

// ---------------------------------------------------------------- lookups

namespace {

// Window scan on the array-of-structures sorted array (one key and its row
// ID per slot): keys of slots [b, b + len) (len <= W) below x, and the row ID
// of the first slot equal to x.  Slots are read with independent loads; the
// row ID comes with its key, so a hit costs no further line.  A 16-byte slot
// holding a 64-bit key is one 16-byte vector load.
template <typename K, int W>
__device__ __forceinline__ uint32_t count_below_slots(const Load<K, true> &L, uint64_t b, uint32_t len, K x,
                                                      bool &eq, uint32_t &row, bool two = true) {
    uint32_t cnt = 0;
    bool e = false;
    uint32_t rw = kMiss;
    if (sizeof(K) == 8 && L.stride == 16) {
        uint4 w[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
            if ((uint32_t)j < len) w[j] = *(const uint4 *)(L.base + (b + j) * 16);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if ((uint32_t)j >= len) continue;
            const K k = (K)(((uint64_t)w[j].y << 32) | w[j].x);
            cnt += k < x ? 1u : 0u;
            if (!e && k == x) {
                e = true;
                rw = w[j].z;
            }
        }
    } else {
        // Two rounds: first the slots whose key lies in the 128-byte line of
        // the window's first key; the rest only when all of those are below x
        // (keys ascend, so otherwise the lower bound is already among them).
        // A window within one line costs that line alone.
        K k[W];
        bool got[W];
        const uint64_t line0 = (uint64_t)(uintptr_t)(L.base + b * (uint64_t)L.stride) >> 7;
        uint32_t n1 = 0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint64_t a = (uint64_t)(uintptr_t)(L.base + (b + j) * (uint64_t)L.stride);
            got[j] = (uint32_t)j < len && (!two || ((a + sizeof(K) - 1) >> 7) == line0);
            k[j] = got[j] ? L.key(b + j) : K(0);
            n1 += got[j] ? 1u : 0u;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) cnt += (got[j] && k[j] < x) ? 1u : 0u;
        if (two && cnt == n1 && n1 < len) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                if ((uint32_t)j >= len || got[j]) continue;
                k[j] = L.key(b + j);
                got[j] = true;
                cnt += k[j] < x ? 1u : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < W; ++j) e |= got[j] && k[j] == x;
        if (e) rw = L.row(b + cnt);
    }
    eq = e;
    row = rw;
    return cnt;
}

// Window scan on the packed array of structures (64-bit key and 32-bit row
// ID per 12-byte slot): the slots [b, b + len) (len <= W) are read as aligned
// 16-byte chunks, every chunk of a round issued at once, and keys and row IDs
// are taken from the registers, so a hit needs no further load.  (Loading the
// row ID after the keys were counted often found its line evicted from L2:
// with hundreds of thousands of lookups in flight per XCD a line does not
// stay there long.)  Two rounds as in count_below_slots: first the chunks of
// the 128-byte line of the window's first chunk, the rest only when every
// slot read so far is below x.  A slot starts at word S + 3 j of the chunks,
// S = (12 b mod 16) / 4 differing from lane to lane: the loads do not depend
// on S (so no lane waits for another's), and each word is selected from the
// four candidates by S after they arrive.
template <int W>
__device__ __forceinline__ uint32_t count_below_packed(const char *__restrict__ base, uint64_t b, uint32_t len,
                                                       uint64_t x, bool &eq, uint32_t &row, bool two) {
    constexpr int NC = (3 * 4 + W * 12 + 15) / 16;  // chunks covering W slots from any word S <= 3
    const char *p0 = base + ((b * 12) & ~(uint64_t)15);
    const uint32_t S = (uint32_t)((b * 12) & 15) >> 2;
    const uint64_t line0 = (uint64_t)(uintptr_t)p0 >> 7;
    const uint32_t end_word = S + 3 * len;  // words [S, end_word) hold the window
    uint4 w[NC];
    uint32_t got = 0;  // bit c: chunk c loaded
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const bool need = (uint32_t)(4 * c) < end_word;
        const bool first = !two || ((uint64_t)(uintptr_t)(p0 + 16 * c) >> 7) == line0;
        w[c] = make_uint4(0u, 0u, 0u, 0u);
        if (need && first) {
            w[c] = *(const uint4 *)(p0 + 16 * c);
            got |= 1u << c;
        }
    }
    auto word = [&](int i) -> uint32_t {  // static i
        const uint4 &v = w[i >> 2];
        return (i & 3) == 0 ? v.x : (i & 3) == 1 ? v.y : (i & 3) == 2 ? v.z : v.w;
    };
    auto pick = [&](int i) -> uint32_t {  // word S + i
        const uint32_t a = word(i), bb = word(i + 1), c = word(i + 2), d = word(i + 3);
        return S == 0 ? a : S == 1 ? bb : S == 2 ? c : d;
    };
    auto slot_in = [&](int j) -> bool {  // all three words of slot j loaded
        const uint32_t k0 = S + 3 * (uint32_t)j;
        return ((got >> (k0 >> 2)) & 1u) && ((got >> ((k0 + 2) >> 2)) & 1u);
    };
    uint32_t cnt = 0, avail = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const bool in = (uint32_t)j < len && slot_in(j);
        const uint64_t k = ((uint64_t)pick(3 * j + 1) << 32) | pick(3 * j);
        avail += in ? 1u : 0u;
        cnt += (in && k < x) ? 1u : 0u;
    }
    if (two && cnt == avail && avail < len) {
        // every slot read is below x: the lower bound lies further on
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (!((got >> c) & 1u) && (uint32_t)(4 * c) < end_word) {
                w[c] = *(const uint4 *)(p0 + 16 * c);
                got |= 1u << c;
            }
        cnt = 0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint64_t k = ((uint64_t)pick(3 * j + 1) << 32) | pick(3 * j);
            cnt += ((uint32_t)j < len && k < x) ? 1u : 0u;
        }
    }
    // the lower bound is slot cnt: a hit when its key equals x
    bool e = false;
    uint32_t rw = kMiss;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const uint64_t k = ((uint64_t)pick(3 * j + 1) << 32) | pick(3 * j);
        if ((uint32_t)j == cnt && (uint32_t)j < len && slot_in(j) && k == x) {
            e = true;
            rw = pick(3 * j + 2);
        }
    }
    eq = e;
    row = rw;
    return cnt;
}

// Windows are narrowed with binary-search steps down to STOP keys: 15 on the
// structure-of-arrays layout (its scan reads 16 keys in 9 vector loads), 7
// on the array of structures (8 slots, each with its row ID).
template <bool AOS>
constexpr uint32_t window_stop() {
    return AOS ? 7u : 15u;
}

template <typename K, int R, bool SORT, bool AOS, bool TWO>
__global__ __launch_bounds__(1024) void k_point_learned(Load<K, AOS> keys, uint64_t n, RootRec root,
                                                        const LeafRec *__restrict__ leaves, QueryIO<K> io) {
    extern __shared__ __align__(16) char smem[];
    constexpr uint32_t STOP = window_stop<AOS>();
    const uint64_t tile = (uint64_t)blockDim.x * R;
    for (uint64_t it = blockIdx.x; it < io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, io.ntiles, io.xcd);
        if (tl >= io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R];
        uint32_t src[R];
        uint32_t b[R], len[R];  // ranks: n < 2^32
        tile_load<K, R, SORT>(io, smem, t0, x, src);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint64_t w0, wl;
            learned_window(root, leaves, (uint64_t)x[r], w0, wl);
            b[r] = (uint32_t)w0;
            len[r] = tile_valid(io.m, t0, src_of<R, SORT>(src, r)) ? (uint32_t)wl : 0u;
        }
        // The lower bound lies in [b, b + len].  Narrow wide windows with
        // binary-search steps, then read the last <= STOP keys and the key
        // after them in one round of independent loads.
        bool more = true;
        while (more) {
            more = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (len[r] > STOP) {
                    const uint32_t half = len[r] >> 1;
                    b[r] = keys.key(b[r] + half - 1) < x[r] ? b[r] + half : b[r];
                    len[r] -= half;
                    more |= len[r] > STOP;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t res = kMiss;
            if (tile_valid(io.m, t0, src_of<R, SORT>(src, r))) {
                const uint64_t sl = ((uint64_t)len[r] + 1) < (n - b[r]) ? ((uint64_t)len[r] + 1) : (n - b[r]);
                bool eq;
                if constexpr (AOS) {
                    uint32_t row;
                    if (sizeof(K) == 8 && keys.stride == 12)
                        (void)count_below_packed<STOP + 1>(keys.base, b[r], (uint32_t)sl, (uint64_t)x[r], eq, row, TWO);
                    else
                        (void)count_below_slots<K, STOP + 1>(keys, b[r], (uint32_t)sl, x[r], eq, row, TWO);
                    if (eq) res = row;
                } else {
                    const uint32_t c = count_below<K, 16>(keys.k, b[r], (uint32_t)sl, x[r], eq, TWO);
                    if (eq) res = keys.r[(uint64_t)b[r] + c];
                }
            }
            tile_put<K, SORT>(io, smem, t0, src_of<R, SORT>(src, r), res);
        }
        tile_flush<K, R, SORT>(io, smem, t0);
    }
}

// ------------------------------------------------------------- leaf lines

// The leaf lines (line layout at line_scan), one thread per 16-byte chunk,
// so that a wave writes eight whole lines.  A workgroup writes kLinesGroups
// groups of 32 leaves in turn; a group's leaves cover one contiguous rank
// range, and when it is short enough its keys and row IDs are first copied
// to LDS with consecutive loads.
constexpr uint32_t kLinesBlock = 256;                         // threads: 32 leaves x 8 chunks
constexpr uint32_t kLinesStage = 1024;                        // keys staged per group at most
constexpr uint32_t kLinesGroups = 8;  // groups of 32 leaves per workgroup (fewer workgroups to dispatch)
template <typename K, bool AOS>
__global__ __launch_bounds__(kLinesBlock) void k_leaf_lines(Load<K, AOS> keys, const LeafRec *__restrict__ leaves,
                                                            uint32_t L, uint4 *__restrict__ lines) {
    __shared__ K s_key[kLinesStage];
    __shared__ uint32_t s_row[kLinesStage];
    constexpr uint32_t GL = kLinesBlock / kLineChunks;  // leaves per group
    for (uint32_t gi = 0; gi < kLinesGroups; ++gi) {
        const uint64_t l0 = ((uint64_t)blockIdx.x * kLinesGroups + gi) * GL;
        if (l0 >= L) return;  // workgroup-uniform
        const uint64_t l1 = l0 + GL < L ? l0 + GL : L;
        const uint64_t kb = leaves[l0].base, ke = (uint64_t)leaves[l1 - 1].base + leaves[l1 - 1].size;
        const bool staged = ke - kb <= kLinesStage;  // workgroup-uniform
        if (staged) {
            for (uint64_t i = kb + threadIdx.x; i < ke; i += kLinesBlock) {
                s_key[i - kb] = keys.key(i);
                s_row[i - kb] = keys.row(i);
            }
            __syncthreads();
        }
        const uint64_t t = l0 * kLineChunks + threadIdx.x;
        if (t < (uint64_t)L * kLineChunks) {
            const uint32_t l = (uint32_t)(t / kLineChunks), c = (uint32_t)(t % kLineChunks);
            const LeafRec r = leaves[l];
            auto key_at = [&](uint64_t i) -> uint64_t {
                return staged ? (uint64_t)s_key[i - kb] : (uint64_t)keys.key(i);
            };
            auto row_at = [&](uint64_t i) -> uint32_t { return staged ? s_row[i - kb] : keys.row(i); };
            constexpr uint32_t C = line_slots<K>();
            constexpr uint32_t KW = sizeof(K) / 4;  // words per key
            uint32_t v[4];
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) {
                const uint32_t wi = 4 * c + i;
                uint32_t x = 0;
                if (wi == 0) {
                    x = r.base;
                } else if (wi == 1) {
                    x = r.size;
                } else if (wi < 2 + C * KW) {
                    const uint32_t j = (wi - 2) / KW;
                    if (j < r.size) {
                        const uint64_t k = key_at((uint64_t)r.base + j);
                        x = (KW == 2 && ((wi - 2) & 1u)) ? (uint32_t)(k >> 32) : (uint32_t)k;
                    }
                } else {
                    const uint32_t j = wi - 2 - C * KW;
                    if (j < r.size) x = row_at((uint64_t)r.base + j);
                }
                v[i] = x;
            }
            lines[t] = make_uint4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();  // the next group restages
    }
}

// Answer for x in the window [b, b + len] of the sorted array: halved while
// it spans more than the scan's width, then the short-window scan.
template <typename K, bool AOS>
__device__ __forceinline__ uint32_t window_find(const Load<K, AOS> &keys, uint64_t n, uint64_t b, uint64_t len, K x,
                                                bool two) {
    constexpr uint32_t STOP = window_stop<AOS>();
    while (len > STOP) {
        const uint64_t half = len >> 1;
        b = keys.key(b + half - 1) < x ? b + half : b;
        len -= half;
    }
    const uint64_t sl = (len + 1) < (n - b) ? (len + 1) : (n - b);
    bool eq;
    if constexpr (AOS) {
        uint32_t row;
        if (sizeof(K) == 8 && keys.stride == 12)
            (void)count_below_packed<STOP + 1>(keys.base, b, (uint32_t)sl, (uint64_t)x, eq, row, two);
        else
            (void)count_below_slots<K, STOP + 1>(keys, b, (uint32_t)sl, x, eq, row, two);
        return eq ? row : kMiss;
    } else {
        const uint32_t c = count_below<K, 16>(keys.k, b, (uint32_t)sl, x, eq, two);
        return eq ? keys.r[b + c] : kMiss;
    }
}

// The same, kept out of line: called only for the few lookups that go past
// their leaf's line, so the callers' loops over their lookups stay small
// enough to unroll.
template <typename K, bool AOS>
__device__ __noinline__ uint32_t window_find_call(Load<K, AOS> keys, uint64_t n, uint64_t b, uint64_t len, K x,
                                                  bool two) {
    return window_find<K, AOS>(keys, n, b, len, x, two);
}

// Point lookups through the leaf lines, one lane per lookup (the sorted-tile
// form): the R lookups of a lane load their leaves' lines together (eight
// independent 16-byte loads of one line each), then each is answered from
// its registers; a lookup past every key of its line in a larger leaf
// searches the rest of that leaf in the sorted array.
template <typename K, int R, bool SORT, bool AOS, bool TWO>
__global__ __launch_bounds__(256) void k_point_lines(Load<K, AOS> keys, uint64_t n, RootRec root,
                                                     const uint4 *__restrict__ lines, QueryIO<K> io) {
    extern __shared__ __align__(16) char smem[];
    const uint64_t tile = (uint64_t)blockDim.x * R;
    for (uint64_t it = blockIdx.x; it < io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, io.ntiles, io.xcd);
        if (tl >= io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R];
        uint32_t src[R];
        tile_load<K, R, SORT>(io, smem, t0, x, src);
        uint4 w[R][kLineChunks];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool v = tile_valid(io.m, t0, src_of<R, SORT>(src, r));
            const uint4 *p = lines + (uint64_t)leaf_of(root, (uint64_t)x[r]) * kLineChunks;
#pragma unroll
            for (int c = 0; c < (int)kLineChunks; ++c) w[r][c] = v ? p[c] : make_uint4(0u, 0u, 0u, 0u);
        }
        // answers from the lines first, so that no line is held while the
        // rest of a larger leaf is searched
        uint32_t res[R];
        uint64_t b[R], len[R];
        bool big[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            res[r] = kMiss;
            big[r] = false;
            b[r] = len[r] = 0;
            if (tile_valid(io.m, t0, src_of<R, SORT>(src, r))) {
                uint32_t cnt, row;
                bool eq;
                if (line_scan<K>(w[r], x[r], cnt, eq, row, b[r], len[r])) {
                    if (eq) res[r] = row;
                } else {
                    big[r] = true;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (big[r]) res[r] = window_find_call<K, AOS>(keys, n, b[r], len[r], x[r], TWO);
            tile_put<K, SORT>(io, smem, t0, src_of<R, SORT>(src, r), res[r]);
        }
        tile_flush<K, R, SORT>(io, smem, t0);
    }
}

// Point lookups through the leaf lines, two lanes per lookup: lane h of a
// pair loads the line's half h (four 16-byte loads).  A lane reading a whole
// line with eight loads makes the memory system serve far fewer random lines
// per second than lanes sharing it (measured on MI355X: 13 against 48 G
// lines/s).  Each lane counts its half's keys below x and at most x; the pair
// adds both counts with one exchange each, and a hit is a key equal to x
// (more keys at most x than below it).  The row IDs lie in the upper half, so
// its lane writes the answer; when x lies past every key of the line in a
// leaf that has more, the lower lane searches the rest of the leaf in the
// sorted array and writes.
template <typename K, int R, bool AOS, bool TWO>
__global__ __launch_bounds__(256) void k_point_lines_pair(Load<K, AOS> keys, uint64_t n, RootRec root,
                                                          const uint4 *__restrict__ lines, QueryIO<K> io) {
    constexpr uint32_t C = line_slots<K>();
    constexpr uint32_t KW = sizeof(K) / 4;  // words per key
    constexpr uint32_t R0 = 2 + C * KW;     // first row ID word (>= 16: in the upper half)
    static_assert(R0 >= 16, "row IDs in the upper half of the line");
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = blockDim.x / 2, pi = threadIdx.x / 2;
    const uint64_t tile = pairs * R;
    for (uint64_t it = blockIdx.x; it < io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, io.ntiles, io.xcd);
        if (tl >= io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R];
        bool v[R];
        uint4 w[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t qi = t0 + (uint64_t)r * pairs + pi;
            v[r] = qi < io.m;
            x[r] = v[r] ? io.q[qi] : K(0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint4 *p = lines + (uint64_t)leaf_of(root, (uint64_t)x[r]) * kLineChunks + 4 * hf;
#pragma unroll
            for (int c = 0; c < 4; ++c) w[r][c] = v[r] ? p[c] : make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t res[R];
        uint64_t b[R], len[R];
        bool big[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            auto word = [&](int i) -> uint32_t {  // static i: word 16 hf + i of the line
                const uint4 &c = w[r][i >> 2];
                return (i & 3) == 0 ? c.x : (i & 3) == 1 ? c.y : (i & 3) == 2 ? c.z : c.w;
            };
            res[r] = kMiss;
            b[r] = len[r] = 0;
            const uint32_t other = __shfl_xor(w[r][0].y, 1);
            const uint32_t size = hf ? other : w[r][0].y;
            uint32_t lt = 0, le = 0;
#pragma unroll
            for (int i = 0; i < 16; i += (int)KW) {
                const uint32_t wi = 16 * hf + (uint32_t)i;
                K key;
                if constexpr (KW == 2) key = ((uint64_t)word(i + 1) << 32) | word(i);
                else key = word(i);
                const bool in = wi >= 2 && wi < R0 && (wi - 2) / KW < size;
                lt += (in && key < x[r]) ? 1u : 0u;
                le += (in && key <= x[r]) ? 1u : 0u;
            }
            lt += __shfl_xor(lt, 1);
            le += __shfl_xor(le, 1);
            // past every key of the line in a leaf that has more: the rest
            // of the leaf is searched in the sorted array (by the lower lane)
            big[r] = lt == C && size > C;
            if (!big[r]) {
                if (le > lt) {
                    const uint32_t ri = R0 - 16 + lt;  // the row ID's word in the upper half
                    uint32_t row = 0;
#pragma unroll
                    for (int i = 0; i < 16; ++i) row = (uint32_t)i == ri ? word(i) : row;
                    res[r] = row;
                }
            } else if (hf == 0) {
                b[r] = (uint64_t)w[r][0].x + C;
                len[r] = size - C;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t qi = t0 + (uint64_t)r * pairs + pi;
            if (big[r] && hf == 0) res[r] = window_find_call<K, AOS>(keys, n, b[r], len[r], x[r], TWO);
            if (v[r] && hf == (big[r] ? 0u : 1u)) io.out[io.pos ? io.pos[qi] : qi] = res[r];
        }
    }
}

}  // namespace

// Write the model's leaf lines unless they are there.
int ensure_lines(idx_index *h, hipStream_t s) {
    LearnedModel *M = h->learned;
    if (M->lines) return IDX_OK;
    const uint32_t L = M->root.L;
    const size_t bytes = (size_t)L * kLineBytes;
    uint4 *lines = nullptr;
    if (h->spare_lines && h->spare_lines_bytes == bytes) {
        lines = (uint4 *)h->spare_lines;  // every line is rewritten below
    } else {
        if (h->spare_lines) h->alloc.put(h->spare_lines, s);
        lines = (uint4 *)h->alloc.get(bytes, s);
    }
    h->spare_lines = nullptr;
    h->spare_lines_bytes = 0;
    if (!lines) return IDX_ERR_NOMEM;
    const uint64_t groups = ((uint64_t)L + kLinesBlock / kLineChunks - 1) / (kLinesBlock / kLineChunks);
    const uint32_t g = (uint32_t)((groups + kLinesGroups - 1) / kLinesGroups);
    if (h->u64) {
        if (h->aos) hipLaunchKernelGGL((k_leaf_lines<uint64_t, true>), dim3(g), dim3(256), 0, s, make_load<uint64_t, true>(h), M->leaves, L, lines);
        else hipLaunchKernelGGL((k_leaf_lines<uint64_t, false>), dim3(g), dim3(256), 0, s, make_load<uint64_t, false>(h), M->leaves, L, lines);
    } else {
        if (h->aos) hipLaunchKernelGGL((k_leaf_lines<uint32_t, true>), dim3(g), dim3(256), 0, s, make_load<uint32_t, true>(h), M->leaves, L, lines);
        else hipLaunchKernelGGL((k_leaf_lines<uint32_t, false>), dim3(g), dim3(256), 0, s, make_load<uint32_t, false>(h), M->leaves, L, lines);
    }
    if (hipGetLastError() != hipSuccess) {
        h->alloc.put(lines, s);
        return IDX_ERR_HIP;
    }
    M->lines = lines;
    return IDX_OK;
}

namespace {
// Query IO of a leaf-line launch over tiles of `tile` lookups, and its grid.
template <typename KT>
QueryIO<KT> lines_io(const idx_index *h, const PointIO &pio, uint64_t tile, uint32_t &grid) {
    QueryIO<KT> io{};
    io.q = (const KT *)pio.q;
    io.out = pio.out;
    io.m = pio.m;
    io.local_sort = pio.local_sort ? 1u : 0u;
    io.xcd = pio.xcd ? 1u : 0u;
    io.sort_off = 0;
    io.rounds = h->params.window_rounds == 1 ? 1u : 2u;
    io.pos = pio.pos;
    set_tiles(io, tile);
    uint64_t g = io.iters;
    if (h->params.persistent) {
        uint64_t cap = (uint64_t)h->cu_count * h->params.persistent;
        if (io.xcd && cap >= kXcds) cap -= cap % kXcds;
        if (g > cap) g = cap;
    }
    grid = (uint32_t)(g ? (g > 0x7FFFFFFFull ? 0x7FFFFFFFull : g) : 1);
    return io;
}

template <typename KT, int RR>
void launch_lines(idx_index *h, const PointIO &pio, uint32_t block, hipStream_t s) {
    const LearnedModel *M = h->learned;
    uint32_t g;
    if (pio.local_sort) {  // one lane per lookup, at most 4 lookups per lane
        constexpr int RS = RR > 4 ? 4 : RR;
        const uint64_t tile = (uint64_t)block * RS;
        const QueryIO<KT> io = lines_io<KT>(h, pio, tile, g);
        const size_t smem = sort_lds_bytes((uint32_t)tile, sizeof(KT));
        if (h->aos && io.rounds == 2)
            hipLaunchKernelGGL((k_point_lines<KT, RS, true, true, true>), dim3(g), dim3(block), smem, s,
                               make_load<KT, true>(h), h->n, M->root, M->lines, io);
        else if (h->aos)
            hipLaunchKernelGGL((k_point_lines<KT, RS, true, true, false>), dim3(g), dim3(block), smem, s,
                               make_load<KT, true>(h), h->n, M->root, M->lines, io);
        else if (io.rounds == 2)
            hipLaunchKernelGGL((k_point_lines<KT, RS, true, false, true>), dim3(g), dim3(block), smem, s,
                               make_load<KT, false>(h), h->n, M->root, M->lines, io);
        else
            hipLaunchKernelGGL((k_point_lines<KT, RS, true, false, false>), dim3(g), dim3(block), smem, s,
                               make_load<KT, false>(h), h->n, M->root, M->lines, io);
        return;
    }
    const QueryIO<KT> io = lines_io<KT>(h, pio, (uint64_t)(block / 2) * RR, g);
    if (h->aos && io.rounds == 2)
        hipLaunchKernelGGL((k_point_lines_pair<KT, RR, true, true>), dim3(g), dim3(block), 0, s,
                           make_load<KT, true>(h), h->n, M->root, M->lines, io);
    else if (h->aos)
        hipLaunchKernelGGL((k_point_lines_pair<KT, RR, true, false>), dim3(g), dim3(block), 0, s,
                           make_load<KT, true>(h), h->n, M->root, M->lines, io);
    else if (io.rounds == 2)
        hipLaunchKernelGGL((k_point_lines_pair<KT, RR, false, true>), dim3(g), dim3(block), 0, s,
                           make_load<KT, false>(h), h->n, M->root, M->lines, io);
    else
        hipLaunchKernelGGL((k_point_lines_pair<KT, RR, false, false>), dim3(g), dim3(block), 0, s,
                           make_load<KT, false>(h), h->n, M->root, M->lines, io);
}

// Point lookups through the leaf lines: at most 256 threads per workgroup.
int point_lines(idx_index *h, const PointIO &pio, hipStream_t s) {
    const uint32_t block = h->params.block > 256 ? 256u : h->params.block;
    const uint32_t R = h->params.per_lane;
    if (h->u64) {
        switch (R) {
            case 1: launch_lines<uint64_t, 1>(h, pio, block, s); break;
            case 2: launch_lines<uint64_t, 2>(h, pio, block, s); break;
            case 4: launch_lines<uint64_t, 4>(h, pio, block, s); break;
            default: launch_lines<uint64_t, 8>(h, pio, block, s); break;
        }
    } else {
        switch (R) {
            case 1: launch_lines<uint32_t, 1>(h, pio, block, s); break;
            case 2: launch_lines<uint32_t, 2>(h, pio, block, s); break;
            case 4: launch_lines<uint32_t, 4>(h, pio, block, s); break;
            default: launch_lines<uint32_t, 8>(h, pio, block, s); break;
        }
    }
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

}  // namespace

int point_learned(idx_index *h, const PointIO &pio, hipStream_t s) {
    if (h->params.leaf_lines == 1) {
        const int rc = ensure_lines(h, s);
        return rc != IDX_OK ? rc : point_lines(h, pio, s);
    }
    const LearnedModel *M = h->learned;
    const uint32_t block = h->params.block;
    const uint32_t R = h->params.per_lane;
    const uint64_t tile = (uint64_t)block * R;
#define IDX_LEARNED_KERNELS(KT, RR, TW)                                                                     \
    do {                                                                                                    \
        if (h->aos && io.local_sort)                                                                        \
            hipLaunchKernelGGL((k_point_learned<KT, RR, true, true, TW>), dim3(g), dim3(block), smem, s,    \
                               make_load<KT, true>(h), h->n, M->root, M->leaves, io);                       \
        else if (h->aos)                                                                                    \
            hipLaunchKernelGGL((k_point_learned<KT, RR, false, true, TW>), dim3(g), dim3(block), smem, s,   \
                               make_load<KT, true>(h), h->n, M->root, M->leaves, io);                       \
        else if (io.local_sort)                                                                             \
            hipLaunchKernelGGL((k_point_learned<KT, RR, true, false, TW>), dim3(g), dim3(block), smem, s,   \
                               make_load<KT, false>(h), h->n, M->root, M->leaves, io);                      \
        else                                                                                                \
            hipLaunchKernelGGL((k_point_learned<KT, RR, false, false, TW>), dim3(g), dim3(block), smem, s,  \
                               make_load<KT, false>(h), h->n, M->root, M->leaves, io);                      \
    } while (0)
#define IDX_LEARNED_LAUNCH(KT, RR)                                                                          \
    do {                                                                                                    \
        QueryIO<KT> io{};                                                                                   \
        io.q = (const KT *)pio.q;                                                                           \
        io.out = pio.out;                                                                                   \
        io.m = pio.m;                                                                                       \
        io.local_sort = pio.local_sort ? 1u : 0u;                                                           \
        io.xcd = pio.xcd ? 1u : 0u;                                                                         \
        io.sort_off = 0;                                                                                    \
        io.rounds = h->params.window_rounds == 1 ? 1u : 2u;                                                 \
        io.pos = pio.pos;                                                                                   \
        set_tiles(io, tile);                                                                                \
        uint64_t grid = io.iters;                                                                           \
        if (h->params.persistent) {                                                                         \
            uint64_t cap = (uint64_t)h->cu_count * h->params.persistent;                                    \
            if (io.xcd && cap >= kXcds) cap -= cap % kXcds;                                                 \
            if (grid > cap) grid = cap;                                                                     \
        }                                                                                                   \
        const uint32_t g = (uint32_t)(grid ? (grid > 0x7FFFFFFFull ? 0x7FFFFFFFull : grid) : 1);            \
        const size_t smem = io.local_sort ? sort_lds_bytes((uint32_t)tile, sizeof(KT)) : 0;                 \
        if (io.rounds == 2) IDX_LEARNED_KERNELS(KT, RR, true);                                              \
        else IDX_LEARNED_KERNELS(KT, RR, false);                                                            \
    } while (0)
    if (h->u64) {
        switch (R) {
            case 1: IDX_LEARNED_LAUNCH(uint64_t, 1); break;
            case 2: IDX_LEARNED_LAUNCH(uint64_t, 2); break;
            case 4: IDX_LEARNED_LAUNCH(uint64_t, 4); break;
            default: IDX_LEARNED_LAUNCH(uint64_t, 8); break;
        }
    } else {
        switch (R) {
            case 1: IDX_LEARNED_LAUNCH(uint32_t, 1); break;
            case 2: IDX_LEARNED_LAUNCH(uint32_t, 2); break;
            case 4: IDX_LEARNED_LAUNCH(uint32_t, 4); break;
            default: IDX_LEARNED_LAUNCH(uint32_t, 8); break;
        }
    }
#undef IDX_LEARNED_LAUNCH
#undef IDX_LEARNED_KERNELS
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

namespace {
// Rank of the first key >= x through the model (the window holds it).
template <typename K, bool AOS>
__device__ __forceinline__ uint64_t model_lower_rank(const Load<K, AOS> &keys, uint64_t n, const RootRec &root,
                                                     const LeafRec *__restrict__ leaves, K x) {
    if constexpr (!AOS) {
        return learned_lower_rank(keys.k, n, root, leaves, x);
    } else {
        uint64_t b, len;
        learned_window(root, leaves, (uint64_t)x, b, len);
        while (len > window_stop<true>()) {
            const uint64_t half = len >> 1;
            b = keys.key(b + half - 1) < x ? b + half : b;
            len -= half;
        }
        bool eq;
        uint32_t row;
        return b + count_below_slots<K, window_stop<true>() + 1>(keys, b, (uint32_t)len, x, eq, row);
    }
}

template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_range_count_learned(Load<K, AOS> keys, uint64_t n, RootRec root,
                                                             const LeafRec *__restrict__ leaves,
                                                             const K *__restrict__ lo, const K *__restrict__ hi,
                                                             uint64_t m, uint32_t *__restrict__ first,
                                                             uint64_t *__restrict__ count) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const K L = lo[q], U = hi[q];
    uint64_t r0 = 0, r1 = 0;
    if (L <= U) {
        r0 = model_lower_rank(keys, n, root, leaves, L);
        r1 = (U == ~K(0)) ? n : model_lower_rank(keys, n, root, leaves, (K)(U + 1));
    }
    first[q] = (uint32_t)r0;
    count[q] = r1 > r0 ? r1 - r0 : 0;
}

// Lower-bound rank of x in the window [b, b + len] of the sorted array.
template <typename K, bool AOS>
__device__ __forceinline__ uint64_t window_lower_rank(const Load<K, AOS> &keys, uint64_t b, uint64_t len, K x) {
    constexpr uint32_t STOP = window_stop<AOS>();
    while (len > STOP) {
        const uint64_t half = len >> 1;
        b = keys.key(b + half - 1) < x ? b + half : b;
        len -= half;
    }
    bool eq;
    uint32_t row;
    if constexpr (AOS) return b + count_below_slots<K, STOP + 1>(keys, b, (uint32_t)len, x, eq, row);
    else return b + count_below<K, 16>(keys.k, b, (uint32_t)len, x, eq);
}

// Lower-bound rank of x from half hf of its leaf's line (w), as two lanes of
// a pair hold it (both call this together; the lower lane gets the rank):
// the base rank plus the line's keys below x, or, when x lies past every key
// of the line in a leaf that has more, a search of the rest of the leaf by
// the lower lane.
template <typename K, bool AOS>
__device__ __forceinline__ uint64_t pair_lower_rank(const Load<K, AOS> &keys, const uint4 (&w)[4], uint32_t hf, K x) {
    constexpr uint32_t C = line_slots<K>();
    constexpr uint32_t KW = sizeof(K) / 4;
    constexpr uint32_t R0 = 2 + C * KW;
    auto word = [&](int i) -> uint32_t {  // static i
        const uint4 &c = w[i >> 2];
        return (i & 3) == 0 ? c.x : (i & 3) == 1 ? c.y : (i & 3) == 2 ? c.z : c.w;
    };
    const uint32_t other = __shfl_xor(w[0].y, 1);
    const uint32_t size = hf ? other : w[0].y;
    uint32_t lt = 0;
#pragma unroll
    for (int i = 0; i < 16; i += (int)KW) {
        const uint32_t wi = 16 * hf + (uint32_t)i;
        K key;
        if constexpr (KW == 2) key = ((uint64_t)word(i + 1) << 32) | word(i);
        else key = word(i);
        lt += (wi >= 2 && wi < R0 && (wi - 2) / KW < size && key < x) ? 1u : 0u;
    }
    lt += __shfl_xor(lt, 1);
    if (lt < C || size <= C) return (uint64_t)w[0].x + lt;
    if (hf != 0) return 0;
    return window_lower_rank<K, AOS>(keys, (uint64_t)w[0].x + C, size - C, x);
}

// Range counts through the leaf lines, two lanes per range (each loads one
// half of both bounds' lines, all eight loads together); the lower lane
// writes the range's first rank and count.
template <typename K, bool AOS>
__global__ __launch_bounds__(256) void k_range_count_lines(Load<K, AOS> keys, uint64_t n, RootRec root,
                                                           const uint4 *__restrict__ lines, const K *__restrict__ lo,
                                                           const K *__restrict__ hi, uint64_t m,
                                                           uint32_t *__restrict__ first, uint64_t *__restrict__ count) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1;
    const bool live = q < m;  // the same for both lanes of a pair
    const K L = live ? lo[q] : K(0), U = live ? hi[q] : K(0);
    const bool act = live && L <= U, top = U == ~K(0);
    const K x1 = top ? U : (K)(U + 1);
    uint4 w0[4], w1[4];
    const uint4 *p0 = lines + (uint64_t)leaf_of(root, (uint64_t)L) * kLineChunks + 4 * hf;
    const uint4 *p1 = lines + (uint64_t)leaf_of(root, (uint64_t)x1) * kLineChunks + 4 * hf;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        w0[c] = act ? p0[c] : make_uint4(0u, 0u, 0u, 0u);
        w1[c] = act && !top ? p1[c] : make_uint4(0u, 0u, 0u, 0u);
    }
    const uint64_t r0 = pair_lower_rank<K, AOS>(keys, w0, hf, L);
    const uint64_t r1u = pair_lower_rank<K, AOS>(keys, w1, hf, x1);
    if (!live || hf != 0) return;
    const uint64_t r1 = !act ? 0 : top ? n : r1u;
    first[q] = act ? (uint32_t)r0 : 0u;
    count[q] = act && r1 > r0 ? r1 - r0 : 0;
}

template <typename K, bool AOS>
void launch_range_count(const idx_index *h, const void *lo, const void *hi, uint64_t m, uint32_t *first,
                        uint64_t *count, hipStream_t s) {
    const LearnedModel *M = h->learned;
    if (M->lines && h->params.leaf_lines == 1)
        hipLaunchKernelGGL((k_range_count_lines<K, AOS>), dim3(grid_for(2 * m, 256)), dim3(256), 0, s,
                           make_load<K, AOS>(h), h->n, M->root, M->lines, (const K *)lo, (const K *)hi, m, first,
                           count);
    else
        hipLaunchKernelGGL((k_range_count_learned<K, AOS>), dim3(grid_for(m, 256)), dim3(256), 0, s,
                           make_load<K, AOS>(h), h->n, M->root, M->leaves, (const K *)lo, (const K *)hi, m, first,
                           count);
}
}  // namespace

int range_count_learned(idx_index *h, const void *lo, const void *hi, uint64_t m, uint32_t *first, uint64_t *count,
                        bool may_alloc, hipStream_t s) {
    if (h->params.leaf_lines == 1 && may_alloc) {
        const int rc = ensure_lines(h, s);
        if (rc != IDX_OK) return rc;
    }
    if (h->u64) {
        if (h->aos) launch_range_count<uint64_t, true>(h, lo, hi, m, first, count, s);
        else launch_range_count<uint64_t, false>(h, lo, hi, m, first, count, s);
    } else {
        if (h->aos) launch_range_count<uint32_t, true>(h, lo, hi, m, first, count, s);
        else launch_range_count<uint32_t, false>(h, lo, hi, m, first, count, s);
    }
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

// ----------------------------------------------------- gradient evaluation

namespace {
// leaf parameters given as (b0, b1) pairs
__global__ void k_set_leaf_params(LeafRec *leaves, const float *ab, uint32_t L) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    leaves[l].b0 = ab[2 * l];
    leaves[l].b1 = ab[2 * l + 1];
}

template <typename K, bool AOS>
int eval_t(idx_index *h, uint32_t mode, const float *root_ab, uint32_t L, const float *leaf_ab, double *root_acc_h,
           double *leaf_acc_d, hipStream_t s) {
    const uint64_t n = h->n;
    const Load<K, AOS> keys = make_load<K, AOS>(h);
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t leaf_b = up256((size_t)L * sizeof(LeafRec));
    char *tmp = (char *)h->alloc.get(512 + leaf_b + layout_scratch_bytes(L), s);
    if (!tmp) return IDX_ERR_NOMEM;
    RootRec *d_root = (RootRec *)tmp;
    double *racc = (double *)(tmp + 256);
    LeafRec *leaves = (LeafRec *)(tmp + 512);
    unsigned long long *count = (unsigned long long *)(tmp + 512 + leaf_b);
    uint64_t *partial = (uint64_t *)((char *)count + up256(((size_t)L + 1) * 8));
    int rc = IDX_OK;
    do {
        RootRec R{root_ab[0], root_ab[1], mode, L};
        if (hipMemcpyAsync(d_root, &R, sizeof(R), hipMemcpyHostToDevice, s) != hipSuccess) { rc = IDX_ERR_HIP; break; }
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, racc, (uint64_t)NACC);
        const uint32_t rblocks = grid_for((n + LT * 8 - 1) / (LT * 8), 1) > 2048 ? 2048u
                                                                                : grid_for((n + LT * 8 - 1) / (LT * 8), 1);
        hipLaunchKernelGGL((k_root_accum<K, AOS>), dim3(rblocks), dim3(LT), 0, s, keys, n, d_root, racc);
        if (leaf_ab && leaf_acc_d) {
            const uint32_t cblocks = grid_for((n + CHUNK - 1) / CHUNK, LT);
            rc = leaf_layout<K, AOS>(keys, n, d_root, L, count, partial, leaves, s);
            if (rc != IDX_OK) break;
            uint32_t *d_big = (uint32_t *)(tmp + 256 + 128);
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, d_big, (uint64_t)1, 0u);
            hipLaunchKernelGGL(k_set_leaf_params, dim3(grid_for(L, 256)), dim3(256), 0, s, leaves, leaf_ab, L);
            const uint32_t cap = stage_cap(n, L);
            hipLaunchKernelGGL((k_leaf_accum_small<K, AOS>), dim3(grid_for(L, kLeafBlock)), dim3(kLeafBlock),
                               (size_t)cap * sizeof(K), s, keys, leaves, L, leaf_acc_d, d_big, cap);
            hipLaunchKernelGGL((k_leaf_accum_big<K, AOS>), dim3(cblocks), dim3(LT), 0, s, keys, n, d_root, leaves,
                               leaf_acc_d, d_big);
        }
        if (hipGetLastError() != hipSuccess) { rc = IDX_ERR_HIP; break; }
        if (hipMemcpyAsync(root_acc_h, racc, NACC * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = IDX_ERR_HIP; break; }
    } while (0);
    h->alloc.put(tmp, s);
    return rc;
}
}  // namespace

int learn_eval(idx_index *h, uint32_t mode, const float *root_ab, uint32_t L, const float *leaf_ab, double *root_acc,
               double *leaf_acc, hipStream_t s) {
    if (h->layout != IDX_BS || h->n == 0) return IDX_ERR_ARG;
    if (mode != IDX_FEATURE_LINEAR && mode != IDX_FEATURE_LOG) return IDX_ERR_ARG;
    if (L == 0 || L > (1u << 26) || !root_ab || !root_acc) return IDX_ERR_ARG;
    if (h->u64)
        return h->aos ? eval_t<uint64_t, true>(h, mode, root_ab, L, leaf_ab, root_acc, leaf_acc, s)
                      : eval_t<uint64_t, false>(h, mode, root_ab, L, leaf_ab, root_acc, leaf_acc, s);
    return h->aos ? eval_t<uint32_t, true>(h, mode, root_ab, L, leaf_ab, root_acc, leaf_acc, s)
                  : eval_t<uint32_t, false>(h, mode, root_ab, L, leaf_ab, root_acc, leaf_acc, s);
}

}  // namespace idx
