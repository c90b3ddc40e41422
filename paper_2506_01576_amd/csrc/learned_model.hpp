// The learned rank model's records and its evaluation, shared by the
// training/lookup kernels (learned.hip) and the batched launch (batch.hip).
#pragma once

#include "internal.hpp"
#include "search.hpp"

namespace idx {

struct RootRec {
    float a0, a1;           // linear roots: t = a1 * x + a0, leaf = clamp(floor(t), 0, L - 1)
    uint32_t mode;          // IDX_FEATURE_LINEAR / IDX_FEATURE_LOG / IDX_FEATURE_SPLINE
    uint32_t L;
    const uint64_t *knots;  // spline: G + 1 keys, the sorted keys at ranks floor(j (n - 1) / G)
    const float *scale;     // spline: per segment, its leaves per unit of key offset
    uint32_t G;             // spline: segments, a power of two
    uint32_t pad;
};
static_assert(sizeof(RootRec) == 40, "root record is 40 bytes");

struct __align__(16) LeafRec {
    uint64_t kmin;     // smallest build key of the leaf (0 when empty)
    uint32_t base;     // rank of kmin
    uint32_t size;     // keys in the leaf
    float b0, b1;      // local rank prediction b1 * f32(key - kmin) + b0
    int32_t elo, ehi;  // min / max of (true local rank - predicted local rank)
};
static_assert(sizeof(LeafRec) == 32, "leaf record is 32 bytes");

struct LearnedModel {
    RootRec root{};
    LeafRec *leaves = nullptr;  // device, L records
    void *spline = nullptr;     // device: G + 1 knot keys, then G scales (spline root only)
    idx_learn_stats stats{};
};

inline const LeafRec *model_leaves(const idx_index *h) { return h->learned->leaves; }
inline RootRec model_root(const idx_index *h) { return h->learned->root; }

// Monotone key feature in [0, 1].  LINEAR: the key itself; LOG: the bit
// pattern of the key rounded to FP32, read as an integer -- a piecewise
// linear approximation of log2(key).  Both use only correctly rounded
// conversions and power-of-two scalings.
__device__ __forceinline__ float key_feature(uint64_t key, uint32_t mode) {
    const float f = (float)key;
    if (mode == IDX_FEATURE_LINEAR) return f * 0x1p-64f;
    return (float)__float_as_uint(f) * 0x1p-31f;
}

// Spline segments for n keys and L leaves: the largest power of two G <= 4096
// with at least 64 keys and 8 leaves per segment (1 for tiny sets).
inline uint32_t spline_segments(uint64_t n, uint32_t L) {
    uint32_t G = 1;
    while (G < 4096 && (uint64_t)G * 2 * 64 <= n && (uint64_t)G * 2 * 8 <= L) G <<= 1;
    return G;
}

// Bytes of the G + 1 knot keys (256-byte aligned, the scales follow).
inline size_t spline_knot_bytes(uint32_t G) { return (((size_t)G + 1) * 8 + 255) & ~(size_t)255; }

// First leaf of spline segment j: segments share the L leaves as evenly as
// integers allow.
__host__ __device__ __forceinline__ uint32_t seg_leaf(uint32_t j, uint32_t L, uint32_t G) {
    return (uint32_t)(((uint64_t)j * L) / G);
}

// Spline root: the segment j of the last knot <= key gives leaves
// [seg_leaf(j), seg_leaf(j + 1)); inside it the leaf offset is
// f32(key - knot j) * scale[j], truncated (one rounding each).  Non-decreasing
// in the key, so each leaf's keys are one rank interval.
__device__ __forceinline__ uint32_t spline_leaf(const RootRec &R, uint64_t key, float *coord = nullptr) {
    const uint64_t *K = R.knots;
    if (key < K[0]) {
        if (coord) *coord = 0.f;
        return 0;
    }
    uint32_t j = 0;
    for (uint32_t h = R.G; h > 0; h >>= 1)
        if (j + h <= R.G && K[j + h] <= key) j += h;
    if (j >= R.G) {
        if (coord) *coord = (float)R.L;
        return R.L - 1;
    }
    const uint32_t f0 = seg_leaf(j, R.L, R.G), f1 = seg_leaf(j + 1, R.L, R.G);
    if (f1 == f0) {
        if (coord) *coord = (float)f0;
        return f0 < R.L ? f0 : R.L - 1;
    }
    const float f = __fmul_rn((float)(key - K[j]), R.scale[j]);
    const uint32_t span = f1 - f0;
    if (coord) *coord = __fadd_rn((float)f0, f < (float)span ? f : (float)span);
    return f0 + (f < (float)span ? (uint32_t)f : span - 1);
}

// Multiply, then add, each rounded on its own (no contraction), so the same
// key always lands in the same leaf wherever this is evaluated.
__device__ __forceinline__ uint32_t leaf_of(const RootRec &R, uint64_t key) {
    if (R.mode == IDX_FEATURE_SPLINE) return spline_leaf(R, key);
    const float x = key_feature(key, R.mode);
    const float t = __fadd_rn(__fmul_rn(R.a1, x), R.a0);
    if (!(t > 0.f)) return 0;
    if (t >= (float)R.L) return R.L - 1;
    return (uint32_t)t;
}

__device__ __forceinline__ float local_feature(const LeafRec &L, uint64_t key) {
    return (float)(key > L.kmin ? key - L.kmin : 0ull);
}

__device__ __forceinline__ uint32_t pred_local(const LeafRec &L, uint64_t key) {
    const float p = __fadd_rn(__fmul_rn(L.b1, local_feature(L, key)), L.b0);
    if (!(p > 0.f)) return 0;
    if (p >= (float)L.size) return L.size;
    return (uint32_t)p;
}

// Search window [first, first + len] of x: the leaf's predicted local rank
// widened by the leaf's measured errors, clamped to the leaf's rank interval.
__device__ __forceinline__ void learned_window(const RootRec &root, const LeafRec *__restrict__ leaves, uint64_t x,
                                               uint64_t &first, uint64_t &len) {
    const LeafRec L = leaves[leaf_of(root, x)];
    const int64_t p = (int64_t)pred_local(L, x);
    int64_t w0 = p + L.elo, w1 = p + (int64_t)L.ehi + 1;
    w0 = w0 < 0 ? 0 : (w0 > (int64_t)L.size ? (int64_t)L.size : w0);
    w1 = w1 < w0 ? w0 : (w1 > (int64_t)L.size ? (int64_t)L.size : w1);
    first = L.base + (uint64_t)w0;
    len = (uint64_t)(w1 - w0);
}

// Lower-bound rank of x through the model (exact: the window holds it).
template <typename K>
__device__ __forceinline__ uint64_t learned_lower_rank(const K *__restrict__ keys, uint64_t n, const RootRec &root,
                                                       const LeafRec *__restrict__ leaves, K x) {
    uint64_t b, len;
    learned_window(root, leaves, (uint64_t)x, b, len);
    while (len > 15) {
        const uint64_t half = len >> 1;
        b = keys[b + half - 1] < x ? b + half : b;
        len -= half;
    }
    bool eq;
    return b + count_below<K, 16>(keys, b, (uint32_t)len, x, eq);
}

// ---- training helpers shared by the single-index and batched trainers

// Accumulator layout per linear model: N, Sx, Sxx, Sr, Srx, Srr (FP64).
constexpr int NACC = 6;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Newton step on a linear model from its accumulated sums; a non-negative
// slope is enforced (the fitted slope of rank against a non-decreasing
// feature is non-negative up to rounding).
__device__ __forceinline__ void newton_linear(const double *a, float &c0, float &c1) {
    const double N = a[0], Sx = a[1], Sxx = a[2], Sr = a[3], Srx = a[4];
    if (N < 1.0) {
        c0 = 0.f;
        c1 = 0.f;
        return;
    }
    const double det = Sxx * N - Sx * Sx;
    double n1 = c1, n0 = c0;
    if (N >= 2.0 && det > 1e-12 * Sxx * N && det > 0.0) {
        // [d1, d0] = H^-1 g with g = (Srx, Sr), H = [[Sxx, Sx], [Sx, N]] (the 2s cancel)
        const double d1 = (N * Srx - Sx * Sr) / det;
        const double d0 = (Sxx * Sr - Sx * Srx) / det;
        n1 -= d1;
        n0 -= d0;
    } else {
        n1 = 0.0;
        n0 = (double)c0 + (double)c1 * (Sx / N) - Sr / N;  // the mean target
    }
    if (n1 < 0.0) {
        // keep the model monotone: best constant
        const double mean_t = (double)c0 + (double)c1 * (Sx / N) - Sr / N;
        n1 = 0.0;
        n0 = mean_t;
    }
    c1 = (float)n1;
    c0 = (float)n0;
}

// Flush a thread's running sums for leaf `l`: when the whole wave holds the
// same leaf, reduce across the wave first and add once.
template <int NV, typename T, typename F>
__device__ __forceinline__ void flush(uint32_t l, T *v, bool active, F &&add) {
    const uint64_t act = __ballot(active);
    const uint32_t lead = __shfl((int)l, __builtin_ctzll(act ? act : 1ull), kWave);
    const bool uniform = act != 0 && __ballot(active && l == lead) == act && act == __ballot(true);
    if (uniform) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
        if ((threadIdx.x & (kWave - 1)) == 0) add(l, v);
    } else if (active) {
        add(l, v);
    }
}

}  // namespace idx
