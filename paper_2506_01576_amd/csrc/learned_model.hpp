// The learned rank model's records and its evaluation, shared by the
// training/lookup kernels (learned.hip) and the batched launch (batch.hip).
#pragma once

#include <climits>

#include "internal.hpp"
#include "search.hpp"

namespace idx {

// One bin of the spline root: a key x of the bin goes to leaf
// first + ((max(x - anchor, 0) >> shift) * mul) >> 32, at most L - 1.
struct __align__(16) SplineBin {
    uint64_t anchor;       // smallest build key of the bin (0 for an empty bin)
    uint32_t mul;          // leaves per key offset, 32-bit fixed point
    uint32_t first_shift;  // bits 0-25: first leaf of the bin; bits 26-31: shift (<= 32)
};
static_assert(sizeof(SplineBin) == 16, "spline bin is 16 bytes");

struct RootRec {
    float a0, a1;           // linear roots: t = a1 * x + a0, leaf = clamp(floor(t), 0, L - 1)
    uint32_t mode;          // IDX_FEATURE_LINEAR / IDX_FEATURE_LOG / IDX_FEATURE_SPLINE
    uint32_t L;
    const SplineBin *bins;  // spline: nb bin records
    uint64_t f_lo;          // spline: bin feature of the smallest build key
    uint32_t shift;         // spline: bin = (feature - f_lo) >> shift (64: a single bin)
    uint32_t nb;            // spline: bins in use
    uint32_t bfeat;         // spline: bin feature, IDX_FEATURE_LINEAR or IDX_FEATURE_LOG
    uint32_t pad;
};
static_assert(sizeof(RootRec) == 48, "root record is 48 bytes");

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
    SplineBin *spline = nullptr;  // device: the spline root's bins (spline root only)
    uint4 *lines = nullptr;       // device: one 128-byte line per leaf, written on first use
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

// Bins of the spline root for n keys: the largest power of two <= 65536 with
// at least 64 keys per bin (1 for tiny sets).
__host__ __device__ inline uint32_t spline_bins(uint64_t n) {
    uint32_t B = 1;
    while (B < 65536u && (uint64_t)B * 2 * 64 <= n) B <<= 1;
    return B;
}

// Integer key features of the spline bins, both exact and non-decreasing.
// LINEAR: the key.  LOG: floor(log2 key) in bits 58-63, then the 58 bits
// below the key's leading one (a 64-bit float-like code; 0 and 1 map to 0).
__host__ __device__ __forceinline__ uint64_t bin_feature(uint64_t key, uint32_t bfeat) {
    if (bfeat == IDX_FEATURE_LINEAR || key == 0) return key;
    const uint32_t e = 63u - (uint32_t)__builtin_clzll(key);
    return ((uint64_t)e << 58) | (((key << (63 - e)) << 1) >> 6);
}

__host__ __device__ __forceinline__ uint32_t bin_of(const RootRec &R, uint64_t key) {
    const uint64_t u = bin_feature(key, R.bfeat);
    if (u <= R.f_lo || R.shift >= 64) return 0;
    const uint64_t b = (u - R.f_lo) >> R.shift;
    return b < R.nb ? (uint32_t)b : R.nb - 1;
}

// The bin geometry for build keys kmin..kmax: nb = ((f(kmax) - f(kmin)) >>
// shift) + 1 bins with the smallest shift that keeps nb <= spline_bins(n).
__host__ __device__ inline void spline_geometry(RootRec &R, uint64_t kmin, uint64_t kmax, uint64_t n) {
    const uint32_t B = spline_bins(n);
    R.f_lo = bin_feature(kmin, R.bfeat);
    const uint64_t span = bin_feature(kmax, R.bfeat) - R.f_lo;
    uint32_t sh = 0;
    while (sh < 64 && (span >> sh) >= B) ++sh;
    R.shift = sh;
    R.nb = sh >= 64 ? 1u : (uint32_t)(span >> sh) + 1u;
}

// Spline root: one bin record, then a fixed-point product.  Non-decreasing in
// the key: inside a bin by construction, and across bins because the bin's
// multiplier keeps every key below the bin's upper boundary under the next
// bin's first leaf.  coord, when asked for, is the unrounded leaf coordinate.
__device__ __forceinline__ uint32_t spline_leaf(const RootRec &R, uint64_t key, float *coord = nullptr) {
    const SplineBin r = R.bins[bin_of(R, key)];
    const uint64_t d = key > r.anchor ? key - r.anchor : 0ull;
    const uint32_t sh = r.first_shift >> 26;
    const uint64_t prod = (uint64_t)(uint32_t)(d >> sh) * (uint64_t)r.mul;
    const uint64_t leaf = (uint64_t)(r.first_shift & 0x3FFFFFFu) + (prod >> 32);
    if (coord) *coord = __fadd_rn((float)(r.first_shift & 0x3FFFFFFu), __fmul_rn((float)prod, 0x1p-32f));
    return leaf < R.L ? (uint32_t)leaf : R.L - 1;
}

// Estimated lookup cost of a trained model, to choose between a linear and a
// spline root: the binary-search steps over the key-weighted mean window, plus
// one for the spline root's bin record.  A tie keeps the linear root.
__host__ __device__ inline double window_cost(double mean_window, bool spline) {
    return log2(1.0 + mean_window) + (spline ? 1.0 : 0.0);
}

// Smallest key whose bin is at least b (1 <= b < nb): a binary search over the
// 64-bit key range of the non-decreasing bin function.
__host__ __device__ inline uint64_t bin_lower_key(const RootRec &R, uint32_t b) {
    uint64_t lo = 0, hi = ~0ull;  // bin(hi) >= b always (b < nb)
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (bin_of(R, mid) >= b) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Record of bin b over n sorted keys (key(i) reads rank i).  Ranks r_b (keys
// in bins below b) come from binary searches; the bin takes the leaves
// [floor(r_b L / n), floor(r_b+1 L / n)).  Its multiplier is the largest
// 32-bit fixed-point value that maps the bin's whole key range, up to the
// next bin's lower boundary, below that span.
template <typename KeyAt>
__host__ __device__ inline SplineBin spline_bin(const KeyAt &key, uint64_t n, const RootRec &R, uint32_t b) {
    auto rank_below = [&](uint32_t bin) -> uint64_t {  // keys with bin < `bin`
        if (bin == 0) return 0;
        if (bin >= R.nb) return n;
        uint64_t lo = 0, len = n;
        while (len > 0) {
            const uint64_t half = len >> 1;
            if (bin_of(R, key(lo + half)) < bin) {
                lo += half + 1;
                len -= half + 1;
            } else {
                len = half;
            }
        }
        return lo;
    };
    const uint64_t r0 = rank_below(b), r1 = rank_below(b + 1);
    const uint64_t f0 = (r0 * R.L) / n, f1 = (r1 * R.L) / n;
    SplineBin out{0ull, 0u, (uint32_t)f0};
    if (r1 == r0 || f1 == f0) {
        if (r1 > r0) out.anchor = key(r0);
        return out;
    }
    out.anchor = key(r0);
    const uint64_t wm1 = b + 1 >= R.nb ? ~out.anchor : bin_lower_key(R, b + 1) - 1 - out.anchor;
    uint32_t sh = 0;
    while ((wm1 >> sh) > 0xFFFFFFFFull) ++sh;
    const uint64_t ws = (wm1 >> sh) + 1;  // <= 2^32
    const uint64_t m = ((f1 - f0) << 32) / ws;
    out.mul = m > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)m;
    out.first_shift = (uint32_t)f0 | (sh << 26);
    return out;
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

// Search window [first, first + len] of x in leaf L: the leaf's predicted
// local rank widened by its measured errors, clamped to its rank interval.
__device__ __forceinline__ void leaf_window(const LeafRec &L, uint64_t x, uint64_t &first, uint64_t &len) {
    const int64_t p = (int64_t)pred_local(L, x);
    int64_t w0 = p + L.elo, w1 = p + (int64_t)L.ehi + 1;
    w0 = w0 < 0 ? 0 : (w0 > (int64_t)L.size ? (int64_t)L.size : w0);
    w1 = w1 < w0 ? w0 : (w1 > (int64_t)L.size ? (int64_t)L.size : w1);
    first = L.base + (uint64_t)w0;
    len = (uint64_t)(w1 - w0);
}

// The window of x in the leaf the root sends it to.
__device__ __forceinline__ void learned_window(const RootRec &root, const LeafRec *__restrict__ leaves, uint64_t x,
                                               uint64_t &first, uint64_t &len) {
    leaf_window(leaves[leaf_of(root, x)], x, first, len);
}

// ---- leaf lines: one 128-byte line per leaf, so that a lookup in a small
// leaf reads one line after the root.  The root is non-decreasing in the
// key, so every build key below x lies in a leaf before x's leaf or in it,
// and every key above x in it or after it: the lower bound of x is the
// leaf's base rank plus the leaf's keys below x.  Line layout (32-bit
// words): word 0 the base rank, word 1 the size; from byte 8 the leaf's
// first min(size, line_slots) keys in ascending order, then their row IDs.
// When x is above every key the line holds and the leaf has more, its lower
// bound lies among the leaf's remaining keys [base + line_slots, base +
// size), which are searched in the sorted array.
constexpr uint32_t kLineBytes = 128;
constexpr uint32_t kLineChunks = kLineBytes / 16;

template <typename K>
__host__ __device__ constexpr uint32_t line_slots() {
    return (kLineBytes - 8) / (uint32_t)(sizeof(K) + 4);  // 64-bit keys: 10; 32-bit keys: 15
}

// Word i (static) of a line held in registers.
__device__ __forceinline__ uint32_t line_word(const uint4 (&w)[kLineChunks], int i) {
    const uint4 &v = w[i >> 2];
    return (i & 3) == 0 ? v.x : (i & 3) == 1 ? v.y : (i & 3) == 2 ? v.z : v.w;
}

template <typename K>
__device__ __forceinline__ K line_key(const uint4 (&w)[kLineChunks], int j) {
    if constexpr (sizeof(K) == 8) return ((uint64_t)line_word(w, 3 + 2 * j) << 32) | line_word(w, 2 + 2 * j);
    else return line_word(w, 2 + j);
}

// The line's keys below x (cnt), and the row ID of the key at rank cnt when
// it equals x.  False when the lower bound lies past the line's keys in a
// leaf that has more: [tail, tail + tail_len] then holds it.
template <typename K>
__device__ __forceinline__ bool line_scan(const uint4 (&w)[kLineChunks], K x, uint32_t &cnt, bool &eq,
                                          uint32_t &row, uint64_t &tail, uint64_t &tail_len) {
    constexpr uint32_t C = line_slots<K>();
    constexpr int R0 = 2 + (int)(C * sizeof(K) / 4);  // first row ID word
    const uint32_t size = w[0].y;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < (int)C; ++j) c += ((uint32_t)j < size && line_key<K>(w, j) < x) ? 1u : 0u;
    if (c == C && size > C) {
        tail = (uint64_t)w[0].x + C;
        tail_len = size - C;
        return false;
    }
    bool e = false;
    uint32_t r = kMiss;
#pragma unroll
    for (int j = 0; j < (int)C; ++j)
        if ((uint32_t)j == c && (uint32_t)j < size && line_key<K>(w, j) == x) {
            e = true;
            r = line_word(w, R0 + j);
        }
    cnt = c;
    eq = e;
    row = r;
    return true;
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

// Per-leaf reductions over the consecutive keys [b, e) walked by one wave, 64
// keys per step (lane j takes key b + 64 s + j), so every load is coalesced.
// For key i, step(i, leaf, v) sets its leaf and its NV values and returns
// whether the key takes part (keys that do not are skipped).  Leaf ids never
// decrease along the keys, so a step holds few distinct leaves: each is
// reduced across the wave with comb and merged into a carry that all lanes
// hold; a finished carry goes to add(leaf, values), called by lane 0 (once per
// leaf the wave touches instead of once per lane and leaf).
template <int NV, typename T, typename Comb, typename Step, typename Add>
__device__ __forceinline__ void wave_leaf_reduce(uint64_t b, uint64_t e, T ident, Comb &&comb, Step &&step,
                                                 Add &&add) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    uint32_t carry_leaf = 0xFFFFFFFFu;
    T carry[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) carry[j] = ident;
    for (uint64_t s0 = b; s0 < e; s0 += kWave) {
        const uint64_t i = s0 + lane;
        const bool live = i < e;
        uint32_t l = 0xFFFFFFFFu;
        T v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = ident;
        const bool part = live && step(i, l, v);
        uint64_t todo = __ballot(part);
        while (todo) {
            const uint32_t lead = (uint32_t)__shfl((int)l, __builtin_ctzll(todo), kWave);
            const bool mine = part && l == lead;
            todo &= ~__ballot(mine);
            T sv[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                T x = mine ? v[j] : ident;
#pragma unroll
                for (int off = kWave / 2; off > 0; off >>= 1) x = comb(x, __shfl_xor(x, off, kWave));
                sv[j] = x;
            }
            if (lead != carry_leaf) {
                if (carry_leaf != 0xFFFFFFFFu && lane == 0) add(carry_leaf, carry);
                carry_leaf = lead;
#pragma unroll
                for (int j = 0; j < NV; ++j) carry[j] = sv[j];
            } else {
#pragma unroll
                for (int j = 0; j < NV; ++j) carry[j] = comb(carry[j], sv[j]);
            }
        }
    }
    if (carry_leaf != 0xFFFFFFFFu && lane == 0) add(carry_leaf, carry);
}

// Leaves of at most kLeafCap keys are walked by one thread each in the
// per-leaf passes (their key ranges are known after the layout); larger
// leaves go through the wave walk.  The cap keeps the edge leaves of a linear
// root (where the fitted line leaves the key range) on the cheap path.
constexpr uint32_t kLeafCap = 4096;

// A key's terms of the leaf line fit: count, d, d^2, r, r d, r^2, with d the
// leaf-local key offset and r the residual of the leaf's prediction at rank i.
__device__ __forceinline__ void leaf_terms(const LeafRec &L, uint64_t i, uint64_t key, double *a) {
    const float d = local_feature(L, key);
    const float y = (float)(uint32_t)(i - L.base);
    const float r = __fsub_rn(__fadd_rn(__fmul_rn(L.b1, d), L.b0), y);
    a[0] = 1.0;
    a[1] = d;
    a[2] = (double)d * d;
    a[3] = r;
    a[4] = (double)r * d;
    a[5] = (double)r * r;
}

// A key's error: true local rank minus the predicted local rank.
__device__ __forceinline__ long long leaf_err(const LeafRec &L, uint64_t i, uint64_t key) {
    return (long long)(i - L.base) - (long long)pred_local(L, key);
}

// Keys a leaf-walking thread loads before using any of them, so that its
// loads are in flight together.
constexpr int kLeafBatch = 8;

// Per-leaf passes run one thread per leaf, kLeafBlock leaves per workgroup;
// those leaves cover one contiguous rank range (the bases are the exclusive
// scan of the sizes).  When it holds no more keys than the staging area
// (kStageKeys at most) the workgroup copies it into LDS with consecutive
// loads and each thread walks its leaf there: a thread walking its leaf in
// global memory issues loads that touch 64 different lines per wave.
constexpr uint32_t kLeafBlock = 256;
constexpr uint32_t kStageKeys = 8192;

// Keys staged per workgroup of the per-leaf passes over n keys in L leaves
// (dynamic LDS of the launch): twice a workgroup's mean key count as a power
// of two in [1024, kStageKeys].  A small area lets more workgroups share a
// compute unit (the full one allows two).  A workgroup whose leaves hold more
// keys than the area reads them from memory; where that is the rule (long
// leaves) the full area stays, since those per-thread walks ran slower at
// the higher occupancy a small area allows (batched training of 64-key
// leaves: 240 -> 270 ms without an area).
inline uint32_t stage_cap(uint64_t n, uint64_t L) {
    if (L == 0) return kStageKeys;
    const uint64_t mean = (uint64_t)kLeafBlock * ((n + L - 1) / L);
    uint32_t cap = 1024;
    while (cap < 2 * mean && cap < kStageKeys) cap <<= 1;
    return cap;
}

// Copies keys [kb, ke) (ke - kb <= kStageKeys) into s_key, then a barrier.
template <typename K, typename KeyAt>
__device__ __forceinline__ void stage_keys(const KeyAt &key, uint64_t kb, uint64_t ke, K *s_key) {
    constexpr int U = 8;
    for (uint64_t i0 = kb; i0 < ke; i0 += (uint64_t)U * kLeafBlock) {
        K v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kLeafBlock + threadIdx.x;
            v[u] = i < ke ? key(i) : K(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kLeafBlock + threadIdx.x;
            if (i < ke) s_key[i - kb] = v[u];
        }
    }
    __syncthreads();
}

// The sums of one leaf, walked by one thread (key(i) reads rank i).
template <typename KeyAt>
__device__ __forceinline__ void leaf_sums_thread(const KeyAt &key, const LeafRec &L, double *a) {
    for (int j = 0; j < NACC; ++j) a[j] = 0.0;
    const uint64_t end = (uint64_t)L.base + L.size;
    for (uint64_t i0 = L.base; i0 < end; i0 += kLeafBatch) {
        uint64_t kb[kLeafBatch];
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) kb[u] = i0 + u < end ? key(i0 + u) : 0ull;
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) {
            if (i0 + u >= end) continue;
            double t[NACC];
            leaf_terms(L, i0 + u, kb[u], t);
#pragma unroll
            for (int j = 0; j < NACC; ++j) a[j] += t[j];
        }
    }
}

// A key's squared FP32 forward residual (the loss term of leaf_terms).
__device__ __forceinline__ double leaf_sq_residual(const LeafRec &L, uint64_t i, uint64_t key) {
    const float d = local_feature(L, key);
    const float y = (float)(uint32_t)(i - L.base);
    const float r = __fsub_rn(__fadd_rn(__fmul_rn(L.b1, d), L.b0), y);
    return (double)r * r;
}

// The error bounds of one leaf, walked by one thread; with loss, the leaf's
// squared residuals are added to *loss in the same walk.
template <typename KeyAt>
__device__ __forceinline__ void leaf_errs_thread(const KeyAt &key, const LeafRec &L, long long &lo, long long &hi,
                                                 double *loss = nullptr) {
    lo = INT_MAX;
    hi = INT_MIN;
    const uint64_t end = (uint64_t)L.base + L.size;
    for (uint64_t i0 = L.base; i0 < end; i0 += kLeafBatch) {
        uint64_t kb[kLeafBatch];
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) kb[u] = i0 + u < end ? key(i0 + u) : 0ull;
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) {
            if (i0 + u >= end) continue;
            const long long e = leaf_err(L, i0 + u, kb[u]);
            lo = e < lo ? e : lo;
            hi = e > hi ? e : hi;
            if (loss) *loss += leaf_sq_residual(L, i0 + u, kb[u]);
        }
    }
}

// Keys per leaf over the wave's keys [b, e), 64 consecutive keys per step:
// a step's leaves form runs of equal values, and the last lane of each run
// calls add(leaf, run length), the start of the run coming from the ballot of
// run ends.  The runs partition the step's keys, so every key is counted
// once; with ascending keys and a monotone leaf map a leaf appears in at
// most one run per step.  Integer work only (no cross-lane FP64).
template <typename LeafAt, typename Add>
__device__ __forceinline__ void wave_leaf_counts(uint64_t b, uint64_t e, LeafAt &&leaf_at, Add &&add) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    constexpr int U = 4;  // steps whose keys are loaded before any atomic
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    for (uint64_t s0 = b; s0 < e; s0 += (uint64_t)U * kWave) {
        uint32_t l[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = s0 + (uint64_t)u * kWave + lane;
            l[u] = i < e ? leaf_at(i) : kNone;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t next = __shfl_down(l[u], 1);
            const bool last = l[u] != kNone && (lane == kWave - 1 || next != l[u]);
            const uint64_t ends = __ballot(last);
            if (last) {
                const uint64_t before = ends & ((1ull << lane) - 1ull);
                const uint32_t start = before ? 64u - (uint32_t)__builtin_clzll(before) : 0u;
                add(l[u], lane + 1u - start);
            }
        }
    }
}

template <int NV, typename Step, typename Add>
__device__ __forceinline__ void wave_leaf_sums(uint64_t b, uint64_t e, Step &&step, Add &&add) {
    wave_leaf_reduce<NV, double>(b, e, 0.0, [](double x, double y) { return x + y; }, step, add);
}

// Error bounds: per leaf the max of -err and of err (err = true local rank -
// predicted local rank), as int64.
template <typename Step, typename Add>
__device__ __forceinline__ void wave_leaf_maxes(uint64_t b, uint64_t e, Step &&step, Add &&add) {
    wave_leaf_reduce<2, long long>(b, e, (long long)INT64_MIN,
                                   [](long long x, long long y) { return x > y ? x : y; }, step, add);
}

}  // namespace idx
