// Batched training of learned rank models: the models of many sorted-array
// indexes are trained by one sequence of launches whose every kernel spans
// all of them, so a thousand small indexes cost what one large one does
// (same stages, same arithmetic and same Newton steps as the single-index
// trainer in learned.hip; only the work split differs).
//
// The keys of every index are cut into units of UNIT consecutive keys (one
// workgroup each; a unit never straddles two indexes).  Root sums of all root
// candidates (linear over either key feature, spline over either bin feature)
// are accumulated in one pass; within each family the lower loss is picked on
// the device, and with both families the leaves are trained under each root
// and the lower estimated lookup cost is kept, per index, also on the device.
// The whole sequence synchronises the host once, at the end, to read back the
// roots and statistics.
#include <climits>

#include <new>
#include <unordered_set>
#include <vector>

#include "internal.hpp"
#include "learned_model.hpp"

namespace idx {
namespace {

constexpr int BT = 256;                      // threads per workgroup
constexpr int BCH = 32;                      // consecutive keys per thread in the leaf passes
constexpr uint64_t UNIT = (uint64_t)BT * BCH;  // keys per unit
constexpr int NST = 4;                       // per-index stats: sum w*size, max w, leaf loss, root loss

struct TDesc {
    const void *keys;
    uint64_t n;
    LeafRec *leaves;    // the index's model table
    uint64_t leaf_off;  // its first leaf in the accumulator arrays
    SplineBin *spline;  // the index's spline bins (when a spline root may be kept)
    uint32_t L;
    uint32_t pad;
};

struct Unit {
    uint64_t begin, end;  // key range of one index
    uint32_t index;
    uint32_t pad;
};

// Root candidates per index: 0 = linear over the LINEAR feature, 1 = linear
// over the LOG feature, 2 = spline over LINEAR bins, 3 = spline over LOG bins
// (bit c of cmask enables candidate c).
constexpr int NCAND = 4;

template <typename K>
__global__ __launch_bounds__(BT) void k_bt_root_accum(const Unit *__restrict__ units, const TDesc *__restrict__ d,
                                                      const RootRec *__restrict__ roots, uint32_t cmask,
                                                      double *__restrict__ acc) {
    __shared__ double s[BT / kWave][NCAND * NACC];
    const Unit u = units[blockIdx.x];
    const TDesc D = d[u.index];
    const K *keys = (const K *)D.keys;
    RootRec R[NCAND];
#pragma unroll
    for (int c = 0; c < NCAND; ++c) R[c] = roots[NCAND * u.index + c];
    const double scale = (double)D.L / (double)D.n;
    double a[NCAND * NACC];
#pragma unroll
    for (int j = 0; j < NCAND * NACC; ++j) a[j] = 0.0;
    for (uint64_t i = u.begin + threadIdx.x; i < u.end; i += BT) {
        const uint64_t key = (uint64_t)keys[i];
        const float t = (float)((double)i * scale);
#pragma unroll
        for (int c = 0; c < NCAND; ++c) {
            if (!(cmask & (1u << c))) continue;
            float x, pred;
            if (c >= 2) {
                x = 0.f;
                (void)spline_leaf(R[c], key, &pred);
            } else {
                x = key_feature(key, R[c].mode);
                pred = __fadd_rn(__fmul_rn(R[c].a1, x), R[c].a0);
            }
            const float r = __fsub_rn(pred, t);
            double *b = a + c * NACC;
            b[0] += 1.0;
            b[1] += x;
            b[2] += (double)x * x;
            b[3] += r;
            b[4] += (double)r * x;
            b[5] += (double)r * r;
        }
    }
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NCAND * NACC; ++j) {
        const double v = wave_sum(a[j]);
        if (lane == 0) s[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NCAND * NACC && (cmask & (1u << (threadIdx.x / NACC)))) {
        double v = 0;
        for (int w = 0; w < BT / kWave; ++w) v += s[w][threadIdx.x];
        atomicAdd(&acc[(uint64_t)u.index * NCAND * NACC + threadIdx.x], v);
    }
}

// Newton steps for the two linear candidates.
__global__ void k_bt_root_update(RootRec *__restrict__ roots, const double *__restrict__ acc, uint32_t count,
                                 uint32_t cmask) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = t / 2, c = t % 2;
    if (i >= count || !(cmask & (1u << c))) return;
    RootRec R = roots[NCAND * i + c];
    newton_linear(acc + ((uint64_t)NCAND * i + c) * NACC, R.a0, R.a1);
    roots[NCAND * i + c].a0 = R.a0;
    roots[NCAND * i + c].a1 = R.a1;
}

// Per family, the lowest final loss wins (the lower candidate number on a
// tie): best_lin / best_sp and their losses in stats entry 3.  The spline
// winner will read its bins from the index's own table; src gets the
// scratch table they are copied from.
__global__ void k_bt_root_pick(const RootRec *__restrict__ roots, const double *__restrict__ acc,
                               const TDesc *__restrict__ d, uint32_t count, uint32_t cmask,
                               RootRec *__restrict__ best_lin, RootRec *__restrict__ best_sp,
                               const SplineBin **__restrict__ src, double *__restrict__ st_lin,
                               double *__restrict__ st_sp) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    for (int fam = 0; fam < 2; ++fam) {
        int f = -1;
        double fl = 0.0;
        for (int c = 2 * fam; c < 2 * fam + 2; ++c) {
            if (!(cmask & (1u << c))) continue;
            const double l = acc[((uint64_t)NCAND * i + c) * NACC + 5];
            if (f < 0 || l < fl) {
                f = c;
                fl = l;
            }
        }
        if (f < 0) continue;
        RootRec R = roots[NCAND * i + f];
        if (fam == 0) {
            best_lin[i] = R;
            st_lin[(uint64_t)i * NST + 3] = fl;
        } else {
            src[i] = R.bins;
            R.bins = d[i].spline;
            best_sp[i] = R;
            st_sp[(uint64_t)i * NST + 3] = fl;
        }
    }
}

// Spline geometry of candidates 2 and 3 of every index (one thread each).
template <typename K>
__global__ void k_bt_spline_geometry(const TDesc *__restrict__ d, RootRec *__restrict__ roots, uint32_t count,
                                     uint32_t cmask) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = t / 2, c = 2 + t % 2;
    if (i >= count || !(cmask & (1u << c))) return;
    const K *keys = (const K *)d[i].keys;
    spline_geometry(roots[NCAND * i + c], (uint64_t)keys[0], (uint64_t)keys[d[i].n - 1], d[i].n);
}

// Bins of spline candidate 2 + blockIdx.z of index blockIdx.x, one thread per
// bin, into the candidate's scratch table.
template <typename K>
__global__ void k_bt_spline_bins(const TDesc *__restrict__ d, const RootRec *__restrict__ roots, uint32_t cmask) {
    const uint32_t i = blockIdx.x, c = 2 + blockIdx.z;
    if (!(cmask & (1u << c))) return;
    const RootRec R = roots[NCAND * i + c];
    const uint32_t b = blockIdx.y * blockDim.x + threadIdx.x;
    if (b >= R.nb) return;
    const K *keys = (const K *)d[i].keys;
    ((SplineBin *)R.bins)[b] = spline_bin([&](uint64_t r) { return (uint64_t)keys[r]; }, d[i].n, R, b);
}

// The winning spline bins into each index's own table.
__global__ void k_bt_copy_bins(const RootRec *__restrict__ best_sp, const SplineBin *const *__restrict__ src) {
    const uint32_t i = blockIdx.x;
    const uint32_t b = blockIdx.y * blockDim.x + threadIdx.x;
    const RootRec R = best_sp[i];
    if (b < R.nb) ((SplineBin *)R.bins)[b] = src[i][b];
}

__global__ void k_bt_zero(double *p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_bt_zero_u32(uint32_t *p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// This wave's BCH * 64 consecutive keys of the unit.
__device__ __forceinline__ void wave_range(const Unit &u, uint64_t &b, uint64_t &e) {
    b = u.begin + (uint64_t)(threadIdx.x & ~(uint32_t)(kWave - 1)) * BCH;
    e = b + (uint64_t)kWave * BCH < u.end ? b + (uint64_t)kWave * BCH : u.end;
}

template <typename K>
__global__ __launch_bounds__(BT) void k_bt_leaf_count(const Unit *__restrict__ units, const TDesc *__restrict__ d,
                                                      const RootRec *__restrict__ best, uint32_t *__restrict__ cnt) {
    const Unit u = units[blockIdx.x];
    uint64_t b, e;
    wave_range(u, b, e);
    const TDesc D = d[u.index];
    const K *keys = (const K *)D.keys;
    const RootRec R = best[u.index];
    uint32_t *c = cnt + D.leaf_off;
    wave_leaf_counts(
        b, e, [&](uint64_t i) { return leaf_of(R, (uint64_t)keys[i]); },
        [&](uint32_t l, uint32_t n) { atomicAdd(&c[l], n); });
}

// One workgroup per index: leaf bases (exclusive scan of the counts), sizes,
// first keys; parameters start at zero.
template <typename K>
__global__ __launch_bounds__(1024) void k_bt_leaf_layout(const TDesc *__restrict__ d, const uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_tot[1024 / kWave];
    __shared__ uint32_t s_run;
    const TDesc D = d[blockIdx.x];
    const K *keys = (const K *)D.keys;
    const uint32_t *c = cnt + D.leaf_off;
    if (threadIdx.x == 0) s_run = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (uint32_t c0 = 0; c0 < D.L; c0 += 1024) {
        const uint32_t l = c0 + threadIdx.x;
        const uint32_t v = l < D.L ? c[l] : 0;
        uint32_t incl = v;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t x = __shfl_up(incl, off, kWave);
            if (lane >= (uint32_t)off) incl += x;
        }
        if (lane == kWave - 1) s_tot[wave] = incl;
        __syncthreads();
        uint32_t before = s_run;
        for (uint32_t w = 0; w < wave; ++w) before += s_tot[w];
        if (l < D.L) {
            LeafRec r{};
            r.base = before + incl - v;
            r.size = v;
            r.kmin = v ? (uint64_t)keys[r.base] : 0ull;
            r.b0 = 0.f;
            r.b1 = 0.f;
            r.elo = INT_MAX;
            r.ehi = INT_MIN;
            D.leaves[l] = r;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            uint32_t tot = 0;
            for (int w = 0; w < 1024 / kWave; ++w) tot += s_tot[w];
            s_run += tot;
        }
        __syncthreads();
    }
}

// Index owning global leaf g: the last i with d[i].leaf_off <= g.
__device__ __forceinline__ uint32_t leaf_owner(const TDesc *__restrict__ d, uint32_t count, uint64_t g) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (d[mid].leaf_off <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The workgroup's leaves' keys into LDS, when all its leaves belong to one
// index and their range holds at most `cap` keys (else false).
template <typename K>
__device__ __forceinline__ bool bt_stage_leaf_keys(const TDesc *__restrict__ d, uint32_t count, uint64_t total,
                                                   K *s_key, uint32_t cap, uint64_t &kb) {
    const uint64_t g0 = (uint64_t)blockIdx.x * kLeafBlock;
    if (g0 >= total) return false;  // workgroup-uniform, as every test below
    const uint64_t g1 = g0 + kLeafBlock < total ? g0 + kLeafBlock : total;
    const uint32_t o = leaf_owner(d, count, g0);
    if (leaf_owner(d, count, g1 - 1) != o) return false;
    const TDesc D = d[o];
    kb = D.leaves[g0 - D.leaf_off].base;
    const LeafRec last = D.leaves[g1 - 1 - D.leaf_off];
    const uint64_t ke = (uint64_t)last.base + last.size;
    if (ke - kb > cap) return false;
    const K *keys = (const K *)D.keys;
    stage_keys<K>([&](uint64_t i) { return keys[i]; }, kb, ke, s_key);
    return true;
}

// Per-leaf sums, one thread per leaf (global leaf g) over its key range; a
// leaf of more than kLeafCap keys gets zero sums and raises *big.
template <typename K>
// (The staging area holds `cap` keys: dynamic LDS sized by stage_cap.)
__global__ __launch_bounds__(kLeafBlock) void k_bt_leaf_accum_small(const TDesc *__restrict__ d, uint32_t count,
                                                                    uint64_t total, double *__restrict__ acc,
                                                                    uint32_t *big, uint32_t cap) {
    extern __shared__ __align__(16) char smem_stage[];
    K *s_key = (K *)smem_stage;
    uint64_t kb;
    const bool staged = bt_stage_leaf_keys(d, count, total, s_key, cap, kb);
    const uint64_t g = (uint64_t)blockIdx.x * kLeafBlock + threadIdx.x;
    if (g >= total) return;
    const TDesc D = d[leaf_owner(d, count, g)];
    const K *keys = (const K *)D.keys;
    const LeafRec r = D.leaves[g - D.leaf_off];
    double a[NACC] = {0, 0, 0, 0, 0, 0};
    if (r.size > kLeafCap) *big = 1u;
    else if (staged) leaf_sums_thread([&](uint64_t i) { return (uint64_t)s_key[i - kb]; }, r, a);
    else leaf_sums_thread([&](uint64_t i) { return (uint64_t)keys[i]; }, r, a);
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[g * NACC + j] = a[j];
}

// The keys of leaves larger than kLeafCap: the wave walk over the units,
// skipping every step without such a key.
template <typename K>
__global__ __launch_bounds__(BT) void k_bt_leaf_accum_big(const Unit *__restrict__ units, const TDesc *__restrict__ d,
                                                          const RootRec *__restrict__ best, double *__restrict__ acc,
                                                          const uint32_t *big) {
    if (*big == 0u) return;
    const Unit u = units[blockIdx.x];
    uint64_t b, e;
    wave_range(u, b, e);
    const TDesc D = d[u.index];
    const K *keys = (const K *)D.keys;
    const RootRec R = best[u.index];
    double *A = acc + D.leaf_off * NACC;
    wave_leaf_sums<NACC>(
        b, e,
        [&](uint64_t i, uint32_t &l, double *a) {
            const uint64_t key = (uint64_t)keys[i];
            l = leaf_of(R, key);
            const LeafRec L = D.leaves[l];
            if (L.size <= kLeafCap) return false;
            leaf_terms(L, i, key, a);
            return true;
        },
        [&](uint32_t l, const double *v) {
#pragma unroll
            for (int j = 0; j < NACC; ++j) atomicAdd(&A[(uint64_t)l * NACC + j], v[j]);
        });
}

__global__ void k_bt_leaf_update(const TDesc *__restrict__ d, uint32_t count, uint64_t total,
                                 const double *__restrict__ acc) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const TDesc D = d[leaf_owner(d, count, g)];
    LeafRec *r = &D.leaves[g - D.leaf_off];
    float b0 = r->b0, b1 = r->b1;
    newton_linear(acc + g * NACC, b0, b1);
    r->b0 = b0;
    r->b1 = b1;
}

// Per-leaf error bounds, one thread per leaf of at most kLeafCap keys.
template <typename K>
__global__ __launch_bounds__(kLeafBlock) void k_bt_leaf_errors_small(const TDesc *__restrict__ d, uint32_t count,
                                                                     uint64_t total, uint32_t cap) {
    extern __shared__ __align__(16) char smem_stage[];
    K *s_key = (K *)smem_stage;
    uint64_t kb;
    const bool staged = bt_stage_leaf_keys(d, count, total, s_key, cap, kb);
    const uint64_t g = (uint64_t)blockIdx.x * kLeafBlock + threadIdx.x;
    if (g >= total) return;
    const TDesc D = d[leaf_owner(d, count, g)];
    const K *keys = (const K *)D.keys;
    LeafRec *p = &D.leaves[g - D.leaf_off];
    const LeafRec r = *p;
    if (r.size == 0 || r.size > kLeafCap) return;
    long long lo, hi;
    if (staged) leaf_errs_thread([&](uint64_t i) { return (uint64_t)s_key[i - kb]; }, r, lo, hi);
    else leaf_errs_thread([&](uint64_t i) { return (uint64_t)keys[i]; }, r, lo, hi);
    p->elo = (int32_t)lo;
    p->ehi = (int32_t)hi;
}

// Error bounds of the leaves larger than kLeafCap (the wave walk).
template <typename K>
__global__ __launch_bounds__(BT) void k_bt_leaf_errors_big(const Unit *__restrict__ units, const TDesc *__restrict__ d,
                                                           const RootRec *__restrict__ best, const uint32_t *big) {
    if (*big == 0u) return;
    const Unit u = units[blockIdx.x];
    uint64_t b, e;
    wave_range(u, b, e);
    const TDesc D = d[u.index];
    const K *keys = (const K *)D.keys;
    const RootRec R = best[u.index];
    wave_leaf_maxes(
        b, e,
        [&](uint64_t i, uint32_t &l, long long *a) {
            const uint64_t key = (uint64_t)keys[i];
            l = leaf_of(R, key);
            const LeafRec L = D.leaves[l];
            if (L.size <= kLeafCap) return false;
            const long long err = leaf_err(L, i, key);
            a[0] = -err;
            a[1] = err;
            return true;
        },
        [&](uint32_t l, const long long *v) {
            atomicMin(&D.leaves[l].elo, (int32_t)(-v[0]));
            atomicMax(&D.leaves[l].ehi, (int32_t)v[1]);
        });
}

// Empty leaves get a zero window; per-index window statistics and leaf loss.
__global__ __launch_bounds__(256) void k_bt_leaf_finish(const TDesc *__restrict__ d, uint32_t count, uint64_t total,
                                                        const double *__restrict__ acc, double *__restrict__ stats) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < total;
    const uint32_t i = live ? leaf_owner(d, count, g) : 0xFFFFFFFFu;
    double ws = 0.0, wmax = 0.0, loss = 0.0;
    if (live) {
        const TDesc D = d[i];
        LeafRec *r = &D.leaves[g - D.leaf_off];
        const LeafRec v = *r;
        if (v.size == 0 || v.elo > v.ehi) {
            r->elo = 0;
            r->ehi = -1;
        } else {
            wmax = (double)v.ehi - (double)v.elo + 2.0;  // window slots incl. one past
            ws = wmax * v.size;
        }
        loss = acc[g * NACC + 5];
    }
    auto put = [&](uint32_t ix, double s0, double m, double s2) {
        double *st = stats + (uint64_t)ix * NST;
        atomicAdd(&st[0], s0);
        atomicAdd(&st[2], s2);
        unsigned long long *p = (unsigned long long *)&st[1];  // max via CAS (values >= 0)
        unsigned long long old = *p;
        while (__longlong_as_double(old) < m) {
            const unsigned long long prev = atomicCAS(p, old, __double_as_longlong(m));
            if (prev == old) break;
            old = prev;
        }
    };
    // leaves of one index are consecutive: most waves hold a single index
    const uint64_t act = __ballot(live);
    const uint32_t lead = (uint32_t)__shfl((int)i, __builtin_ctzll(act ? act : 1ull), kWave);
    if (act != 0 && __ballot(live && i == lead) == act) {
        ws = wave_sum(ws);
        loss = wave_sum(loss);
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double o = __shfl_xor(wmax, off, kWave);
            wmax = o > wmax ? o : wmax;
        }
        if ((threadIdx.x & (kWave - 1)) == 0) put(lead, ws, wmax, loss);
    } else if (live) {
        put(i, ws, wmax, loss);
    }
}

// With both root families: per index, the lower estimated lookup cost wins
// (a tie keeps the linear root); the final root and statistics.
__global__ void k_bt_choose(const TDesc *__restrict__ d, uint32_t count, const RootRec *__restrict__ best_lin,
                            const RootRec *__restrict__ best_sp, const double *__restrict__ st_lin,
                            const double *__restrict__ st_sp, RootRec *__restrict__ best, double *__restrict__ stats,
                            uint32_t *__restrict__ pick) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double n = (double)d[i].n;
    const bool sp = window_cost(st_sp[(uint64_t)i * NST] / n, true) < window_cost(st_lin[(uint64_t)i * NST] / n, false);
    pick[i] = sp ? 1u : 0u;
    best[i] = sp ? best_sp[i] : best_lin[i];
    for (int j = 0; j < NST; ++j) stats[(uint64_t)i * NST + j] = sp ? st_sp[(uint64_t)i * NST + j] : st_lin[(uint64_t)i * NST + j];
}

// Leaves trained under a chosen spline root replace the linear root's.
__global__ void k_bt_copy_leaves(const TDesc *__restrict__ d, uint32_t count, uint64_t total,
                                 const LeafRec *__restrict__ alt, const uint32_t *__restrict__ pick) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const uint32_t i = leaf_owner(d, count, g);
    if (pick[i]) d[i].leaves[g - d[i].leaf_off] = alt[g];
}

uint32_t blocks_for(uint64_t threads, uint32_t block) {
    uint64_t b = (threads + block - 1) / block;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) b = 0x7FFFFFFFull;
    return (uint32_t)b;
}

template <typename K>
int train_batch_t(idx_index *const *hs, uint32_t count, const uint32_t *leaves, uint32_t epochs, uint32_t feature,
                  hipStream_t s) {
    const bool want_lin = feature != IDX_FEATURE_SPLINE, want_sp = feature == IDX_FEATURE_AUTO ||
                                                                   feature == IDX_FEATURE_SPLINE;
    const bool both = want_lin && want_sp;
    std::vector<TDesc> desc(count), desc_alt;
    std::vector<Unit> units;
    std::vector<uint64_t> bin_off(count);
    uint64_t total_leaves = 0, total_bins = 0, total_keys = 0;
    uint32_t max_bins = 1;
    for (uint32_t i = 0; i < count; ++i) {
        const idx_index *h = hs[i];
        total_keys += h->n;
        desc[i] = TDesc{h->keys, h->n, h->learned->leaves, total_leaves, h->learned->spline, leaves[i], 0};
        total_leaves += leaves[i];
        bin_off[i] = total_bins;
        if (want_sp) {
            total_bins += spline_bins(h->n);
            max_bins = spline_bins(h->n) > max_bins ? spline_bins(h->n) : max_bins;
        }
        for (uint64_t b = 0; b < h->n; b += UNIT) units.push_back(Unit{b, b + UNIT < h->n ? b + UNIT : h->n, i, 0});
    }
    if (units.size() > 0x7FFFFFFFull) return IDX_ERR_ARG;
    const uint32_t nunits = (uint32_t)units.size();
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t b_desc = up(sizeof(TDesc) * count), b_units = up(sizeof(Unit) * nunits);
    const size_t b_roots = up(sizeof(RootRec) * NCAND * count), b_best = up(sizeof(RootRec) * count);
    const size_t b_racc = up(sizeof(double) * NCAND * NACC * count), b_stats = up(sizeof(double) * NST * count);
    const size_t b_lacc = up(sizeof(double) * NACC * total_leaves), b_cnt = up(sizeof(uint32_t) * total_leaves);
    const size_t b_bins = up(sizeof(SplineBin) * 2 * total_bins), b_src = up(sizeof(void *) * count);
    const size_t b_alt = both ? up(sizeof(LeafRec) * total_leaves) : 0, b_pick = up(sizeof(uint32_t) * count);
    const size_t b_flag = 256;
    const Alloc &A = hs[0]->alloc;
    const size_t total_b = 2 * b_desc + b_units + b_roots + 3 * b_best + b_racc + 3 * b_stats + b_lacc + b_cnt +
                           b_bins + b_src + b_alt + b_pick + b_flag;
    char *tmp = (char *)A.get(total_b, s);
    if (!tmp) return IDX_ERR_NOMEM;
    char *p = tmp;
    auto take = [&](size_t b) { char *q = p; p += b; return q; };
    TDesc *d_desc = (TDesc *)take(b_desc);
    TDesc *d_desc_alt = (TDesc *)take(b_desc);
    Unit *d_units = (Unit *)take(b_units);
    RootRec *d_roots = (RootRec *)take(b_roots);
    RootRec *d_best = (RootRec *)take(b_best);
    RootRec *d_best_lin = (RootRec *)take(b_best);
    RootRec *d_best_sp = (RootRec *)take(b_best);
    double *d_racc = (double *)take(b_racc);
    double *d_stats = (double *)take(b_stats);
    double *d_st_lin = (double *)take(b_stats);
    double *d_st_sp = (double *)take(b_stats);
    double *d_lacc = (double *)take(b_lacc);
    uint32_t *d_cnt = (uint32_t *)take(b_cnt);
    SplineBin *d_bins = (SplineBin *)take(b_bins);
    const SplineBin **d_src = (const SplineBin **)take(b_src);
    LeafRec *d_alt = (LeafRec *)take(b_alt);
    uint32_t *d_pick = (uint32_t *)take(b_pick);
    uint32_t *d_big = (uint32_t *)take(b_flag);  // a leaf larger than kLeafCap exists
    uint32_t cmask = 0;
    if (feature == IDX_FEATURE_AUTO) cmask = 15u;
    else if (feature == IDX_FEATURE_SPLINE) cmask = 12u;
    else cmask = 1u << (feature - 1);
    std::vector<RootRec> roots((size_t)NCAND * count);
    for (uint32_t i = 0; i < count; ++i) {
        for (int c = 0; c < NCAND; ++c) {
            RootRec R{};
            R.L = leaves[i];
            if (c < 2) {
                R.mode = c == 0 ? IDX_FEATURE_LINEAR : IDX_FEATURE_LOG;
            } else {
                R.mode = IDX_FEATURE_SPLINE;
                R.bfeat = c == 2 ? IDX_FEATURE_LINEAR : IDX_FEATURE_LOG;
                R.bins = d_bins + (c == 2 ? 0 : total_bins) + bin_off[i];
            }
            roots[(size_t)NCAND * i + c] = R;
        }
    }
    if (both) {
        desc_alt = desc;
        for (uint32_t i = 0; i < count; ++i) desc_alt[i].leaves = d_alt + desc[i].leaf_off;
    }
    std::vector<RootRec> best(count);
    std::vector<double> stats((size_t)NST * count);
    const uint32_t cap = stage_cap(total_keys, total_leaves);  // keys staged per workgroup of the leaf passes
    // the leaf stage under the roots `br` into the tables of `dd`, statistics
    // (entries 0-2) into `st`
    auto leaf_stage = [&](const TDesc *dd, const RootRec *br, double *st) {
        hipLaunchKernelGGL(k_bt_zero_u32, dim3(blocks_for(total_leaves, 256)), dim3(256), 0, s, d_cnt, total_leaves);
        hipLaunchKernelGGL((k_bt_leaf_count<K>), dim3(nunits), dim3(BT), 0, s, d_units, dd, br, d_cnt);
        hipLaunchKernelGGL((k_bt_leaf_layout<K>), dim3(count), dim3(1024), 0, s, dd, d_cnt);
        hipLaunchKernelGGL(k_bt_zero_u32, dim3(1), dim3(64), 0, s, d_big, (uint64_t)1);
        for (uint32_t ep = 0; ep <= epochs; ++ep) {
            hipLaunchKernelGGL((k_bt_leaf_accum_small<K>), dim3(blocks_for(total_leaves, kLeafBlock)), dim3(kLeafBlock),
                               (size_t)cap * sizeof(K), s, dd, count, total_leaves, d_lacc, d_big, cap);
            hipLaunchKernelGGL((k_bt_leaf_accum_big<K>), dim3(nunits), dim3(BT), 0, s, d_units, dd, br, d_lacc, d_big);
            if (ep < epochs)
                hipLaunchKernelGGL(k_bt_leaf_update, dim3(blocks_for(total_leaves, 256)), dim3(256), 0, s, dd, count,
                                   total_leaves, d_lacc);
        }
        hipLaunchKernelGGL((k_bt_leaf_errors_small<K>), dim3(blocks_for(total_leaves, kLeafBlock)), dim3(kLeafBlock),
                           (size_t)cap * sizeof(K), s, dd, count, total_leaves, cap);
        hipLaunchKernelGGL((k_bt_leaf_errors_big<K>), dim3(nunits), dim3(BT), 0, s, d_units, dd, br, d_big);
        hipLaunchKernelGGL(k_bt_leaf_finish, dim3(blocks_for(total_leaves, 256)), dim3(256), 0, s, dd, count,
                           total_leaves, d_lacc, st);
    };
    int rc = IDX_OK;
    do {
        if (hipMemcpyAsync(d_desc, desc.data(), sizeof(TDesc) * count, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d_units, units.data(), sizeof(Unit) * nunits, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d_roots, roots.data(), sizeof(RootRec) * NCAND * count, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            (both && hipMemcpyAsync(d_desc_alt, desc_alt.data(), sizeof(TDesc) * count, hipMemcpyHostToDevice, s) !=
                         hipSuccess)) {
            rc = IDX_ERR_HIP;
            break;
        }
        // ---- stage 1: root candidates -- the two linear roots take `epochs`
        // Newton steps, the two spline roots are built from the keys' ranks
        // -- and the final loss of each
        if (want_sp) {
            hipLaunchKernelGGL((k_bt_spline_geometry<K>), dim3(blocks_for(2ull * count, 256)), dim3(256), 0, s, d_desc,
                               d_roots, count, cmask);
            hipLaunchKernelGGL((k_bt_spline_bins<K>), dim3(count, (max_bins + 255) / 256, 2), dim3(256), 0, s, d_desc,
                               d_roots, cmask);
        }
        for (uint32_t ep = 0; ep <= epochs; ++ep) {
            hipLaunchKernelGGL(k_bt_zero, dim3(blocks_for((uint64_t)NCAND * NACC * count, 256)), dim3(256), 0, s,
                               d_racc, (uint64_t)NCAND * NACC * count);
            hipLaunchKernelGGL((k_bt_root_accum<K>), dim3(nunits), dim3(BT), 0, s, d_units, d_desc, d_roots, cmask,
                               d_racc);
            if (ep < epochs && (cmask & 3u))
                hipLaunchKernelGGL(k_bt_root_update, dim3(blocks_for(2ull * count, 256)), dim3(256), 0, s, d_roots,
                                   d_racc, count, cmask);
        }
        hipLaunchKernelGGL(k_bt_zero, dim3(blocks_for((uint64_t)NST * count, 256)), dim3(256), 0, s, d_st_lin,
                           (uint64_t)NST * count);
        hipLaunchKernelGGL(k_bt_zero, dim3(blocks_for((uint64_t)NST * count, 256)), dim3(256), 0, s, d_st_sp,
                           (uint64_t)NST * count);
        hipLaunchKernelGGL(k_bt_root_pick, dim3(blocks_for(count, 256)), dim3(256), 0, s, d_roots, d_racc, d_desc,
                           count, cmask, d_best_lin, d_best_sp, d_src, d_st_lin, d_st_sp);
        if (want_sp)
            hipLaunchKernelGGL(k_bt_copy_bins, dim3(count, (max_bins + 255) / 256), dim3(256), 0, s, d_best_sp, d_src);
        // ---- stage 2: leaves under each family's root; with both, the lower
        // estimated lookup cost wins per index
        RootRec *d_final = want_lin ? d_best_lin : d_best_sp;
        double *d_final_st = want_lin ? d_st_lin : d_st_sp;
        leaf_stage(d_desc, d_final, d_final_st);
        if (both) {
            leaf_stage(d_desc_alt, d_best_sp, d_st_sp);
            hipLaunchKernelGGL(k_bt_choose, dim3(blocks_for(count, 256)), dim3(256), 0, s, d_desc, count, d_best_lin,
                               d_best_sp, d_st_lin, d_st_sp, d_best, d_stats, d_pick);
            hipLaunchKernelGGL(k_bt_copy_leaves, dim3(blocks_for(total_leaves, 256)), dim3(256), 0, s, d_desc, count,
                               total_leaves, d_alt, d_pick);
            d_final = d_best;
            d_final_st = d_stats;
        }
        if (hipGetLastError() != hipSuccess) {
            rc = IDX_ERR_HIP;
            break;
        }
        if (hipMemcpyAsync(best.data(), d_final, sizeof(RootRec) * count, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(stats.data(), d_final_st, sizeof(double) * NST * count, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = IDX_ERR_HIP;
            break;
        }
    } while (0);
    A.put(tmp, s);
    if (rc != IDX_OK) return rc;
    for (uint32_t i = 0; i < count; ++i) {
        LearnedModel *M = hs[i]->learned;
        M->root = best[i];
        M->stats.leaves = leaves[i];
        M->stats.epochs = epochs;
        M->stats.feature = best[i].mode;
        M->stats.root_a0 = best[i].a0;
        M->stats.root_a1 = best[i].a1;
        M->stats.root_loss = stats[(size_t)i * NST + 3];
        M->stats.leaf_loss = stats[(size_t)i * NST + 2];
        M->stats.mean_window = stats[(size_t)i * NST + 0] / (double)hs[i]->n;
        M->stats.max_window = stats[(size_t)i * NST + 1];
        M->stats.segments = best[i].mode == IDX_FEATURE_SPLINE ? best[i].nb : 0;
        M->stats.bin_feature = best[i].mode == IDX_FEATURE_SPLINE ? best[i].bfeat : 0;
        if (best[i].mode != IDX_FEATURE_SPLINE && M->spline) {
            hs[i]->alloc.put(M->spline, s);
            M->spline = nullptr;
        }
    }
    return IDX_OK;
}

}  // namespace

int learn_batch(idx_index *const *hs, uint32_t count, const uint32_t *leaves, uint32_t epochs, uint32_t feature,
                hipStream_t s) {
    if (!hs || !leaves || count == 0 || epochs == 0 || epochs > 16 || feature > IDX_FEATURE_SPLINE) return IDX_ERR_ARG;
    std::unordered_set<const idx_index *> seen;
    for (uint32_t i = 0; i < count; ++i) {
        const idx_index *h = hs[i];
        if (!h || h->layout != IDX_BS || h->aos || h->n == 0 || h->u64 != hs[0]->u64) return IDX_ERR_ARG;
        if (leaves[i] == 0 || leaves[i] > (1u << 22)) return IDX_ERR_ARG;
        if (!seen.insert(h).second) return IDX_ERR_ARG;  // each index once
    }
    for (uint32_t i = 0; i < count; ++i) {
        idx_index *h = hs[i];
        drop_model(h, s);
        LearnedModel *M = new (std::nothrow) LearnedModel();
        if (M) M->leaves = (LeafRec *)h->alloc.get((size_t)leaves[i] * sizeof(LeafRec), s);
        if (M && M->leaves && (feature == IDX_FEATURE_AUTO || feature == IDX_FEATURE_SPLINE))
            M->spline = (SplineBin *)h->alloc.get((size_t)spline_bins(h->n) * sizeof(SplineBin), s);
        if (!M || !M->leaves || ((feature == IDX_FEATURE_AUTO || feature == IDX_FEATURE_SPLINE) && !M->spline)) {
            if (M && M->leaves) h->alloc.put(M->leaves, s);
            delete M;
            for (uint32_t j = 0; j < i; ++j) drop_model(hs[j], s);
            return IDX_ERR_NOMEM;
        }
        h->learned = M;
    }
    const int rc = hs[0]->u64 ? train_batch_t<uint64_t>(hs, count, leaves, epochs, feature, s)
                              : train_batch_t<uint32_t>(hs, count, leaves, epochs, feature, s);
    if (rc != IDX_OK)
        for (uint32_t i = 0; i < count; ++i) drop_model(hs[i], s);
    return rc;
}

}  // namespace idx
