// Batched point lookups on the three layouts (gfx950, wave64).
//
//  BS   lower-bound binary search on the sorted array (Section 3), branchless
//       with a fixed step count, then an equality test.
//  EBS  Eytzinger binary search (Section 3): from slot 1 go to 2i when the
//       key is >= the target, else 2i+1, until i exceeds n.  The lower-bound
//       slot is recovered from the final i by dropping its trailing right
//       turns and the last left turn (i >> (ctz(~i) + 1); Khuong and Morin,
//       "Array layouts for comparison-based searching", 2017).
//  EKS  Eytzinger k-ary search (Section 6.2).  (group): a group of lanes loads
//       one node's k-1 pivots with one coalesced access, a 64-bit wave ballot
//       masked to the group and a popcount give j = #pivots < target, the
//       search continues at node c*k + 1 + j (slot i*k + (j+1)(k-1)).
//       (single): one lane per lookup reads the whole node (vector loads when
//       the node is 16-byte aligned) and counts in registers.
//
// Every lane (or lane group) holds R independent lookups and advances them
// level by level together, so R dependent-load chains are in flight per lane.
// Optional cache pinning (Section 7.3) copies the top levels into LDS once per
// workgroup; with a persistent grid (Section 7.2, limited concurrency) the
// copy is amortised over many tiles.  The lower bound is tracked during the
// descent (deepest candidate), so only the row ID needs one more load.
// Queries enter and answers leave through qio.hpp (plain, locally sorted per
// tile, or a batch partitioned by rank bucket with XCD-contiguous tiles).
#include <type_traits>

#include "internal.hpp"
#include "access.hpp"
#include "qio.hpp"
#include "search.hpp"

namespace idx {
namespace {

template <typename K, bool AOS>
struct PointArgs {
    Load<K, AOS> L;
    Geo G;
    QueryIO<K> io;
    const K *__restrict__ pin;
    uint32_t pin_entries;
    uint32_t pin_levels;
    uint32_t early;     // stop at an equal key (unique keys only)
    uint32_t bs_iters;  // binary-search steps over n keys
};

// Cooperative copy of the pin table into LDS.
template <typename K>
__device__ __forceinline__ void load_pin(K *s_pin, const K *__restrict__ pin, uint32_t count) {
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) s_pin[i] = pin[i];
    __syncthreads();
}

// ----------------------------------------------------------------------- BS

template <typename K, bool AOS, int R, bool SORT>
__global__ __launch_bounds__(1024) void k_point_bs(PointArgs<K, AOS> a) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    if (a.pin_levels) load_pin(s_pin, a.pin, a.pin_entries);
    const uint64_t n = a.G.n;
    const uint64_t tile = (uint64_t)blockDim.x * R;
    for (uint64_t it = blockIdx.x; it < a.io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, a.io.ntiles, a.io.xcd);
        if (tl >= a.io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R];
        uint32_t src[R];
        tile_load<K, R, SORT>(a.io, smem, t0, x, src);
        uint64_t base[R];
#pragma unroll
        for (int r = 0; r < R; ++r) base[r] = 0;
        uint64_t len = n;
        if (!SORT && a.io.bkt) {
            // partitioned batch: each lookup's bucket bounds its lower bound,
            // so the search starts inside that bucket's rank interval (the
            // steps above it are the same for the whole bucket)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t qi = t0 + src_of<R, SORT>(src, r);
                base[r] = qi < a.io.m ? bucket_start(a.io.bkt[qi], a.io.bstep) : 0;
            }
            len = a.io.bspan;
        } else if (a.pin_levels) {
            uint32_t v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = 1;
            for (uint32_t d = 0; d < a.pin_levels; ++d) {
                const uint64_t half = len >> 1;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool go = s_pin[v[r]] < x[r];
                    base[r] += go ? half : 0;
                    v[r] = 2 * v[r] + (go ? 1u : 0u);
                }
                len -= half;
            }
        }
        // SoA: stop the dependent probes at a window of at most 15 keys and
        // read it (plus the key after it) with independent 16-byte loads
        const uint64_t stop = AOS ? 1 : 15;
        while (len > stop) {
            const uint64_t half = len >> 1;
#pragma unroll
            for (int r = 0; r < R; ++r) base[r] = (a.L.key(base[r] + half) < x[r]) ? base[r] + half : base[r];
            len -= half;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t res = kMiss;
            if (n > 0 && tile_valid(a.io.m, t0, src_of<R, SORT>(src, r))) {
                if constexpr (!AOS) {
                    const uint64_t sl = (len + 1) < (n - base[r]) ? (len + 1) : (n - base[r]);
                    bool eq;
                    const uint32_t c = count_below<K, 16>(a.L.k, base[r], (uint32_t)sl, x[r], eq, a.io.rounds == 2);
                    if (eq) res = a.L.row(base[r] + c);
                } else {
                    const K kb = a.L.key(base[r]);
                    const uint64_t pos = base[r] + (kb < x[r] ? 1 : 0);
                    if (pos < n) {
                        const K kp = kb < x[r] ? a.L.key(pos) : kb;
                        if (kp == x[r]) res = a.L.row(pos);
                    }
                }
            }
            tile_put<K, SORT>(a.io, smem, t0, src_of<R, SORT>(src, r), res);
        }
        tile_flush<K, R, SORT>(a.io, smem, t0);
    }
}

// ---------------------------------------------------------------------- EBS

template <typename K, bool AOS, int R, bool SORT>
__global__ __launch_bounds__(1024) void k_point_ebs(PointArgs<K, AOS> a) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    if (a.pin_levels) load_pin(s_pin, a.pin, a.pin_entries);
    const uint64_t n = a.G.n;
    const uint32_t m_full = a.G.m;
    const uint64_t tile = (uint64_t)blockDim.x * R;
    for (uint64_t it = blockIdx.x; it < a.io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, a.io.ntiles, a.io.xcd);
        if (tl >= a.io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R], ck[R];
        uint32_t src[R];
        uint64_t i[R];
        tile_load<K, R, SORT>(a.io, smem, t0, x, src);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            i[r] = 1;
            ck[r] = key_max<K>();
        }
        uint32_t lvl = 0;
        for (; lvl < a.pin_levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const K kk = s_pin[i[r]];
                const bool right = kk < x[r];
                ck[r] = right ? ck[r] : kk;
                i[r] = 2 * i[r] + (right ? 1 : 0);
            }
        }
        for (; lvl < m_full; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const K kk = a.L.key(i[r]);
                const bool right = kk < x[r];
                ck[r] = right ? ck[r] : kk;
                i[r] = 2 * i[r] + (right ? 1 : 0);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (i[r] <= n) {
                const K kk = a.L.key(i[r]);
                const bool right = kk < x[r];
                ck[r] = right ? ck[r] : kk;
                i[r] = 2 * i[r] + (right ? 1 : 0);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t j = i[r] >> (__builtin_ctzll(~i[r]) + 1);
            const uint32_t res = (tile_valid(a.io.m, t0, src_of<R, SORT>(src, r)) && j != 0 && ck[r] == x[r]) ? a.L.row(j) : kMiss;
            tile_put<K, SORT>(a.io, smem, t0, src_of<R, SORT>(src, r), res);
        }
        tile_flush<K, R, SORT>(a.io, smem, t0);
    }
}

// --------------------------------------------------------------- EKS group

// GL lanes per lookup (a power of two >= k-1); 64/GL lookups per wave per
// register slot; R register slots.
template <typename K, bool AOS, int GL, int R>
__global__ __launch_bounds__(1024) void k_point_eks_group(PointArgs<K, AOS> a) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    if (a.pin_levels) load_pin(s_pin, a.pin, a.pin_entries);
    constexpr int GPW = kWave / GL;  // groups per wave
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t sub = lane & (GL - 1);
    const uint32_t grp = lane / GL;
    const uint64_t gmask = (GL == kWave) ? ~0ull : (((1ull << GL) - 1ull) << (grp * GL));
    const uint64_t n = a.G.n;
    const uint32_t g = a.G.g;
    const uint32_t kf = a.G.k;
    const bool lane_ok = sub < g;
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t tile = (uint64_t)waves * GPW * R;
    for (uint64_t it = blockIdx.x; it < a.io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, a.io.ntiles, a.io.xcd);
        if (tl >= a.io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        const uint64_t wbase = t0 + (uint64_t)wave * GPW * R;
        K x[R];
        uint64_t c[R], cand[R];
        bool ceq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t qi = wbase + (uint64_t)r * GPW + grp;
            x[r] = qi < a.io.m ? a.io.q[qi] : K(0);
            c[r] = qi < a.io.m ? 0 : ~0ull;  // node index; ~0 = finished
            cand[r] = 0;
            ceq[r] = false;
        }
        for (uint32_t lvl = 0; lvl < a.G.levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool live = c[r] != ~0ull;
                const uint64_t i = live ? c[r] * g : n;  // node's first slot
                const uint64_t s = i + sub;
                const bool valid = live && lane_ok && s < n;
                K kk = key_max<K>();
                if (valid) kk = (lvl < a.pin_levels) ? s_pin[s] : a.L.nkey(c[r], sub);
                const uint64_t lt = __ballot(valid && kk < x[r]) & gmask;
                const uint64_t eq = __ballot(valid && kk == x[r]) & gmask;
                const uint32_t j = (uint32_t)__popcll(lt);
                if (live) {
                    const uint64_t nv = (n - i) < g ? (n - i) : g;  // pivots present in the node
                    if (j < nv) {
                        cand[r] = i + j;
                        ceq[r] = eq != 0;
                    }
                    const uint64_t child = c[r] * kf + 1 + j;
                    const bool stop = (a.early && eq != 0) || child * g >= n;
                    c[r] = stop ? ~0ull : child;
                }
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t qi = wbase + (uint64_t)r * GPW + grp;
                if (qi < a.io.m) a.io.out[a.io.pos ? a.io.pos[qi] : qi] = ceq[r] ? a.L.row(cand[r]) : kMiss;
            }
        }
    }
}

// --------------------------------------------------------- EKS vector group

// VG lanes per lookup, each lane reading V = 16 / sizeof(K) consecutive
// pivots with one 16-byte load, so a node of up to VG*V pivots arrives with
// one load instruction per lane group (a 64-byte node of 8 u64 keys: 4 lanes).
// j = sum over the V key positions of popcount(ballot(key_e < x) & group).
// Requires 16-byte aligned nodes (k-1 a multiple of V; AoS blocks too).
template <typename K, bool AOS, int VG, int R>
__global__ __launch_bounds__(1024) void k_point_eks_vgroup(PointArgs<K, AOS> a) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    if (a.pin_levels) load_pin(s_pin, a.pin, a.pin_entries);
    constexpr int V = 16 / sizeof(K);
    constexpr int GPW = kWave / VG;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t sub = lane & (VG - 1);
    const uint32_t grp = lane / VG;
    const uint64_t gmask = (VG == kWave) ? ~0ull : (((1ull << VG) - 1ull) << (grp * VG));
    const uint64_t n = a.G.n;
    const uint32_t g = a.G.g;
    const uint32_t kf = a.G.k;
    const uint32_t first = sub * V;  // first pivot of this lane within the node
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t tile = (uint64_t)waves * GPW * R;
    for (uint64_t it = blockIdx.x; it < a.io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, a.io.ntiles, a.io.xcd);
        if (tl >= a.io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        const uint64_t wbase = t0 + (uint64_t)wave * GPW * R;
        K x[R];
        uint64_t c[R], cand[R];
        bool ceq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t qi = wbase + (uint64_t)r * GPW + grp;
            x[r] = qi < a.io.m ? a.io.q[qi] : K(0);
            c[r] = qi < a.io.m ? 0 : ~0ull;
            cand[r] = 0;
            ceq[r] = false;
        }
        for (uint32_t lvl = 0; lvl < a.G.levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool live = c[r] != ~0ull;
                const uint64_t i = live ? c[r] * g : n;
                const bool lane_live = live && first < g && i + first < n;
                K kk[V];
#pragma unroll
                for (int e = 0; e < V; ++e) kk[e] = key_max<K>();
                if (lane_live) {
                    uint4 w;
                    if (lvl < a.pin_levels) w = *(const uint4 *)(s_pin + i + first);
                    else w = *(const uint4 *)(a.L.node_ptr(c[r]) + first);
                    if constexpr (sizeof(K) == 8) {
                        kk[0] = ((uint64_t)w.y << 32) | w.x;
                        kk[1] = ((uint64_t)w.w << 32) | w.z;
                    } else {
                        kk[0] = w.x;
                        kk[1] = w.y;
                        kk[2] = w.z;
                        kk[3] = w.w;
                    }
                }
                uint32_t j = 0;
                bool eql = false;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const bool valid = lane_live && first + e < g && i + first + e < n;
                    j += (uint32_t)__popcll(__ballot(valid && kk[e] < x[r]) & gmask);
                    eql |= valid && kk[e] == x[r];
                }
                const uint64_t eq = __ballot(eql) & gmask;
                if (live) {
                    const uint64_t nv = (n - i) < g ? (n - i) : g;
                    if (j < nv) {
                        cand[r] = i + j;
                        ceq[r] = eq != 0;
                    }
                    const uint64_t child = c[r] * kf + 1 + j;
                    const bool stop = (a.early && eq != 0) || child * g >= n;
                    c[r] = stop ? ~0ull : child;
                }
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t qi = wbase + (uint64_t)r * GPW + grp;
                if (qi < a.io.m) a.io.out[a.io.pos ? a.io.pos[qi] : qi] = ceq[r] ? a.L.row(cand[r]) : kMiss;
            }
        }
    }
}

// -------------------------------------------------------------- EKS single

// One lane per lookup.  GMAX = pivots read per node (>= k-1); VEC = nodes are
// exactly GMAX keys, 16-byte aligned, read with 16-byte loads (SoA only).
template <typename K, bool AOS, int GMAX, bool VEC, int R, bool SORT>
__global__ __launch_bounds__(1024) void k_point_eks_single(PointArgs<K, AOS> a) {
    extern __shared__ __align__(16) char smem[];
    K *s_pin = (K *)smem;
    if (a.pin_levels) load_pin(s_pin, a.pin, a.pin_entries);
    const uint64_t n = a.G.n;
    const uint32_t g = a.G.g;
    const uint32_t kf = a.G.k;
    const uint64_t tile = (uint64_t)blockDim.x * R;
    for (uint64_t it = blockIdx.x; it < a.io.iters; it += gridDim.x) {
        const uint64_t tl = tile_of(it, a.io.ntiles, a.io.xcd);
        if (tl >= a.io.ntiles) continue;
        const uint64_t t0 = tl * tile;
        K x[R];
        uint32_t src[R];
        uint64_t c[R], cand[R];
        bool ceq[R];
        tile_load<K, R, SORT>(a.io, smem, t0, x, src);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            c[r] = tile_valid(a.io.m, t0, src_of<R, SORT>(src, r)) ? 0 : ~0ull;
            cand[r] = 0;
            ceq[r] = false;
        }
        for (uint32_t lvl = 0; lvl < a.G.levels; ++lvl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (c[r] == ~0ull) continue;
                const uint64_t i = c[r] * g;
                const uint64_t nv = (n - i) < g ? (n - i) : g;
                K kk[GMAX];
                if (lvl < a.pin_levels) {
#pragma unroll
                    for (int e = 0; e < GMAX; ++e) kk[e] = (e < (int)nv) ? s_pin[i + e] : key_max<K>();
                } else if constexpr (VEC) {
                    // full node of GMAX keys, 16-byte aligned; partial last node
                    // reads stay inside the padded allocation and are masked
                    constexpr int W = 16 / sizeof(K);
                    const uint4 *p = (const uint4 *)a.L.node_ptr(c[r]);
#pragma unroll
                    for (int v = 0; v < GMAX / W; ++v) {
                        const uint4 w = p[v];
                        if constexpr (sizeof(K) == 8) {
                            kk[2 * v] = ((uint64_t)w.y << 32) | w.x;
                            kk[2 * v + 1] = ((uint64_t)w.w << 32) | w.z;
                        } else {
                            kk[4 * v] = w.x;
                            kk[4 * v + 1] = w.y;
                            kk[4 * v + 2] = w.z;
                            kk[4 * v + 3] = w.w;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < GMAX; ++e)
                        if (e >= (int)nv) kk[e] = key_max<K>();
                } else {
#pragma unroll
                    for (int e = 0; e < GMAX; ++e) kk[e] = (e < (int)nv) ? a.L.nkey(c[r], e) : key_max<K>();
                }
                uint32_t j = 0;
                bool eq = false;
#pragma unroll
                for (int e = 0; e < GMAX; ++e) {
                    j += (e < (int)nv && kk[e] < x[r]) ? 1u : 0u;
                    eq |= (e < (int)nv && kk[e] == x[r]);
                }
                if (j < nv) {
                    cand[r] = i + j;
                    ceq[r] = eq;
                }
                const uint64_t child = c[r] * kf + 1 + j;
                c[r] = ((a.early && eq) || child * g >= n) ? ~0ull : child;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) tile_put<K, SORT>(a.io, smem, t0, src_of<R, SORT>(src, r), ceq[r] ? a.L.row(cand[r]) : kMiss);
        tile_flush<K, R, SORT>(a.io, smem, t0);
    }
}

// ---------------------------------------------------------------- dispatch

template <typename K, bool AOS>
PointArgs<K, AOS> make_args(const idx_index *h, const PointIO &io, uint32_t pin_levels, bool early) {
    PointArgs<K, AOS> a{};
    a.L = make_load<K, AOS>(h);
    a.G = h->geo;
    a.io.q = (const K *)io.q;
    a.io.out = io.out;
    a.io.m = io.m;
    a.io.local_sort = io.local_sort ? 1u : 0u;
    a.io.xcd = io.xcd ? 1u : 0u;
    a.io.rounds = h->params.window_rounds == 1 ? 1u : 2u;
    a.io.pos = io.pos;
    a.io.bkt = io.bkt;
    a.io.bstep = io.bstep;
    a.io.bspan = io.bspan;
    a.pin = (const K *)h->pin;
    a.pin_entries = pin_levels ? h->pin_keys : 0;
    a.pin_levels = pin_levels;
    a.early = early ? 1u : 0u;
    a.bs_iters = 0;
    return a;
}

struct Launch {
    uint32_t grid, block;
    size_t smem;
};

// Grid, block and LDS of a launch whose workgroups each take tiles of
// `lookups_per_block`; fills the tile walk of `io`.
template <typename K>
Launch plan(const idx_index *h, const idx_lookup_params &p, QueryIO<K> &io, uint64_t lookups_per_block) {
    Launch L{};
    L.block = p.block;
    const size_t pin_bytes = p.lds_levels ? (size_t)h->pin_keys * (h->u64 ? 8 : 4) : 0;
    io.sort_off = (uint32_t)((pin_bytes + 15) & ~(size_t)15);
    L.smem = io.local_sort ? io.sort_off + sort_lds_bytes((uint32_t)lookups_per_block, sizeof(K)) : pin_bytes;
    set_tiles(io, lookups_per_block);
    uint64_t grid = io.iters;
    if (p.persistent) {
        uint64_t cap = (uint64_t)h->cu_count * p.persistent;
        // a persistent grid that is a multiple of the XCD count keeps every
        // workgroup on one XCD's share of the tiles
        if (io.xcd && cap >= kXcds) cap -= cap % kXcds;
        if (grid > cap) grid = cap;
    }
    if (grid > 0x7FFFFFFFull) grid = 0x7FFFFFFFull;
    L.grid = (uint32_t)(grid ? grid : 1);
    return L;
}

template <typename K, bool AOS, int R>
int run_bs(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    auto a = make_args<K, AOS>(h, io, p.lds_levels, false);
    const Launch L = plan(h, p, a.io, (uint64_t)p.block * R);
    if (a.io.local_sort)
        hipLaunchKernelGGL((k_point_bs<K, AOS, R, true>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    else
        hipLaunchKernelGGL((k_point_bs<K, AOS, R, false>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS, int R>
int run_ebs(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    auto a = make_args<K, AOS>(h, io, p.lds_levels, false);
    const Launch L = plan(h, p, a.io, (uint64_t)p.block * R);
    if (a.io.local_sort)
        hipLaunchKernelGGL((k_point_ebs<K, AOS, R, true>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    else
        hipLaunchKernelGGL((k_point_ebs<K, AOS, R, false>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS, int GL, int R>
int run_group(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    auto a = make_args<K, AOS>(h, io, p.lds_levels, p.early_exit == 1 && h->unique);
    const Launch L = plan(h, p, a.io, (uint64_t)(p.block / kWave) * (kWave / GL) * R);
    hipLaunchKernelGGL((k_point_eks_group<K, AOS, GL, R>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS, int VG, int R>
int run_vgroup(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    auto a = make_args<K, AOS>(h, io, p.lds_levels, p.early_exit == 1 && h->unique);
    const Launch L = plan(h, p, a.io, (uint64_t)(p.block / kWave) * (kWave / VG) * R);
    hipLaunchKernelGGL((k_point_eks_vgroup<K, AOS, VG, R>), dim3(L.grid), dim3(L.block), L.smem, s, a);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <typename K, bool AOS, int GMAX, int R>
int run_single(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    auto a = make_args<K, AOS>(h, io, p.lds_levels, p.early_exit == 1 && h->unique);
    const Launch L = plan(h, p, a.io, (uint64_t)p.block * R);
    // 16-byte node loads need 16-byte aligned nodes: SoA nodes of GMAX keys,
    // or AoS blocks whose stride is a multiple of 16
    constexpr bool vec_ok = (GMAX * sizeof(K)) % 16 == 0;
    const bool vec = vec_ok && h->geo.g == GMAX && (!AOS || h->stride % 16 == 0);
    if (vec && a.io.local_sort)
        hipLaunchKernelGGL((k_point_eks_single<K, AOS, GMAX, vec_ok, R, true>), dim3(L.grid), dim3(L.block), L.smem, s,
                           a);
    else if (vec)
        hipLaunchKernelGGL((k_point_eks_single<K, AOS, GMAX, vec_ok, R, false>), dim3(L.grid), dim3(L.block), L.smem, s,
                           a);
    else if (a.io.local_sort)
        hipLaunchKernelGGL((k_point_eks_single<K, AOS, GMAX, false, R, true>), dim3(L.grid), dim3(L.block), L.smem, s,
                           a);
    else
        hipLaunchKernelGGL((k_point_eks_single<K, AOS, GMAX, false, R, false>), dim3(L.grid), dim3(L.block), L.smem, s,
                           a);
    IDX_LAUNCH_CHECK();
    return IDX_OK;
}

template <int R, typename F>
int with_r(uint32_t r, F &&f) {
    switch (r) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return IDX_ERR_ARG;
    }
}

template <typename K, bool AOS>
int point_t(const idx_index *h, const idx_lookup_params &p, const PointIO &io, hipStream_t s) {
    if (h->layout == IDX_BS)
        return with_r<0>(p.per_lane, [&](auto R) { return run_bs<K, AOS, decltype(R)::value>(h, p, io, s); });
    if (h->layout == IDX_EBS)
        return with_r<0>(p.per_lane, [&](auto R) { return run_ebs<K, AOS, decltype(R)::value>(h, p, io, s); });
    if (p.group <= 1) {
        const uint32_t g = h->geo.g;
        return with_r<0>(p.per_lane, [&](auto R) {
            constexpr int RR = decltype(R)::value;
            if (g <= 4) return run_single<K, AOS, 4, RR>(h, p, io, s);
            if (g <= 8) return run_single<K, AOS, 8, RR>(h, p, io, s);
            if (g <= 16) return run_single<K, AOS, 16, RR>(h, p, io, s);
            return run_single<K, AOS, 32, RR>(h, p, io, s);
        });
    }
    if (p.group < h->geo.g) {
        return with_r<0>(p.per_lane, [&](auto R) {
            constexpr int RR = decltype(R)::value;
            switch (p.group) {
                case 2: return run_vgroup<K, AOS, 2, RR>(h, p, io, s);
                case 4: return run_vgroup<K, AOS, 4, RR>(h, p, io, s);
                case 8: return run_vgroup<K, AOS, 8, RR>(h, p, io, s);
                case 16: return run_vgroup<K, AOS, 16, RR>(h, p, io, s);
                case 32: return run_vgroup<K, AOS, 32, RR>(h, p, io, s);
                default: return IDX_ERR_ARG;
            }
        });
    }
    return with_r<0>(p.per_lane, [&](auto R) {
        constexpr int RR = decltype(R)::value;
        switch (p.group) {
            case 2: return run_group<K, AOS, 2, RR>(h, p, io, s);
            case 4: return run_group<K, AOS, 4, RR>(h, p, io, s);
            case 8: return run_group<K, AOS, 8, RR>(h, p, io, s);
            case 16: return run_group<K, AOS, 16, RR>(h, p, io, s);
            case 32: return run_group<K, AOS, 32, RR>(h, p, io, s);
            case 64: return run_group<K, AOS, 64, RR>(h, p, io, s);
            default: return IDX_ERR_ARG;
        }
    });
}

uint32_t pow2_at_least(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

int resolve_params(const idx_index *h, const idx_lookup_params *in, idx_lookup_params *out) {
    idx_lookup_params p{};
    if (in) p = *in;
    const uint32_t g = h->layout == IDX_EKS ? h->geo.g : 1;
    if (h->layout == IDX_EKS) {
        // lanes per lookup: 1 = single; >= k-1 = one pivot per lane; fewer =
        // 16-byte pivot chunks per lane (vector group)
        const uint32_t V = 16 / (h->u64 ? 8 : 4);
        const bool vec_ok = g % V == 0 && (!h->aos || h->stride % 16 == 0);
        const uint32_t vg = pow2_at_least((g + V - 1) / V);
        // Default (measured on MI355X): one lane per lookup reading the node
        // with 16-byte loads when the node is at most 64 bytes and aligned;
        // otherwise 16-byte chunks over a lane group; otherwise one pivot per lane.
        const uint32_t node_bytes = g * (h->u64 ? 8 : 4);
        const bool single_vec = (!h->aos || h->stride % 16 == 0) && node_bytes % 16 == 0 && node_bytes <= 64;
        if (p.group == 0) p.group = single_vec ? 1 : (vec_ok && vg < g) ? vg : pow2_at_least(g);
        if (p.group > 64 || (p.group & (p.group - 1))) return IDX_ERR_ARG;
        if (p.group != 1 && p.group < g && !(vec_ok && p.group >= vg && p.group <= 32)) return IDX_ERR_ARG;
        // EKS (single) keeps a whole node in registers: at most 32 pivots
        if (p.group == 1 && g > 32) return IDX_ERR_ARG;
    } else {
        p.group = 1;
    }
    if (p.block == 0) p.block = 256;
    if (p.block < 64 || p.block > 1024 || (p.block & (p.block - 1))) return IDX_ERR_ARG;
    if (p.per_lane == 0) p.per_lane = (h->layout == IDX_EKS && p.group > 1) ? 2 : 4;
    if (p.per_lane != 1 && p.per_lane != 2 && p.per_lane != 4 && p.per_lane != 8) return IDX_ERR_ARG;
    // cache pinning: at most 64 KiB of LDS and only complete levels
    const size_t kb = h->u64 ? 8 : 4;
    const uint32_t max_levels = pin_levels_for(h, 64 * 1024);
    if (p.lds_levels > max_levels) return IDX_ERR_ARG;
    if (p.persistent > 64) return IDX_ERR_ARG;
    // lookup reordering: 0 = none; 1 = sort each tile of block * per_lane
    // lookups in LDS (one lookup per lane only); 2 = partition the batch by
    // rank bucket first, answers returned by two counting passes; 3 = the
    // same partition, each answer written straight to its position
    if (p.reorder > 3) return IDX_ERR_ARG;
    if (p.reorder == 1) {
        const uint64_t T = (uint64_t)p.block * p.per_lane;
        if (p.group > 1 || T > kMaxSortTile) return IDX_ERR_ARG;
        const size_t pin_bytes = p.lds_levels ? (((size_t)pin_entries_for(h, p.lds_levels) * kb + 15) & ~(size_t)15) : 0;
        if (pin_bytes + sort_lds_bytes((uint32_t)T, kb) > h->lds_max) return IDX_ERR_ARG;
    }
    // early exit: 0 = default (on), 1 = on, 2 = off; only effective for unique keys
    if (p.early_exit == 0) p.early_exit = 1;
    if (p.early_exit > 2) return IDX_ERR_ARG;
    if (p.model > 2) return IDX_ERR_ARG;
    // short-window scan: 0 = default (two rounds), 1 = one round, 2 = two rounds
    if (p.window_rounds == 0) p.window_rounds = 2;
    if (p.window_rounds > 2) return IDX_ERR_ARG;
    // Eytzinger range fill: 0 = default (gather by rank), 1 = hybrid level
    // scan, 2 = single-lane level scan, 3 = gather by rank
    if (p.range_scan == 0) p.range_scan = 3;
    if (p.range_scan > 3) return IDX_ERR_ARG;
    // learned form: 0 = default (off), 1 = one line per leaf, 2 = off
    if (p.leaf_lines == 0) p.leaf_lines = 2;
    if (p.leaf_lines > 2) return IDX_ERR_ARG;
    *out = p;
    return IDX_OK;
}

int point_run(idx_index *h, const PointIO &io, hipStream_t s) {
    const idx_lookup_params &p = h->params;
    if (h->learned && p.model != 2) return point_learned(h, io, s);
    if (p.lds_levels) {
        const int rc = build_pin(h, p.lds_levels, s);
        if (rc != IDX_OK) return rc;
    }
    if (h->u64) return h->aos ? point_t<uint64_t, true>(h, p, io, s) : point_t<uint64_t, false>(h, p, io, s);
    return h->aos ? point_t<uint32_t, true>(h, p, io, s) : point_t<uint32_t, false>(h, p, io, s);
}

int point_lookup(idx_index *h, const void *q, uint64_t m, uint32_t *out, hipStream_t s) {
    if (m == 0) return IDX_OK;
    if (h->params.reorder >= 2) return point_partitioned(h, q, m, out, s);
    PointIO io{q, m, out, h->params.reorder == 1, false};
    return point_run(h, io, s);
}

}  // namespace idx
