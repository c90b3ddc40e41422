// Stable LSD radix sort of (key, rowid) pairs by key -- the build step of the
// sorted-array index (Section 3: BS is a key-value sort; Section 8.5: the
// sort dominates build time).  gfx950, wave64.
//
// One pass per 8-bit digit, three kernels per pass (reduce-then-scan; no
// inter-workgroup waiting anywhere):
//   1. tile histogram: each workgroup counts the digits of its 4096-key tile;
//   2. digit scan: one workgroup per digit turns the per-tile counts into
//      exclusive offsets and a digit total;
//   3. scatter: each workgroup ranks its tile stably (wave-level ballot
//      "peer" masks, items taken in index order), stages the tile in LDS in
//      digit order and writes every digit run out contiguously.
// A first kernel histograms every digit position at once; passes whose digit
// is the same for all keys are skipped (a host read, the sort's only sync).
#include "internal.hpp"

namespace idx {
namespace {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / kWave;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // 4096 keys
constexpr int RS_SCAN_ITEMS = 16;
constexpr uint32_t RS_XCDS = 8;  // workgroups are dealt round-robin over the 8 XCDs

// The tile that workgroup b scatters: XCD x (b % 8) takes a contiguous share
// of the tiles, in order.  A digit's runs from consecutive tiles are adjacent
// in the output, so the partial 128 B lines at their ends are completed in
// one XCD's L2 instead of being written back in pieces from several.
// A bijection of [0, tiles): XCD x holds tiles/8 + (x < tiles%8) workgroups.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t tiles) {
    const uint32_t per = tiles / RS_XCDS, rem = tiles % RS_XCDS;
    const uint32_t x = b % RS_XCDS, i = b / RS_XCDS;
    return x * per + (x < rem ? x : rem) + i;
}

static_assert(RS_THREADS == RS_BINS, "one thread per digit value in the scan phases");

// Exclusive scan of one value per thread across a 256-thread workgroup.
// Returns the exclusive prefix; *total receives the workgroup sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_wave, uint32_t *total) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, kWave);
        if (lane >= (uint32_t)off) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        const uint32_t c = s_wave[w];
        before += (w < (int)wave) ? c : 0;
        sum += c;
    }
    __syncthreads();
    *total = sum;
    return before + incl - v;
}

template <typename K>
__global__ __launch_bounds__(RS_THREADS) void k_global_hist(const K *__restrict__ keys, uint64_t n, int passes,
                                                            uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[8 * RS_BINS];
    for (int i = threadIdx.x; i < passes * RS_BINS; i += RS_THREADS) h[i] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * RS_THREADS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * RS_THREADS) {
        const K key = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p * RS_BINS + ((key >> (p * RS_BITS)) & (RS_BINS - 1))], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * RS_BINS; i += RS_THREADS)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

template <typename K>
__global__ __launch_bounds__(RS_THREADS) void k_tile_hist(const K *__restrict__ keys, uint64_t n, int shift,
                                                          uint32_t *__restrict__ tile_hist, uint32_t tiles) {
    __shared__ uint32_t h[RS_WAVES][RS_BINS];
    const uint32_t wave = threadIdx.x / kWave;
    for (int w = 0; w < RS_WAVES; ++w) h[w][threadIdx.x] = 0;
    __syncthreads();
    // XCD-contiguous tiles, as in the scatter: the per-digit counts of
    // neighbouring tiles share lines of tile_hist.
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint64_t base = (uint64_t)tile * RS_TILE;
    // all of a thread's keys are loaded before the first LDS atomic, so the
    // 16 loads are in flight together
    K kk[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * RS_THREADS + threadIdx.x;
        kk[j] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[wave][(kk[j] >> shift) & (RS_BINS - 1)], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) c += h[w][threadIdx.x];
    tile_hist[(uint64_t)threadIdx.x * tiles + tile] = c;
}

// One workgroup per digit: exclusive scan of that digit's per-tile counts
// (in place) and the digit's total.
__global__ __launch_bounds__(RS_THREADS) void k_digit_scan(uint32_t *__restrict__ tile_hist, uint32_t tiles,
                                                           uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t s_wave[RS_WAVES];
    uint32_t *row = tile_hist + (uint64_t)blockIdx.x * tiles;
    uint32_t running = 0;
    for (uint32_t chunk = 0; chunk < tiles; chunk += RS_THREADS * RS_SCAN_ITEMS) {
        uint32_t v[RS_SCAN_ITEMS];
        uint32_t sum = 0;
        const uint32_t first = chunk + threadIdx.x * RS_SCAN_ITEMS;
#pragma unroll
        for (int j = 0; j < RS_SCAN_ITEMS; ++j) {
            v[j] = (first + j < tiles) ? row[first + j] : 0u;
            sum += v[j];
        }
        uint32_t total;
        uint32_t acc = running + block_exclusive_scan(sum, s_wave, &total);
#pragma unroll
        for (int j = 0; j < RS_SCAN_ITEMS; ++j) {
            if (first + j < tiles) row[first + j] = acc;
            acc += v[j];
        }
        running += total;
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = running;
}

template <typename K>
struct ScatterSmem {
    K keys[RS_TILE];
    uint32_t rows[RS_TILE];
    uint32_t wave_cnt[RS_WAVES][RS_BINS];
    uint32_t digit_start[RS_BINS];
    uint32_t global_base[RS_BINS];
    uint32_t scan_tmp[RS_WAVES];
};

template <typename K>
__global__ __launch_bounds__(RS_THREADS) void k_scatter(const K *__restrict__ keys_in,
                                                        const uint32_t *__restrict__ rows_in,
                                                        K *__restrict__ keys_out, uint32_t *__restrict__ rows_out,
                                                        uint64_t n, int shift,
                                                        const uint32_t *__restrict__ tile_hist, uint32_t tiles,
                                                        const uint32_t *__restrict__ digit_total) {
    __shared__ ScatterSmem<K> sm;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    for (int w = 0; w < RS_WAVES; ++w) sm.wave_cnt[w][threadIdx.x] = 0;

    // Items of a wave are consecutive keys: item j of lane l is key
    // base + j*64 + l, so taking items j = 0, 1, ... with lanes in order
    // visits the wave's keys in index order (stability).
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint64_t tile_base = (uint64_t)tile * RS_TILE;
    const uint64_t wave_base = tile_base + (uint64_t)wave * (RS_ITEMS * kWave);
    K key[RS_ITEMS];
    uint32_t row[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const uint64_t i = wave_base + (uint64_t)j * kWave + lane;
        const bool valid = i < n;
        key[j] = valid ? keys_in[i] : K(0);
        row[j] = valid ? rows_in[i] : 0u;
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const uint64_t i = wave_base + (uint64_t)j * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(key[j] >> shift) & (RS_BINS - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RS_BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t before = sm.wave_cnt[wave][d];
        rank[j] = before + below;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) sm.wave_cnt[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // Per digit (thread = digit): offsets of each wave inside the tile's run
    // of that digit, then the digit runs' starts inside the tile.
    {
        const uint32_t d = threadIdx.x;
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            const uint32_t c = sm.wave_cnt[w][d];
            sm.wave_cnt[w][d] = sum;
            sum += c;
        }
        uint32_t tile_total;
        const uint32_t start = block_exclusive_scan(sum, sm.scan_tmp, &tile_total);
        sm.digit_start[d] = start;
        uint32_t dig_total_all;
        const uint32_t dbase = block_exclusive_scan(digit_total[d], sm.scan_tmp, &dig_total_all);
        sm.global_base[d] = dbase + tile_hist[(uint64_t)d * tiles + tile];
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const uint64_t i = wave_base + (uint64_t)j * kWave + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & (RS_BINS - 1);
            const uint32_t pos = sm.digit_start[d] + sm.wave_cnt[wave][d] + rank[j];
            sm.keys[pos] = key[j];
            sm.rows[pos] = row[j];
        }
    }
    __syncthreads();

    const uint32_t valid_in_tile = (uint32_t)((n - tile_base) < (uint64_t)RS_TILE ? (n - tile_base) : RS_TILE);
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < valid_in_tile; p += RS_THREADS) {
        const K kk = sm.keys[p];
        const uint32_t d = (uint32_t)(kk >> shift) & (RS_BINS - 1);
        const uint64_t o = (uint64_t)sm.global_base[d] + (p - sm.digit_start[d]);
        keys_out[o] = kk;
        rows_out[o] = sm.rows[p];
    }
}

struct TempLayout {
    size_t keys_off, rows_off, tile_off, total_off, ghist_off, bytes;
    uint32_t tiles;
};

TempLayout temp_layout(uint64_t n, bool u64) {
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    TempLayout t{};
    t.tiles = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    if (t.tiles == 0) t.tiles = 1;
    size_t off = 0;
    t.keys_off = off;
    off += up(n * (u64 ? 8 : 4));
    t.rows_off = off;
    off += up(n * 4);
    t.tile_off = off;
    off += up((size_t)t.tiles * RS_BINS * 4);
    t.total_off = off;
    off += up(RS_BINS * 4);
    t.ghist_off = off;
    off += up(8 * RS_BINS * 4);
    t.bytes = off;
    return t;
}

template <typename K>
int sort_impl(const K *keys_in, const uint32_t *rows_in, uint64_t n, K *keys_out, uint32_t *rows_out, void *temp,
              hipStream_t s) {
    constexpr int passes_max = (int)sizeof(K);
    if (n == 0) return IDX_OK;
    const TempLayout tl = temp_layout(n, sizeof(K) == 8);
    char *tb = (char *)temp;
    K *tkeys = (K *)(tb + tl.keys_off);
    uint32_t *trows = (uint32_t *)(tb + tl.rows_off);
    uint32_t *tile_hist = (uint32_t *)(tb + tl.tile_off);
    uint32_t *digit_total = (uint32_t *)(tb + tl.total_off);
    uint32_t *ghist = (uint32_t *)(tb + tl.ghist_off);

    IDX_HIP(hipMemsetAsync(ghist, 0, 8 * RS_BINS * 4, s));
    {
        uint64_t blocks = (n + RS_THREADS * 16 - 1) / (RS_THREADS * 16);
        if (blocks > 2048) blocks = 2048;
        hipLaunchKernelGGL(k_global_hist<K>, dim3((uint32_t)blocks), dim3(RS_THREADS), 0, s, keys_in, n, passes_max,
                           ghist);
        IDX_LAUNCH_CHECK();
    }
    uint32_t hh[8 * RS_BINS];
    IDX_HIP(hipMemcpyAsync(hh, ghist, sizeof(uint32_t) * passes_max * RS_BINS, hipMemcpyDeviceToHost, s));
    IDX_HIP(hipStreamSynchronize(s));
    int run[8], nrun = 0;
    for (int p = 0; p < passes_max; ++p) {
        bool trivial = false;
        for (int d = 0; d < RS_BINS; ++d)
            if (hh[p * RS_BINS + d] == n) trivial = true;
        if (!trivial) run[nrun++] = p;
    }
    if (nrun == 0) {
        IDX_HIP(hipMemcpyAsync(keys_out, keys_in, n * sizeof(K), hipMemcpyDeviceToDevice, s));
        IDX_HIP(hipMemcpyAsync(rows_out, rows_in, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        return IDX_OK;
    }
    // Ping-pong so that the last pass writes keys_out / rows_out.
    const K *src_k = keys_in;
    const uint32_t *src_r = rows_in;
    for (int r = 0; r < nrun; ++r) {
        const bool to_out = ((nrun - 1 - r) % 2) == 0;
        K *dst_k = to_out ? keys_out : tkeys;
        uint32_t *dst_r = to_out ? rows_out : trows;
        const int shift = run[r] * RS_BITS;
        hipLaunchKernelGGL(k_tile_hist<K>, dim3(tl.tiles), dim3(RS_THREADS), 0, s, src_k, n, shift, tile_hist,
                           tl.tiles);
        IDX_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_digit_scan, dim3(RS_BINS), dim3(RS_THREADS), 0, s, tile_hist, tl.tiles, digit_total);
        IDX_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scatter<K>, dim3(tl.tiles), dim3(RS_THREADS), 0, s, src_k, src_r, dst_k, dst_r, n,
                           shift, tile_hist, tl.tiles, digit_total);
        IDX_LAUNCH_CHECK();
        src_k = dst_k;
        src_r = dst_r;
    }
    return IDX_OK;
}

}  // namespace

size_t sort_temp_bytes(uint64_t n, bool u64) { return temp_layout(n, u64).bytes; }

int sort_pairs(const void *keys_in, const uint32_t *rows_in, uint64_t n, bool u64, void *keys_out,
               uint32_t *rows_out, void *temp, hipStream_t s) {
    if (u64)
        return sort_impl<uint64_t>((const uint64_t *)keys_in, rows_in, n, (uint64_t *)keys_out, rows_out, temp, s);
    return sort_impl<uint32_t>((const uint32_t *)keys_in, rows_in, n, (uint32_t *)keys_out, rows_out, temp, s);
}

}  // namespace idx
