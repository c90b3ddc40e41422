/*
 * Seeded synthetic inputs for the static index: build key sets, point-query
 * streams, range bounds and size mixes.  This module is shared input
 * plumbing: the CPU oracle and the GPU path both consume what it writes, and
 * it contains none of the indexing arithmetic (no sorting, no searching, no
 * layout formulas).  Every value is a pure function of (seed, stream, index),
 * so any slice can be regenerated independently and in parallel.
 *
 * Random numbers: counter-based, one splitmix64 finaliser (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to a keyed counter.
 *
 * Unique uniform keys: a keyed bijection f on [0, 2^w) built from invertible
 * w-bit steps (add a constant, xor with a right shift, multiply by an odd
 * constant).  keys[i] = f(i) for i < n are distinct and pseudo-uniform; the
 * values f(j) for j >= n are exactly the complement, which gives misses
 * drawn uniformly from "values not in the set" and the expected answer of
 * every generated query by construction.
 *
 * Zipf: bounded Zipf(s) on {1..N} by rejection-inversion (Hormann and
 * Derflinger, "Rejection-inversion to generate variates from monotone
 * discrete distributions", ACM TOMACS 1996).
 *
 * Lognormal mixture: 64 equally weighted components, mu ~ U[20,50],
 * sigma ~ U[0.5,2] (natural-log scale), key = floor(exp(mu + sigma*Z))
 * clamped to 2^63-1, de-duplicated keeping first occurrences in draw order,
 * then placed by a seeded permutation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GEN_MISS 0xFFFFFFFFu

static inline uint64_t smix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The i-th 64-bit draw of the stream `stream` under `seed`. */
uint64_t gen_draw(uint64_t seed, uint64_t stream, uint64_t i)
{
    return smix(smix(seed ^ smix(stream * 0xD1B54A32D192ED03ull)) + i);
}

/* Uniform integer in [0, range) (range >= 1), multiply-high mapping. */
static inline uint64_t below(uint64_t r, uint64_t range)
{
    return (uint64_t)(((unsigned __int128)r * range) >> 64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

static inline uint64_t wmask(int w) { return w >= 64 ? ~0ull : ((1ull << w) - 1); }

/* Keyed bijection on [0, 2^w), 2 <= w <= 64.  Each step is invertible on
 * w-bit values, so the composition is a permutation of [0, 2^w). */
uint64_t gen_bij(uint64_t key, int w, uint64_t x)
{
    const uint64_t M = wmask(w);
    const int s1 = (w + 1) / 2, s2 = w / 2 > 1 ? w / 2 - 1 : 1, s3 = w / 3 > 0 ? w / 3 : 1;
    uint64_t k0 = smix(key), k1 = smix(k0), k2 = smix(k1), k3 = smix(k2);
    x &= M;
    for (int round = 0; round < 2; ++round) {
        x = (x + k0) & M;
        x ^= x >> s1;
        x = (x * (k1 | 1)) & M;
        x ^= x >> s2;
        x = (x * (k2 | 1)) & M;
        x ^= x >> s3;
        x = (x + k3) & M;
        k0 = smix(k3); k1 = smix(k0); k2 = smix(k1); k3 = smix(k2);
    }
    return x;
}

static inline int bits_for(uint64_t N)
{
    int w = 2;
    while (w < 64 && (1ull << w) < N) ++w;
    return w;
}

/* Keyed bijection on [0, N) by cycle walking over the enclosing power of two. */
uint64_t gen_perm(uint64_t key, uint64_t N, uint64_t x)
{
    if (N <= 1) return 0;
    const int w = bits_for(N);
    uint64_t y = gen_bij(key, w, x);
    while (y >= N) y = gen_bij(key, w, y);
    return y;
}

static inline void put_key(void *keys, int key_bytes, uint64_t i, uint64_t v)
{
    if (key_bytes == 4) ((uint32_t *)keys)[i] = (uint32_t)v;
    else ((uint64_t *)keys)[i] = v;
}

static inline uint64_t get_key(const void *keys, int key_bytes, uint64_t i)
{
    return key_bytes == 4 ? ((const uint32_t *)keys)[i] : ((const uint64_t *)keys)[i];
}

/* n distinct pseudo-uniform keys in [0, 2^w): keys[i] = f(i), rowids[i] = i
 * (insertion position).  rowids may be NULL. */
void gen_unique_keys(uint64_t seed, int w, uint64_t n, void *keys, int key_bytes, uint32_t *rowids)
{
    const uint64_t bkey = gen_draw(seed, 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        put_key(keys, key_bytes, (uint64_t)i, gen_bij(bkey, w, (uint64_t)i));
        if (rowids) rowids[i] = (uint32_t)i;
    }
}

/* m point queries against gen_unique_keys(seed, w, n): exactly n_hits of them
 * (positions chosen by a seeded permutation) are build keys f(i), i uniform
 * in [0, n); the rest are f(j), j uniform in [n, 2^w), i.e. uniform over the
 * values not in the set.  expect[q] = i for a hit, GEN_MISS for a miss
 * (expect may be NULL). */
void gen_point_queries(uint64_t seed, int w, uint64_t n, uint64_t m, uint64_t n_hits, void *q, int key_bytes,
                       uint32_t *expect)
{
    const uint64_t bkey = gen_draw(seed, 1, 0);
    const uint64_t pkey = gen_draw(seed, 2, 0);
    const uint64_t space = w >= 64 ? 0 : (1ull << w); /* 0 stands for 2^64 */
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)m; ++t) {
        const int hit = n > 0 && gen_perm(pkey, m, (uint64_t)t) < n_hits;
        const uint64_t r = gen_draw(seed, 3, (uint64_t)t);
        uint64_t src;
        if (hit) {
            src = below(r, n);
        } else {
            const uint64_t nmiss = space - n; /* wraps correctly when space == 2^64 */
            src = n + below(r, nmiss);
        }
        put_key(q, key_bytes, (uint64_t)t, gen_bij(bkey, w, src));
        if (expect) expect[t] = hit ? (uint32_t)src : GEN_MISS;
    }
}

/* ---- bounded Zipf(s) on {1..N}, rejection-inversion ---------------------- */

typedef struct {
    double s, n, hx1, hxn, scst;
} zipf_t;

static double zh(const zipf_t *z, double x) { return exp(-z->s * log(x)); }

/* (exp(x)-1)/x and log1p(x)/x, continuous at 0 */
static double expm1_over(double x) { return fabs(x) > 1e-8 ? expm1(x) / x : 1.0 + x * 0.5 + x * x / 6.0; }
static double log1p_over(double x) { return fabs(x) > 1e-8 ? log1p(x) / x : 1.0 - x * 0.5 + x * x / 3.0; }

/* H(x) = integral of x^-s, normalised so that it is smooth at s = 1. */
static double zH(const zipf_t *z, double x)
{
    const double lx = log(x);
    return expm1_over((1.0 - z->s) * lx) * lx;
}

static double zHinv(const zipf_t *z, double y)
{
    double t = y * (1.0 - z->s);
    if (t < -1.0) t = -1.0; /* guard rounding at the domain edge */
    return exp(log1p_over(t) * y);
}

static void zipf_init(zipf_t *z, double s, uint64_t N)
{
    z->s = s;
    z->n = (double)N;
    z->hx1 = zH(z, 1.5) - 1.0;
    z->hxn = zH(z, z->n + 0.5);
    z->scst = 2.0 - zHinv(z, zH(z, 2.5) - zh(z, 2.0));
}

static uint64_t zipf_draw(const zipf_t *z, uint64_t seed, uint64_t stream, uint64_t idx)
{
    for (uint64_t attempt = 0;; ++attempt) {
        const double u01 = unit(gen_draw(seed, stream, idx * 64 + (attempt & 63) + (attempt >> 6) * 0x1000003ull));
        const double u = z->hxn + u01 * (z->hx1 - z->hxn);
        const double x = zHinv(z, u);
        double kd = floor(x + 0.5);
        if (kd < 1.0) kd = 1.0;
        if (kd > z->n) kd = z->n;
        if (kd - x <= z->scst || u >= zH(z, kd + 0.5) - zh(z, kd)) return (uint64_t)kd;
    }
}

/* m Zipf(s) popularity ranks in {1..N}, written as uint64 (for distribution tests). */
void gen_zipf_ranks(uint64_t seed, double s, uint64_t N, uint64_t m, uint64_t *out)
{
    zipf_t z;
    zipf_init(&z, s, N);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)m; ++t) out[t] = zipf_draw(&z, seed, 5, (uint64_t)t);
}

/* m queries over a build set of n keys: a fraction of them (exactly n_miss,
 * at seeded positions) are misses, the others hit the key of Zipf(s)
 * popularity rank r, which is build position pi(r-1) for a seeded bijection
 * pi on [0, n) (popularity is independent of key order).
 *   keys == NULL: the set is gen_unique_keys(seed, w, n, ...); misses are
 *     f(j), j uniform in [n, 2^w) and expect[] is exact.
 *   keys != NULL: misses are uniform in [0, 2^w) (a draw can coincide with a
 *     build key with probability n / 2^w; expect[] then says GEN_MISS and
 *     only the oracle is authoritative).
 * expect[q] = build position of a hit, GEN_MISS for a miss; may be NULL. */
void gen_zipf_queries(uint64_t seed, int w, double s, const void *keys, uint64_t n, uint64_t m, uint64_t n_miss,
                      void *q, int key_bytes, uint32_t *expect)
{
    const uint64_t bkey = gen_draw(seed, 1, 0);
    const uint64_t pkey = gen_draw(seed, 2, 0);
    const uint64_t popkey = gen_draw(seed, 6, 0);
    const uint64_t space = w >= 64 ? 0 : (1ull << w);
    zipf_t z;
    zipf_init(&z, s, n ? n : 1);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)m; ++t) {
        const int miss = n == 0 || gen_perm(pkey, m, (uint64_t)t) < n_miss;
        uint64_t v;
        uint32_t e;
        if (!miss) {
            const uint64_t r = zipf_draw(&z, seed, 7, (uint64_t)t);
            const uint64_t pos = gen_perm(popkey, n, r - 1);
            v = keys ? get_key(keys, key_bytes, pos) : gen_bij(bkey, w, pos);
            e = (uint32_t)pos;
        } else if (!keys) {
            v = gen_bij(bkey, w, n + below(gen_draw(seed, 8, (uint64_t)t), space - n));
            e = GEN_MISS;
        } else {
            const uint64_t r = gen_draw(seed, 8, (uint64_t)t);
            v = w >= 64 ? r : below(r, space);
            e = GEN_MISS;
        }
        put_key(q, key_bytes, (uint64_t)t, v);
        if (expect) expect[t] = e;
    }
}

/* ---- lognormal mixture key sets ----------------------------------------- */

#define LN_COMPONENTS 64

static uint64_t lognormal_draw(const double *mu, const double *sg, uint64_t seed, uint64_t i)
{
    const uint64_t c = below(gen_draw(seed, 10, i), LN_COMPONENTS);
    double u1 = unit(gen_draw(seed, 11, i));
    const double u2 = unit(gen_draw(seed, 12, i));
    if (u1 < 1e-300) u1 = 1e-300;
    const double zn = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2); /* Box-Muller */
    const double x = exp(mu[c] + sg[c] * zn);
    if (!(x < 9223372036854775807.0)) return 0x7FFFFFFFFFFFFFFFull; /* clamp to 2^63 - 1 */
    return (uint64_t)floor(x);
}

/* Parameters of the 64 components (for documentation and tests). */
void gen_lognormal_params(uint64_t seed, double *mu, double *sigma)
{
    for (int c = 0; c < LN_COMPONENTS; ++c) {
        mu[c] = 20.0 + 30.0 * unit(gen_draw(seed, 13, (uint64_t)c));
        sigma[c] = 0.5 + 1.5 * unit(gen_draw(seed, 14, (uint64_t)c));
    }
}

/* n distinct uint64 keys from the lognormal mixture, de-duplicated keeping
 * the first n distinct values in draw order, then placed at out[pi(j)] for a
 * seeded bijection pi on [0, n); rowids[i] = i.  Returns 0, or -1 when the
 * distribution cannot supply n distinct values within the draw budget or
 * memory runs out. */
int gen_lognormal_keys(uint64_t seed, uint64_t n, uint64_t *keys, uint32_t *rowids)
{
    double mu[LN_COMPONENTS], sg[LN_COMPONENTS];
    gen_lognormal_params(seed, mu, sg);
    if (n == 0) return 0;
    const uint64_t pkey = gen_draw(seed, 15, 0);
    uint64_t budget = n + n / 2 + 1024;
    for (int tries = 0; tries < 4; ++tries, budget *= 2) {
        uint64_t cap = 1;
        while (cap < 2 * budget) cap <<= 1;
        uint64_t *tk = (uint64_t *)malloc(cap * sizeof(uint64_t));
        uint64_t *ti = (uint64_t *)malloc(cap * sizeof(uint64_t));
        uint64_t *draw = (uint64_t *)malloc(budget * sizeof(uint64_t));
        uint8_t *first = (uint8_t *)malloc(budget);
        if (!tk || !ti || !draw || !first) {
            free(tk); free(ti); free(draw); free(first);
            return -1;
        }
        const uint64_t EMPTY = ~0ull; /* never produced: draws are < 2^63 */
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < (int64_t)cap; ++s) { tk[s] = EMPTY; ti[s] = ~0ull; }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)budget; ++i) draw[i] = lognormal_draw(mu, sg, seed, (uint64_t)i);
        /* concurrent open-addressing set: the slot of a value is unique
         * (claimed by compare-and-swap); it records the smallest draw index */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)budget; ++i) {
            const uint64_t v = draw[i];
            uint64_t h = smix(v ^ 0x5bd1e995ull) & (cap - 1);
            for (;;) {
                uint64_t cur = __atomic_load_n(&tk[h], __ATOMIC_ACQUIRE);
                if (cur == EMPTY) {
                    uint64_t expected = EMPTY;
                    if (__atomic_compare_exchange_n(&tk[h], &expected, v, 0, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE))
                        cur = v;
                    else
                        cur = expected;
                }
                if (cur == v) {
                    uint64_t old = __atomic_load_n(&ti[h], __ATOMIC_RELAXED);
                    while ((uint64_t)i < old &&
                           !__atomic_compare_exchange_n(&ti[h], &old, (uint64_t)i, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED))
                        ;
                    break;
                }
                h = (h + 1) & (cap - 1);
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)budget; ++i) {
            const uint64_t v = draw[i];
            uint64_t h = smix(v ^ 0x5bd1e995ull) & (cap - 1);
            while (tk[h] != v) h = (h + 1) & (cap - 1);
            first[i] = ti[h] == (uint64_t)i;
        }
        free(tk);
        free(ti);
        /* first n distinct values in draw order, placed by the permutation */
        uint64_t got = 0;
        for (uint64_t i = 0; i < budget && got < n; ++i)
            if (first[i]) draw[got++] = draw[i];
        free(first);
        if (got == n) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < (int64_t)n; ++j) {
                keys[gen_perm(pkey, n, (uint64_t)j)] = draw[j];
                if (rowids) rowids[j] = (uint32_t)j;
            }
            free(draw);
            return 0;
        }
        free(draw);
    }
    return -1;
}

/* ---- sizes and ranges ---------------------------------------------------- */

/* count sizes floor(2^u), u ~ U[log2 lo, log2 hi], clipped to [lo, hi]. */
void gen_log_uniform(uint64_t seed, uint64_t stream, uint64_t lo, uint64_t hi, uint64_t count, uint64_t *out)
{
    const double a = log2((double)lo), b = log2((double)hi);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)count; ++t) {
        const double u = a + (b - a) * unit(gen_draw(seed, 100 + stream, (uint64_t)t));
        double v = floor(exp2(u));
        if (v < (double)lo) v = (double)lo;
        if (v > (double)hi) v = (double)hi;
        out[t] = (uint64_t)v;
    }
}

/* Range bounds over a build set given in ascending order (`ordered`, n keys):
 * query t covers c_t consecutive ranks, c_t uniform in [cmin, cmax] (clipped to
 * n), starting at a rank uniform in [0, n - c_t]: lo = ordered[r],
 * hi = ordered[r + c_t - 1].  Writes the rank count to counts (may be NULL). */
void gen_ranges(uint64_t seed, const void *ordered, int key_bytes, uint64_t n, uint64_t m, uint64_t cmin,
                uint64_t cmax, void *lo, void *hi, uint32_t *counts, uint64_t *ranks)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)m; ++t) {
        uint64_t c = cmin + below(gen_draw(seed, 20, (uint64_t)t), cmax - cmin + 1);
        if (c > n) c = n;
        if (c == 0) {
            /* empty build set: an empty range lo > hi */
            put_key(lo, key_bytes, (uint64_t)t, 1);
            put_key(hi, key_bytes, (uint64_t)t, 0);
            if (counts) counts[t] = 0;
            if (ranks) ranks[t] = 0;
            continue;
        }
        const uint64_t r = below(gen_draw(seed, 21, (uint64_t)t), n - c + 1);
        put_key(lo, key_bytes, (uint64_t)t, get_key(ordered, key_bytes, r));
        put_key(hi, key_bytes, (uint64_t)t, get_key(ordered, key_bytes, r + c - 1));
        if (counts) counts[t] = (uint32_t)c;
        if (ranks) ranks[t] = r;
    }
}

/* Uniform random values in [0, 2^w) (arbitrary query bounds for tests). */
void gen_uniform_values(uint64_t seed, uint64_t stream, int w, uint64_t m, void *out, int key_bytes)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)m; ++t) {
        uint64_t r = gen_draw(seed, 200 + stream, (uint64_t)t);
        if (w < 64) r &= wmask(w);
        put_key(out, key_bytes, (uint64_t)t, r);
    }
}
