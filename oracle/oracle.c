/*
 * CPU ORACLE for the static index -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or helper with the
 * GPU library and never calls it.  Everything here is the plain definition of
 * what the index computes, written for obviousness, not speed.
 *
 * Keys are unsigned integers; 32-bit keys are widened to 64 bits by the caller
 * (widening preserves unsigned order).  Row IDs are uint32.
 *
 *  O1  build order: stable sort of (key, rowid) pairs by key
 *      (Section 1 problem statement; Section 3: building BS is a key-value sort).
 *  O2  point lookup: first position r with K[r] >= x (lower bound); the answer
 *      is R[r] when K[r] == x, else the miss sentinel 0xFFFFFFFF
 *      (Section 1 point lookup: the row ID of the row whose key is X).
 *  O3  range lookup [L, U]: all R[r] with L <= K[r] <= U, in ascending key
 *      order (ties in input order); per-query offsets are the exclusive prefix
 *      sum of the counts (Section 1 range lookup).
 *  O4  Eytzinger layouts: the level-order linearisation of the complete search
 *      tree (Section 3, Figures 4-5; k-ary generalisation Section 6, Figure 10),
 *      produced by an in-order walk of the implicit tree -- NOT by the closed
 *      formula of Sections 4 and 6.1.  Node a holds level-order slots
 *      a(k-1) .. a(k-1)+k-2, its children are nodes a*k+1+j (j = 0..k-1); the
 *      walk visits child j before pivot j and the last child after the last
 *      pivot, handing out ascending ranks; slots >= n do not exist.  The binary
 *      Eytzinger layout (EBS) is k = 2 stored 1-based with slot 0 empty.
 *  O5  learned rank model (two-stage linear): loss, gradient and Hessian of
 *      the squared rank error in double precision; the key feature and the
 *      leaf a key falls into are taken in single precision, the precision the
 *      model itself evaluates them in.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MISS 0xFFFFFFFFu

/* ---------------- O1: stable sort of (key, rowid) by key ------------------ */

static void merge_pass(uint64_t *k, uint32_t *r, uint64_t *tk, uint32_t *tr, uint64_t lo, uint64_t hi)
{
    if (hi - lo < 2) return;
    const uint64_t mid = lo + (hi - lo) / 2;
    merge_pass(k, r, tk, tr, lo, mid);
    merge_pass(k, r, tk, tr, mid, hi);
    /* merge [lo,mid) and [mid,hi); on equal keys the left run goes first */
    uint64_t a = lo, b = mid, o = lo;
    while (a < mid && b < hi) {
        if (k[b] < k[a]) { tk[o] = k[b]; tr[o] = r[b]; ++b; }
        else             { tk[o] = k[a]; tr[o] = r[a]; ++a; }
        ++o;
    }
    while (a < mid) { tk[o] = k[a]; tr[o] = r[a]; ++a; ++o; }
    while (b < hi)  { tk[o] = k[b]; tr[o] = r[b]; ++b; ++o; }
    memcpy(k + lo, tk + lo, (hi - lo) * sizeof(uint64_t));
    memcpy(r + lo, tr + lo, (hi - lo) * sizeof(uint32_t));
}

/* Stable sort of n (key, rowid) pairs by key into (out_k, out_r).  Returns 0,
 * or -1 when the scratch buffers cannot be allocated. */
int orc_stable_sort(const uint64_t *keys, const uint32_t *rowids, uint64_t n, uint64_t *out_k, uint32_t *out_r)
{
    memmove(out_k, keys, n * sizeof(uint64_t));
    memmove(out_r, rowids, n * sizeof(uint32_t));
    if (n < 2) return 0;
    uint64_t *tk = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint32_t *tr = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tk || !tr) { free(tk); free(tr); return -1; }
    merge_pass(out_k, out_r, tk, tr, 0, n);
    free(tk);
    free(tr);
    return 0;
}

/* ---------------- O2 / O3: lookups on the sorted array -------------------- */

/* First r in [0, n] with K[r] >= x. */
static uint64_t lower_bound(const uint64_t *K, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (K[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* First r in [0, n] with K[r] > x. */
static uint64_t upper_bound(const uint64_t *K, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (K[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

typedef struct {
    const uint64_t *K;
    const uint32_t *R;
    uint64_t n;
    const uint64_t *a, *b; /* queries (point: a) or bounds (range: a = L, b = U) */
    uint64_t begin, end;
    uint32_t *out;
    uint64_t *lo_rank, *count;
} job_t;

static void *point_worker(void *p)
{
    job_t *j = (job_t *)p;
    for (uint64_t q = j->begin; q < j->end; ++q) {
        const uint64_t r = lower_bound(j->K, j->n, j->a[q]);
        j->out[q] = (r < j->n && j->K[r] == j->a[q]) ? j->R[r] : ORC_MISS;
    }
    return NULL;
}

static void *range_count_worker(void *p)
{
    job_t *j = (job_t *)p;
    for (uint64_t q = j->begin; q < j->end; ++q) {
        const uint64_t L = j->a[q], U = j->b[q];
        uint64_t lo = 0, hi = 0;
        if (L <= U) {
            lo = lower_bound(j->K, j->n, L);
            hi = upper_bound(j->K, j->n, U);
        }
        j->lo_rank[q] = lo;
        j->count[q] = hi > lo ? hi - lo : 0;
    }
    return NULL;
}

static void run_jobs(void *(*fn)(void *), job_t *proto, uint64_t m, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > m) nthreads = m ? (int)m : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    job_t *jobs = (job_t *)malloc(sizeof(job_t) * nthreads);
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].begin = m * t / nthreads;
        jobs[t].end = m * (t + 1) / nthreads;
        if (t == 0) continue;
        pthread_create(&th[t], NULL, fn, &jobs[t]);
    }
    fn(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}

/* O2: out[q] = rowid of the first build key equal to q[q] in sorted order, or
 * 0xFFFFFFFF.  (K, R) is the output of orc_stable_sort. */
void orc_point(const uint64_t *K, const uint32_t *R, uint64_t n, const uint64_t *q, uint64_t m, uint32_t *out,
               int nthreads)
{
    job_t proto = {K, R, n, q, NULL, 0, 0, out, NULL, NULL};
    run_jobs(point_worker, &proto, m, nthreads);
}

/* O3, first half: per query the rank of its first match and its match count
 * (0 when L > U). */
void orc_range_count(const uint64_t *K, uint64_t n, const uint64_t *L, const uint64_t *U, uint64_t m,
                     uint64_t *lo_rank, uint64_t *count, int nthreads)
{
    job_t proto = {K, NULL, n, L, U, 0, 0, NULL, lo_rank, count};
    run_jobs(range_count_worker, &proto, m, nthreads);
}

/* O3, second half: offsets[0..m] = exclusive prefix sum of count; out gets
 * R[lo_rank[q] .. lo_rank[q]+count[q]) at offsets[q], i.e. rowids in key order. */
void orc_range_fill(const uint32_t *R, const uint64_t *lo_rank, const uint64_t *count, uint64_t m,
                    uint64_t *offsets, uint32_t *out)
{
    uint64_t acc = 0;
    for (uint64_t q = 0; q < m; ++q) {
        offsets[q] = acc;
        if (out)
            for (uint64_t c = 0; c < count[q]; ++c) out[acc + c] = R[lo_rank[q] + c];
        acc += count[q];
    }
    offsets[m] = acc;
}

/* ---------------- O4: Eytzinger layouts by in-order walk ------------------ */

typedef struct {
    uint64_t n, k, next_rank;
    uint64_t *slot_rank; /* level-order slot -> sorted rank */
} walk_t;

static void inorder(walk_t *w, uint64_t node)
{
    const uint64_t first = node * (w->k - 1);
    if (first >= w->n) return; /* the node holds no existing slot, nor do its descendants */
    for (uint64_t j = 0; j + 1 < w->k; ++j) {
        inorder(w, node * w->k + 1 + j);
        const uint64_t slot = first + j;
        if (slot < w->n) w->slot_rank[slot] = w->next_rank++;
    }
    inorder(w, node * w->k + w->k);
}

/* Level-order Eytzinger permutation of fan-out k >= 2 over n sorted entries:
 * slot_rank[t] = sorted rank stored at level-order slot t, t in [0, n).
 * (For the binary layout EBS, slot t here is EBS slot t + 1.)
 * Returns 0, or -1 for k < 2. */
int orc_eytzinger_ranks(uint64_t n, uint64_t k, uint64_t *slot_rank)
{
    if (k < 2) return -1;
    walk_t w = {n, k, 0, slot_rank};
    inorder(&w, 0);
    return w.next_rank == n ? 0 : -1;
}

/* ---------------- O5: two-stage linear rank model, fp64 ------------------- */
/*
 * Model: a root line maps a key feature to a leaf id, each of L leaves is a
 * line mapping the leaf-local key offset to a rank.  The oracle works on the
 * features the caller hands in (x = root feature per key, d = leaf-local
 * feature per key, leaf = assigned leaf per key, y = true rank), so it is the
 * plain definition of the loss and of its derivatives:
 *   loss_leaf(a, b) = sum_i (a*d_i + b - y_i)^2 over keys i in the leaf
 *   grad = (2*sum (a d + b - y) d, 2*sum (a d + b - y))
 *   Gauss-Newton (= exact Hessian here) H = 2*[[sum d^2, sum d], [sum d, count]]
 */

/* Per-leaf loss, gradient (2 per leaf) and Hessian (3 per leaf: dd, d1, 11). */
void orc_leaf_grad(const double *d, const double *y, const uint32_t *leaf, uint64_t n, const double *params,
                   uint32_t L, double *loss, double *grad, double *hess)
{
    memset(loss, 0, L * sizeof(double));
    memset(grad, 0, 2 * L * sizeof(double));
    memset(hess, 0, 3 * L * sizeof(double));
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t l = leaf[i];
        const double a = params[2 * l], b = params[2 * l + 1];
        const double r = a * d[i] + b - y[i];
        loss[l] += r * r;
        grad[2 * l] += 2.0 * r * d[i];
        grad[2 * l + 1] += 2.0 * r;
        hess[3 * l] += 2.0 * d[i] * d[i];
        hess[3 * l + 1] += 2.0 * d[i];
        hess[3 * l + 2] += 2.0;
    }
}

/* Root feature of a key, in single precision as the model evaluates it (a
 * floating-point value that decides an integer -- the leaf -- is taken in the
 * model's own precision): mode 1 = the key rounded to float and scaled by
 * 2^-64; mode 2 = the bit pattern of the key rounded to float, as an
 * unsigned integer rounded to float and scaled by 2^-31. */
float orc_key_feature(uint64_t key, uint32_t mode)
{
    const float f = (float)key;
    if (mode == 1) return f * 0x1p-64f;
    uint32_t bits;
    memcpy(&bits, &f, sizeof bits);
    return (float)bits * 0x1p-31f;
}

/* Leaf of each key under root (mode, a0, a1): clamp(floor(a1*x + a0), 0, L-1),
 * multiply then add in single precision, no fused operation.  x_out may be
 * NULL. */
void orc_assign_leaves(const uint64_t *keys, uint64_t n, uint32_t mode, float a0, float a1, uint32_t L,
                       uint32_t *leaf_out, float *x_out)
{
    for (uint64_t i = 0; i < n; ++i) {
        const float x = orc_key_feature(keys[i], mode);
        volatile float prod = a1 * x; /* rounded on its own before the add */
        const float t = prod + a0;
        uint32_t l;
        if (!(t > 0.0f)) l = 0;
        else if (t >= (float)L) l = L - 1;
        else l = (uint32_t)t;
        leaf_out[i] = l;
        if (x_out) x_out[i] = x;
    }
}

/* Spline root (our reading: a linear spline with knots at equal steps of an
 * exact integer key feature; the paper's learned baseline fixes only the
 * predict-then-search-the-window scheme, Section 8).
 *
 * Bin feature u(x): LINEAR u = x.  LOG u = e * 2^58 + floor((x - 2^e) * 2^58
 * / 2^e) with e = floor(log2 x), and u(0) = 0.
 * Geometry: B = the largest power of two <= 65536 with 64 B <= n; shift s =
 * the smallest s with floor((u(kmax) - u(kmin)) / 2^s) < B; nb =
 * floor((u(kmax) - u(kmin)) / 2^s) + 1.  bin(x) = 0 for u(x) <= u(kmin), else
 * min(nb - 1, floor((u(x) - u(kmin)) / 2^s)).
 * Bin b holds the build keys of ranks [r_b, r_(b+1)) and takes the leaves
 * [f_b, f_(b+1)), f_b = floor(r_b L / n).  With keys and f_(b+1) > f_b, its
 * anchor is its smallest key, w the distance from the anchor to the last key
 * of the 64-bit range that still falls in bin b, sh the smallest shift with
 * floor(w / 2^sh) < 2^32, and mul = min(2^32 - 1, floor((f_(b+1) - f_b) 2^32
 * / (floor(w / 2^sh) + 1))); otherwise mul = 0.
 * A key x of bin b goes to leaf min(L - 1, f_b + floor(floor(max(x - anchor,
 * 0) / 2^sh) * mul / 2^32)). */
static uint64_t orc_bin_feature(uint64_t x, uint32_t bfeat)
{
    if (bfeat == 1 || x == 0) return x;
    uint32_t e = 0;
    while (e < 63 && (x >> (e + 1)) != 0) ++e; /* floor(log2 x) */
    const uint64_t frac = x - ((uint64_t)1 << e); /* < 2^e */
    const uint64_t m = e <= 58 ? frac << (58 - e) : frac >> (e - 58);
    return ((uint64_t)e << 58) + m;
}

static uint32_t orc_bin(uint64_t x, uint32_t bfeat, uint64_t f_lo, uint32_t sh, uint32_t nb)
{
    const uint64_t u = orc_bin_feature(x, bfeat);
    if (u <= f_lo || sh >= 64) return 0;
    const uint64_t b = (u - f_lo) >> sh;
    return b < nb ? (uint32_t)b : nb - 1;
}

/* The smallest key x with u(x) >= P (P <= u(2^64 - 1)), by inverting u. */
static uint64_t orc_feature_floor_key(uint64_t P, uint32_t bfeat)
{
    if (bfeat == 1) return P;
    const uint32_t e = (uint32_t)(P >> 58);
    const uint64_t t = P & (((uint64_t)1 << 58) - 1);
    const uint64_t lead = (uint64_t)1 << e;
    if (e > 58) return lead + (t << (e - 58));
    /* e <= 58: u is injective on [2^e, 2^(e+1)), x = 2^e + ceil(t / 2^(58 - e)) */
    const uint32_t d = 58 - e;
    uint64_t q = t >> d;
    if (q << d != t) ++q;
    if (q >= lead) return lead << 1; /* first key of the next binade */
    return lead + q;
}

/* Build the spline root over the n sorted build keys with L leaves and bin
 * feature bfeat (1 LINEAR, 2 LOG).  geo receives f_lo, shift, nb; anchor,
 * mul, first and sh (bins records) must hold spline_bins(n) entries. */
void orc_spline_build(const uint64_t *sorted_keys, uint64_t n, uint32_t L, uint32_t bfeat, uint64_t *geo,
                      uint64_t *anchor, uint32_t *mul, uint32_t *first, uint32_t *shs)
{
    uint32_t B = 1;
    while (B < 65536u && (uint64_t)B * 2 * 64 <= n) B <<= 1;
    const uint64_t f_lo = orc_bin_feature(sorted_keys[0], bfeat);
    const uint64_t span = orc_bin_feature(sorted_keys[n - 1], bfeat) - f_lo;
    uint32_t sh = 0;
    while (sh < 64 && (span >> sh) >= B) ++sh;
    const uint32_t nb = sh >= 64 ? 1u : (uint32_t)(span >> sh) + 1u;
    geo[0] = f_lo;
    geo[1] = sh;
    geo[2] = nb;
    /* r_b by counting the keys of every bin */
    uint64_t *r = (uint64_t *)calloc((size_t)nb + 1, sizeof(uint64_t));
    if (!r) return;
    for (uint64_t i = 0; i < n; ++i) r[orc_bin(sorted_keys[i], bfeat, f_lo, sh, nb) + 1] += 1;
    for (uint32_t b = 0; b < nb; ++b) r[b + 1] += r[b];
    for (uint32_t b = 0; b < nb; ++b) {
        const uint64_t f0 = (r[b] * L) / n, f1 = (r[b + 1] * L) / n;
        anchor[b] = r[b + 1] > r[b] ? sorted_keys[r[b]] : 0;
        mul[b] = 0;
        first[b] = (uint32_t)f0;
        shs[b] = 0;
        if (r[b + 1] == r[b] || f1 == f0) continue;
        uint64_t w; /* distance from the anchor to the last key in bin b */
        if (b + 1 == nb) w = UINT64_MAX - anchor[b];
        else w = orc_feature_floor_key(f_lo + ((uint64_t)(b + 1) << sh), bfeat) - 1 - anchor[b];
        uint32_t k = 0;
        while ((w >> k) > 0xFFFFFFFFull) ++k;
        const unsigned __int128 num = (unsigned __int128)(f1 - f0) << 32;
        const unsigned __int128 m = num / ((w >> k) + 1);
        mul[b] = m > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)m;
        shs[b] = k;
    }
    free(r);
}

/* Leaves of the m keys `keys` under a spline root built by orc_spline_build. */
void orc_spline_assign(const uint64_t *geo, uint32_t bfeat, uint32_t L, const uint64_t *anchor, const uint32_t *mul,
                       const uint32_t *first, const uint32_t *shs, const uint64_t *keys, uint64_t m,
                       uint32_t *leaf_out)
{
    for (uint64_t i = 0; i < m; ++i) {
        const uint32_t b = orc_bin(keys[i], bfeat, geo[0], (uint32_t)geo[1], (uint32_t)geo[2]);
        const uint64_t d = keys[i] > anchor[b] ? keys[i] - anchor[b] : 0;
        const unsigned __int128 prod = (unsigned __int128)(d >> shs[b]) * mul[b];
        const unsigned __int128 leaf = (unsigned __int128)first[b] + (prod >> 32);
        leaf_out[i] = leaf < L ? (uint32_t)leaf : L - 1;
    }
}

/* Root line fit: loss, gradient and Hessian of sum (a*x + b - t)^2. */
void orc_root_grad(const double *x, const double *t, uint64_t n, const double *params, double *loss, double *grad,
                   double *hess)
{
    double ls = 0, g0 = 0, g1 = 0, h0 = 0, h1 = 0, h2 = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const double r = params[0] * x[i] + params[1] - t[i];
        ls += r * r;
        g0 += 2.0 * r * x[i];
        g1 += 2.0 * r;
        h0 += 2.0 * x[i] * x[i];
        h1 += 2.0 * x[i];
        h2 += 2.0;
    }
    *loss = ls;
    grad[0] = g0; grad[1] = g1;
    hess[0] = h0; hess[1] = h1; hess[2] = h2;
}
