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
 *      (Section 1: "find the row ID of the row that contains X").
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

/* Spline root, written from its definition: knot j (j = 0..G) is the sorted
 * build key at rank floor(j (n - 1) / G); segment j owns the leaves
 * [floor(j L / G), floor((j + 1) L / G)).  A key k with knot_j <= k <
 * knot_(j+1) goes to leaf first_j + min(span_j - 1, trunc(f32(k - knot_j) *
 * s_j)), s_j = f32(span_j) / f32(knot_(j+1) - knot_j), every operation
 * rounded to single precision.  Keys below knot_0 go to leaf 0, keys at or
 * above knot_G to leaf L - 1, keys of a segment without leaves to its first
 * leaf index (capped at L - 1).  Leaves of the m keys `keys` are written. */
void orc_spline_leaves(const uint64_t *sorted_keys, uint64_t n, uint32_t L, uint32_t G, const uint64_t *keys,
                       uint64_t m, uint32_t *leaf_out)
{
    uint64_t *knot = (uint64_t *)malloc(((size_t)G + 1) * sizeof(uint64_t));
    float *scale = (float *)malloc(((size_t)G + 1) * sizeof(float));
    if (!knot || !scale) {
        free(knot);
        free(scale);
        return;
    }
    for (uint32_t j = 0; j <= G; ++j) knot[j] = sorted_keys[((uint64_t)j * (n - 1)) / G];
    for (uint32_t j = 0; j < G; ++j) {
        const uint32_t first = (uint32_t)(((uint64_t)j * L) / G);
        const uint32_t next = (uint32_t)(((uint64_t)(j + 1) * L) / G);
        const uint64_t gap = knot[j + 1] - knot[j];
        volatile float num = (float)(next - first);
        volatile float den = (float)gap;
        scale[j] = gap ? num / den : 0.0f;
    }
    for (uint64_t i = 0; i < m; ++i) {
        const uint64_t k = keys[i];
        uint32_t leaf;
        if (k < knot[0]) {
            leaf = 0;
        } else {
            /* last knot <= k: binary search over knot[0..G] */
            uint32_t lo = 0, hi = G + 1; /* knot[lo] <= k, and every index >= hi is > k */
            while (hi - lo > 1) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (knot[mid] <= k) lo = mid;
                else hi = mid;
            }
            if (lo >= G) {
                leaf = L - 1;
            } else {
                const uint32_t first = (uint32_t)(((uint64_t)lo * L) / G);
                const uint32_t next = (uint32_t)(((uint64_t)(lo + 1) * L) / G);
                if (next == first) {
                    leaf = first < L ? first : L - 1;
                } else {
                    volatile float off = (float)(k - knot[lo]);
                    volatile float f = off * scale[lo];
                    const uint32_t span = next - first;
                    leaf = first + (f < (float)span ? (uint32_t)f : span - 1);
                }
            }
        }
        leaf_out[i] = leaf;
    }
    free(knot);
    free(scale);
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
