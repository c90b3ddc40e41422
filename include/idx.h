/*
 * idx.h -- C ABI of the static GPU index library (libidx.so, gfx950 / MI355X).
 *
 * The library indexes a column of unsigned integer keys (32 or 64 bit) with
 * unique 32-bit row IDs and answers the two lookups of the paper's problem
 * statement (Section 1):
 *   - point lookup: the row ID of the row whose key equals X;
 *   - range lookup: the row IDs of all rows whose key e satisfies L <= e <= U.
 * Three physical layouts are offered (Sections 3 and 6):
 *   IDX_BS  -- the (key, rowid) pairs sorted by key, searched by binary search;
 *   IDX_EBS -- binary Eytzinger (level) order, 1-based with an empty slot 0
 *              (Section 3, Figure 5), searched from slot 1 going to 2i or 2i+1;
 *   IDX_EKS -- k-ary Eytzinger order: k-1 sorted pivots per node, no empty
 *              slot, the children of the node starting at slot i start at
 *              i*k + (j+1)*(k-1), j = 0..k-1 (Section 6, Figures 10 and 11).
 * The Eytzinger layouts are produced from the sorted array by a parallel
 * permutation with one read and one write per element (Sections 4 and 6.1).
 *
 * Conventions shared by every call:
 *   - Every data pointer (keys, rowids, queries, bounds, outputs) is a DEVICE
 *     pointer on the current HIP device.  The caller owns inputs and outputs.
 *   - `stream` is a hipStream_t passed as void*; NULL is the legacy null stream.
 *     Calls enqueue their work on it and return without waiting, except where
 *     a call states that it synchronises the stream.
 *   - Keys compare as unsigned integers of the declared width (flags).
 *   - Status codes: IDX_OK (0) or a negative IDX_ERR_* value; no C++
 *     exception crosses this boundary.  After IDX_ERR_HIP the HIP error code
 *     of the failing runtime call is available from idx_last_hip_error().
 */
#ifndef IDX_H
#define IDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct idx_index *idx_handle; /* opaque; owns the layout's device buffers */
typedef void *idx_stream;             /* hipStream_t */

/* layouts */
#define IDX_BS 0
#define IDX_EBS 1
#define IDX_EKS 2

/* build flags (bitwise OR) */
#define IDX_KEY_U32 0u /* keys are uint32 */
#define IDX_KEY_U64 1u /* keys are uint64 */
#define IDX_SOA 0u     /* rowids in an array parallel to the keys (Section 7.1) */
#define IDX_AOS 2u     /* rowids interleaved with the keys (Section 7.1); see idx_build */
#define IDX_AOS_PADDED 4u /* with IDX_AOS: each node block padded to a power of two bytes (whole cache
                             lines), so a node's row IDs share its keys' line; larger footprint */

/* point-lookup miss sentinel; also a reserved row ID value */
#define IDX_MISS 0xFFFFFFFFu

/* status codes */
#define IDX_OK 0
#define IDX_ERR_ARG (-1)            /* invalid argument (null pointer, bad layout/k/flags, size limit) */
#define IDX_ERR_RESERVED_ROWID (-2) /* a row ID equals IDX_MISS */
#define IDX_ERR_NOMEM (-3)          /* device allocation failed */
#define IDX_ERR_HIP (-4)            /* a HIP runtime call or kernel launch failed */
#define IDX_ERR_CAPACITY (-5)       /* range output does not fit the given capacity */
#define IDX_ERR_SCRATCH (-6)        /* request larger than the fixed scratch of idx_range_noalloc */

/* Largest supported number of build keys. */
#define IDX_MAX_KEYS 0xFFFFFFFEull
/* Largest supported EKS fan-out (k - 1 pivots must fit one 64-lane wave). */
#define IDX_MAX_FANOUT 65u

/*
 * Optional device allocator used for the handle's buffers and for the
 * temporary buffers of a call.  alloc(ctx, bytes, stream) returns a device
 * pointer (256-byte aligned) or NULL; release(ctx, ptr, stream) frees it.
 * Both must be stream-ordered with respect to `stream`: a buffer released on
 * a stream may be reused only by work enqueued after the release.  Passing
 * NULL selects hipMallocAsync / hipFreeAsync on the call's stream.
 */
typedef struct idx_allocator {
    void *(*alloc)(void *ctx, size_t bytes, idx_stream stream);
    void (*release)(void *ctx, void *ptr, idx_stream stream);
    void *ctx;
} idx_allocator;

/*
 * idx_build -- build a static index over n (key, rowid) pairs.
 *
 * Sorts the pairs by key with a stable LSD radix sort (Section 3: the BS
 * index is a key-value sort; equal keys keep their input order), then for
 * IDX_EBS / IDX_EKS rearranges the sorted array into Eytzinger order with one
 * read and one write per element, in rank order: the thread of sorted rank r
 * reads entry r and writes it to the level-order slot t whose rank p'(t) is r,
 * the inverse of the map p'(t) of Section 4 (k = 2) and Section 6.1 (any k),
 * evaluated in closed form (idx_rank_slot gives the same map on the host).
 *
 *   keys     device array of n keys (uint32 or uint64 per flags)
 *   rowids   device array of n uint32 row IDs; none may equal IDX_MISS
 *   n        0 <= n <= IDX_MAX_KEYS (n = 0 builds an empty index)
 *   layout   IDX_BS, IDX_EBS or IDX_EKS
 *   k        fan-out: ignored for IDX_BS, must be 2 for IDX_EBS,
 *            2 <= k <= IDX_MAX_FANOUT for IDX_EKS (k - 1 keys per node; the
 *            paper's choice is k - 1 a power of two, any k is accepted)
 *   flags    IDX_KEY_U32 or IDX_KEY_U64, OR-ed with IDX_SOA or IDX_AOS.
 *            AoS stores each node's k-1 keys followed by its k-1 row IDs
 *            (node = one key for BS and EBS), same footprint as SoA.
 *            IDX_AOS | IDX_AOS_PADDED rounds every such block up to a power
 *            of two bytes (e.g. 96 -> 128 for k = 9 with 64-bit keys).
 *   alloc    allocator for the handle and the build's temporaries, or NULL
 *   stream   stream to build on
 *   out      receives the handle (set to NULL on failure)
 *
 * The caller's keys/rowids are only read; they may be freed once the stream
 * reaches the end of the build.  The call synchronises `stream` once, at its
 * end, to read back the reserved-rowid and duplicate-key checks.
 * Errors: IDX_ERR_ARG, IDX_ERR_RESERVED_ROWID (nothing is kept),
 * IDX_ERR_NOMEM, IDX_ERR_HIP.
 */
int idx_build(const void *keys, const uint32_t *rowids, uint64_t n, int layout, uint32_t k, uint32_t flags,
              const idx_allocator *alloc, idx_stream stream, idx_handle *out);

/*
 * idx_relayout -- build an EBS or EKS index (or an AoS copy of a BS index)
 * from an existing sorted-array index without sorting again: only the
 * one-read/one-write permutation of Sections 4 and 6.1 runs (the build of
 * Section 8.5 is sort + rearrangement; this is the rearrangement alone).
 *
 *   src      an IDX_BS index with SoA layout (IDX_ERR_ARG otherwise); it is
 *            only read and stays valid and independent of the result
 *   layout, k, flags, alloc, out   as for idx_build; the key width in
 *            flags must equal src's
 * Enqueued on `stream`, no synchronisation; the build times in idx_info
 * are reported as 0.  Errors: IDX_ERR_ARG, IDX_ERR_NOMEM, IDX_ERR_HIP.
 */
int idx_relayout(idx_handle src, int layout, uint32_t k, uint32_t flags, const idx_allocator *alloc,
                 idx_stream stream, idx_handle *out);

/*
 * idx_merge -- the read-mostly update path (Section 8.5 rebuilds for a batch
 * of updates): a new index over src's pairs plus m new (key, rowid) pairs,
 * laid out as (layout, k, flags) exactly like idx_build.  Only the new pairs
 * are sorted; they are merged into src's sorted array, src's pairs first on
 * equal keys, which is the index idx_build gives for src's pairs followed by
 * the new ones.
 *
 *   src     an IDX_BS index with SoA layout (IDX_ERR_ARG otherwise); unchanged
 *   keys, rowids   m new pairs (device), key width as in flags
 * Synchronises `stream` once.  Errors as idx_build (IDX_ERR_RESERVED_ROWID
 * for a new rowid equal to IDX_MISS).
 */
int idx_merge(idx_handle src, const void *keys, const uint32_t *rowids, uint64_t m, int layout, uint32_t k,
              uint32_t flags, const idx_allocator *alloc, idx_stream stream, idx_handle *out);

/*
 * idx_save -- write the handle (its layout buffers, key order facts and any
 * learned model) to one host byte blob.  *size receives the bytes needed;
 * blob = NULL only asks for the size.  IDX_ERR_CAPACITY when capacity is
 * smaller.  The format belongs to this library build: load it with the same
 * build.  Synchronises `stream`.
 */
int idx_save(idx_handle h, void *blob, uint64_t capacity, uint64_t *size, idx_stream stream);

/*
 * idx_load -- a new handle from a blob written by idx_save (host memory of
 * `size` bytes).  Lookup parameters start at their defaults.  IDX_ERR_ARG for
 * bytes that are not such a blob (marker, sizes).  Synchronises `stream`.
 */
int idx_load(const void *blob, uint64_t size, const idx_allocator *alloc, idx_stream stream, idx_handle *out);

/*
 * idx_point -- batched point lookups (Section 1; search procedures of
 * Sections 3 and 6.2).
 *
 *   queries    device array of m keys of the index's key width
 *   m          number of lookups (0 is allowed)
 *   out_rowid  device array of m uint32: out_rowid[q] is the row ID of the
 *              first build pair (in stable sorted order) whose key equals
 *              queries[q], or IDX_MISS when there is none
 * Enqueued on `stream`, no synchronisation.  Errors: IDX_ERR_ARG, IDX_ERR_HIP.
 */
int idx_point(idx_handle h, const void *queries, uint64_t m, uint32_t *out_rowid, idx_stream stream);

/*
 * idx_range -- batched range lookups [lo[q], hi[q]] (Section 1; level
 * scans of Section 5 for the Eytzinger layouts).
 *
 *   lo, hi       device arrays of m inclusive bounds (lo > hi gives an empty range)
 *   out_offsets  device array of m + 1 uint64: the rowids of query q are
 *                out_rowids[out_offsets[q] .. out_offsets[q+1]), out_offsets[0] = 0
 *   out_rowids   device array of `capacity` uint32, or NULL to count only.
 *                Each query's rowids are in ascending key order (equal keys in
 *                input order), whatever the layout.
 *   capacity     number of uint32 slots in out_rowids
 *   total        host pointer receiving the total number of matches, or NULL
 * Synchronises `stream` once to read the total.  out_offsets is always
 * written; when total > capacity the call returns IDX_ERR_CAPACITY and
 * writes no rowids.  Errors: IDX_ERR_ARG, IDX_ERR_NOMEM, IDX_ERR_HIP,
 * IDX_ERR_CAPACITY.
 */
int idx_range(idx_handle h, const void *lo, const void *hi, uint64_t m, uint64_t *out_offsets,
              uint32_t *out_rowids, uint64_t capacity, uint64_t *total, idx_stream stream);

/*
 * idx_range_noalloc -- idx_range for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, outputs, kernels and errors as
 * idx_range; the call's scratch (4 bytes per range plus one 8-byte partial
 * per 4096 ranges) comes from one statically sized device array instead of
 * the handle's allocator, so no hipMalloc, hipFree or allocating library
 * routine runs.  Each device holds its own array (about 32 MiB, kept until
 * the process ends).  All calls on one device share it: calls that overlap
 * on one device (concurrent streams or threads) race and must be ordered by
 * the caller.  IDX_ERR_SCRATCH when m > IDX_NOALLOC_MAX_RANGES (nothing is
 * enqueued).  The rank-bucket partition (lookup parameter reorder = 2) needs
 * scratch proportional to the batch, so these calls count unpartitioned;
 * and a learned model's leaf lines (leaf_lines = 1) are used only when they
 * exist already (else the leaf records' windows are searched); the answers
 * are the same.  Synchronises `stream` once, like idx_range.
 */
#define IDX_NOALLOC_MAX_RANGES (1ull << 23)
int idx_range_noalloc(idx_handle h, const void *lo, const void *hi, uint64_t m, uint64_t *out_offsets,
                      uint32_t *out_rowids, uint64_t capacity, uint64_t *total, idx_stream stream);

/* idx_destroy -- free the handle and its device buffers (stream-ordered on
 * the stream of the last call that used the handle).  NULL is accepted.
 * IDX_ERR_ARG, and nothing is freed, while a batch (idx_batch_create) holds
 * the handle. */
int idx_destroy(idx_handle h);

/* Text for a status code (static storage). */
const char *idx_strerror(int status);

/* HIP error code (hipError_t) of the most recent IDX_ERR_HIP in this thread. */
int idx_last_hip_error(void);

/* ---------------------------------------------------------------------------
 * Introspection
 * ------------------------------------------------------------------------- */

typedef struct idx_info {
    uint64_t n;               /* build keys */
    uint64_t slots;           /* layout slots (n, or n + 1 for EBS) */
    uint64_t footprint_bytes; /* device bytes permanently held for keys + rowids */
    int32_t layout;
    uint32_t k;               /* fan-out (1 for BS, 2 for EBS) */
    uint32_t flags;
    uint32_t unique;          /* 1 when all build keys are distinct */
    uint32_t levels;          /* tree levels (BS: binary-search steps) */
    uint32_t full_levels;     /* fully occupied levels m (Sections 4, 6.1) */
    uint64_t bottom_keys;     /* keys on the partial lowest level b */
    float build_ms_sort;      /* device time of the sort phase of the last build */
    float build_ms_permute;   /* device time of the permutation phase (0 for BS) */
} idx_info;

int idx_get_info(idx_handle h, idx_info *out);

/*
 * idx_export -- copy the layout, slot by slot, into caller buffers as
 * structure-of-arrays: keys_out[slots] (key width of the index) and
 * rowids_out[slots] (uint32).  For EBS slot 0 is the empty slot (key 0,
 * rowid IDX_MISS).  Either pointer may be NULL.  Enqueued on `stream`.
 */
int idx_export(idx_handle h, void *keys_out, uint32_t *rowids_out, idx_stream stream);

/*
 * idx_slot_rank -- host-side evaluation of the build permutation: the sorted
 * rank of the entry stored at 0-based level-order slot `slot` of the k-ary
 * Eytzinger layout over n keys (k = 2 is the binary layout, whose 1-based
 * slot s is level-order slot s - 1).  This is the inverse permutation p'(t)
 * of Sections 4 and 6.1, which the range level scan evaluates for the slots
 * it visits.  Returns UINT64_MAX when k < 2 or slot >= n.  Pure function, no
 * device use.
 */
uint64_t idx_slot_rank(uint64_t n, uint32_t k, uint64_t slot);

/*
 * idx_rank_slot -- host-side evaluation of the map the layout build kernels
 * evaluate for every sorted rank (Sections 4 and 6.1 read in the other
 * direction): the 0-based level-order slot of the k-ary Eytzinger layout
 * over n keys that holds the key of sorted rank `rank`, the inverse of
 * idx_slot_rank.  Returns UINT64_MAX when k < 2, k > IDX_MAX_FANOUT,
 * n > IDX_MAX_KEYS or rank >= n.  Pure function, no device use.
 */
uint64_t idx_rank_slot(uint64_t n, uint32_t k, uint64_t rank);

/* ---------------------------------------------------------------------------
 * Lookup tuning (Section 7: limiting concurrency, cache pinning, local
 * lookup reordering; Section 6.2: EKS group vs single).  Any field left 0
 * takes the library's default for the index's size class.
 * ------------------------------------------------------------------------- */

typedef struct idx_lookup_params {
    uint32_t group;      /* EKS lanes per lookup: 1 = EKS (single), else a power of
                            two >= k - 1 (EKS (group)); ignored for BS/EBS */
    uint32_t block;      /* threads per workgroup: 64, 128, 256, 512 or 1024 */
    uint32_t per_lane;   /* lookups held per lane (group) at once: 1, 2, 4 or 8 */
    uint32_t lds_levels; /* top tree levels served from LDS (cache pinning); 0 = none */
    uint32_t persistent; /* 0 = one workgroup per tile of lookups; c > 0 = persistent
                            grid of c workgroups per compute unit (limited concurrency) */
    uint32_t reorder;    /* 1 = sort each workgroup's point lookups locally before searching;
                            2 = partition the batch by rank bucket of the index first (point
                            lookups, and the count phase of range lookups by their lower bounds),
                            point answers returned to the caller's order by two counting passes,
                            range counts written straight to their ranges' positions;
                            3 = the same partition, each point answer written straight to its
                            position too */
    uint32_t early_exit; /* 1 = stop at an equal key (only used when keys are unique) */
    uint32_t model;      /* 0/1 = use the learned model when one is trained (idx_learn), 2 = ignore it */
    uint32_t window_rounds; /* short-window scan (BS and learned forms): 0 = default (2); 2 = read the
                               128-byte line of the window's first key, the rest only when all its
                               keys are below the query (fewer lines when they come from HBM);
                               1 = read the whole window at once (shorter chains when it is cached,
                               e.g. skewed or sorted batches) */
    uint32_t range_scan; /* Eytzinger range lookups, how the row IDs are collected: 0 = default (3);
                            1 = level scan (Section 5) with the hybrid coalesced scan of
                            Section 5.1: a lane that meets 64 matches on one level hands its scan
                            to its whole wave; 2 = level scan, every range by its own lane alone;
                            3 = gather by rank: the matches are the ranks [first, first + count)
                            of the count phase, each read at the slot the layout build wrote
                            that rank to (the inverse permutation, no key reads) */
    uint32_t leaf_lines; /* learned form: 0 = default (2); 1 = give every leaf of the model one
                            128-byte line holding its base rank, its size and its first 10 keys
                            (64-bit keys; 15 for 32-bit keys) with their row IDs: a point lookup
                            or a range bound then reads the root's line and nothing else unless
                            it lies past those keys in a larger leaf (then the rest of the leaf
                            is searched in the sorted array); two
                            lanes share each lookup, one per half line (at most 256 threads per
                            workgroup are used, and with reorder = 1, where each lane reads its
                            whole line, at most 4 lookups per lane).  The
                            lines (leaves x 128 bytes of device memory) are written by idx_learn
                            when this is set before training, else by the first lookup that uses
                            them, and freed with the model; 2 = search the leaf record's window
                            in the sorted array */
} idx_lookup_params;

/* Set (p != NULL) or reset to defaults (p == NULL).  Errors: IDX_ERR_ARG for an
 * unsupported combination (the handle keeps its previous parameters). */
int idx_set_params(idx_handle h, const idx_lookup_params *p);
/* The parameters point lookups will use (defaults resolved). */
int idx_get_params(idx_handle h, idx_lookup_params *out);

/* ---------------------------------------------------------------------------
 * Learned rank model (window search on the sorted array).  The model only
 * narrows the search; answers are the same as without it.  The paper's
 * learned-index baseline (Section 8, PGM: predict a position, then binary
 * search within +-epsilon) and its remark that this last-mile search is the
 * expensive step (Section 9) are the anchors.
 * ------------------------------------------------------------------------- */

#define IDX_FEATURE_AUTO 0u   /* train a linear and a spline root, keep the lower estimated lookup cost */
#define IDX_FEATURE_LINEAR 1u /* linear root over the key scaled to [0, 1] */
#define IDX_FEATURE_LOG 2u    /* linear root over the bit pattern of the key rounded to FP32 (log-like) */
#define IDX_FEATURE_SPLINE 3u /* piecewise-linear root over up to 2^16 equal bins of an exact integer
                                 key feature (the key, or a log-like code), at least 64 keys per
                                 bin; each bin takes leaves in proportion to its keys, so clustered
                                 key distributions get even leaves.  One 16-byte bin record per
                                 lookup. */

typedef struct idx_learn_stats {
    uint32_t leaves;     /* L */
    uint32_t epochs;     /* Newton steps per stage */
    uint32_t feature;    /* root feature chosen */
    float root_a0, root_a1;
    double root_loss;    /* sum of squared root residuals (target rank * L / n) */
    double leaf_loss;    /* sum of squared leaf residuals (target local rank) */
    double mean_window;  /* key-weighted mean search window (slots) */
    double max_window;   /* largest window of any leaf (slots) */
    uint32_t segments;     /* spline root: bins in use (0 for a linear root) */
    uint32_t bin_feature;  /* spline root: IDX_FEATURE_LINEAR or IDX_FEATURE_LOG bins (0 otherwise) */
} idx_learn_stats;

/*
 * idx_learn -- train a two-stage FP32 rank model on the GPU from the index's
 * own (key, rank) pairs and attach it to the index.  A linear root maps a
 * monotone key feature to one of `leaves` leaves; each leaf is a line over
 * the leaf-local key offset.  Training runs `epochs` Newton steps per stage
 * (forward/backward kernels accumulate loss, gradient and Hessian sums in
 * FP64).  Then the per-leaf minimum and maximum of (true rank - predicted
 * rank) are measured over all build keys.  Afterwards idx_point and idx_range
 * on h search only the predicted window; their answers are unchanged.
 *
 *   h        an IDX_BS index (any storage: SoA, AoS or line-padded AoS, where
 *            the window scan reads each key with its row ID) with n >= 1
 *            (IDX_ERR_ARG otherwise)
 *   leaves   1 <= leaves <= 2^26 (a linear root resolves about 2^24 leaves in
 *            FP32; beyond that only the spline root spreads keys evenly);
 *            epochs 1..16;  feature IDX_FEATURE_* (LINEAR
 *            and LOG: that linear root; SPLINE: the spline root whose bin
 *            feature has the lower root loss; AUTO: the better linear root and
 *            the spline root each get trained leaves, and the one with the
 *            lower log2(1 + mean window), plus 1 for the spline's bin record,
 *            is kept -- a tie keeps the linear root)
 * With leaf lines selected (lookup parameter leaf_lines = 1) the lines are
 * written here, 128 bytes per leaf; a re-training keeps the replaced model's
 * line buffer and rewrites it when the leaf count is the same, and frees it
 * otherwise (idx_unlearn and idx_destroy free it too).  Work on another
 * stream that still reads the previous model must be ordered before this call.
 * Synchronises `stream`.  Errors: IDX_ERR_ARG, IDX_ERR_NOMEM, IDX_ERR_HIP.
 */
int idx_learn(idx_handle h, uint32_t leaves, uint32_t epochs, uint32_t feature, idx_stream stream);

/*
 * idx_learn_batch -- train the models of `count` indexes at once: every
 * kernel of one launch sequence spans all of them (the batched form of
 * idx_learn: same model, stages and Newton steps; the FP64 sums may add in
 * another order, so weights can differ from idx_learn's in the last FP32
 * bit, while every lookup answer stays exact).
 *
 *   indexes  count distinct IDX_BS SoA indexes, n >= 1, one key width
 *   leaves   count leaf counts (host array), each 1 .. 2^22
 *   epochs   1..16;  feature IDX_FEATURE_* (AUTO picks per index)
 * Each index's previous model is replaced.  Scratch comes from the first
 * index's allocator.  Synchronises `stream` once.  Errors: IDX_ERR_ARG
 * (nothing changed), IDX_ERR_NOMEM, IDX_ERR_HIP (no index keeps a model).
 */
int idx_learn_batch(const idx_handle *indexes, uint32_t count, const uint32_t *leaves, uint32_t epochs,
                    uint32_t feature, idx_stream stream);

/* Statistics of the attached model (IDX_ERR_ARG when there is none). */
int idx_learn_stats_get(idx_handle h, idx_learn_stats *out);

/* Copy the attached model's leaf table (leaves x 32-byte records:
 * uint64 kmin, uint32 base, uint32 size, float b0, float b1, int32 elo,
 * int32 ehi) to the device buffer `leaves_out`.  Enqueued on `stream`. */
int idx_learn_export(idx_handle h, void *leaves_out, idx_stream stream);

/* Drop the attached model (lookups return to the plain layout search). */
int idx_unlearn(idx_handle h);

/*
 * idx_learn_eval -- evaluate the training kernels at given parameters, for
 * gradient checks.  Root: feature `feature` (LINEAR or LOG), parameters
 * root_ab = {a0, a1} (host), target rank * leaves / n.  root_acc (host, 6
 * doubles) receives N, sum x, sum x^2, sum r, sum r*x, sum r^2, where
 * r = a1*x + a0 - target is the FP32 forward residual; the loss gradient is
 * 2 * (sum r*x, sum r).  When leaf_ab (device, 2 * leaves floats: b0, b1 per
 * leaf) and leaf_acc (device, 6 * leaves doubles) are given, keys are
 * assigned to leaves by the root and the same six sums are accumulated per
 * leaf with the leaf-local feature f32(key - first key of the leaf) and
 * target (rank - rank of that first key).  Synchronises `stream`.
 */
int idx_learn_eval(idx_handle h, uint32_t feature, const float *root_ab, uint32_t leaves, const float *leaf_ab,
                   double *root_acc, double *leaf_acc, idx_stream stream);

/* ---------------------------------------------------------------------------
 * Batched lookups over many indexes in one launch
 * ------------------------------------------------------------------------- */

typedef struct idx_batch *idx_batch_t;

#define IDX_BATCH_GRAPH 1u /* replay the launch from a captured HIP graph */

/*
 * idx_batch_create -- gather `count` indexes (same key width, SoA layouts;
 * any of BS, EBS, EKS, or BS with a learned model) into one batch.  Each
 * member's descriptor copies five of its lookup parameters (idx_set_params),
 * so the autotuner can choose them per size class:
 *   model       whether its learned model is used;
 *   early_exit  the EKS early exit on an equal key;
 *   group       EKS lanes per lookup: 1 = one lane reads the whole node
 *               (16-byte loads when nodes are 16-byte aligned), >= k - 1 =
 *               one pivot per lane, fewer = one 16-byte chunk per lane;
 *   lds_levels  top levels served from LDS (cache pinning, Section 7.3): a
 *               workgroup whose chunk of lookups belongs to one member copies
 *               that member's pin table into LDS first (not for the learned
 *               form); the launch reserves LDS for the largest table;
 *   range_scan  how idx_batch_mixed collects an Eytzinger member's range
 *               row IDs (gather by rank, or the level scan).
 * The batch's device descriptors point at the members' layout, pin and model
 * buffers, so until idx_batch_destroy every member is held: on a held handle
 * idx_destroy, idx_learn, idx_unlearn and idx_learn_batch return IDX_ERR_ARG
 * and change nothing, and idx_set_params returns IDX_ERR_ARG for a parameter
 * set that changes any of the five copied parameters.  A handle may belong to
 * several batches.  Synchronises `stream`.  Errors: IDX_ERR_ARG (null, mixed
 * key widths, AoS layout), IDX_ERR_NOMEM.
 */
int idx_batch_create(const idx_handle *indexes, uint32_t count, idx_stream stream, idx_batch_t *out);

/*
 * idx_batch_point -- point lookups for every index of the batch in one
 * persistent launch (the static scheduling of Section 7.2 applied across
 * indexes).  Index i's queries are queries[offsets[i] .. offsets[i+1]) and
 * its answers land at the same positions of out_rowid (rowid or IDX_MISS).
 * Workgroups walk chunks of consecutive queries; within a chunk of one
 * member every lane advances four lookups together (their dependent loads in
 * flight at once), in that member's form and parameters.
 *
 *   queries    device array of offsets[count] keys
 *   offsets    device array of count + 1 non-decreasing uint64, offsets[0] = 0
 *   out_rowid  device array of offsets[count] uint32
 *   flags      0, or IDX_BATCH_GRAPH to launch from a HIP graph captured on
 *              the first call with these three pointers (re-captured when
 *              they change); the graph holds one kernel node, no memset
 * Enqueued on `stream`.  Errors: IDX_ERR_ARG, IDX_ERR_HIP.
 */
int idx_batch_point(idx_batch_t b, const void *queries, const uint64_t *offsets, uint32_t *out_rowid, uint32_t flags,
                    idx_stream stream);

/*
 * idx_batch_mixed -- a stream of point and range lookups over every index of
 * the batch (Section 1's two lookup kinds; range output as idx_range).
 * Queries are grouped by index as in idx_batch_point (offsets: count + 1
 * device u64, offsets[count] = m).  Query p is a point lookup of lo[p] when
 * kind[p] == 0 (hi[p] ignored) and the range [lo[p], hi[p]] when kind[p] == 1
 * (inclusive; lo > hi is empty).
 *
 *   lo, hi         m keys each (device, the batch's key width)
 *   kind           m bytes (device), 0 or 1
 *   out_rowid      m (device): the row ID or IDX_MISS for points, IDX_MISS
 *                  for ranges
 *   range_offsets  m + 1 (device u64): exclusive prefix of the match counts
 *                  (0 for points); range_offsets[m] = total
 *   range_rowids   capacity entries (device): each range's row IDs in key
 *                  order from range_offsets[p]; NULL = counts only
 *   total          host, receives the number of matches (may be NULL)
 * Two persistent launches around one scan: the first answers the points and
 * sizes the ranges, the second writes the ranges.  Synchronises `stream`
 * once (to read the total).  m <= 2^32 - 1.  Errors: IDX_ERR_ARG,
 * IDX_ERR_CAPACITY (total > capacity: offsets and point answers written,
 * no range row IDs), IDX_ERR_HIP.
 */
int idx_batch_mixed(idx_batch_t b, uint64_t m, const void *lo, const void *hi, const uint8_t *kind,
                    const uint64_t *offsets, uint32_t *out_rowid, uint64_t *range_offsets, uint32_t *range_rowids,
                    uint64_t capacity, uint64_t *total, idx_stream stream);

/* Free the batch (synchronises the device first) and release its hold on
 * the member indexes.  NULL is accepted. */
int idx_batch_destroy(idx_batch_t b);

/* ---------------------------------------------------------------------------
 * Measurement
 * ------------------------------------------------------------------------- */

/*
 * idx_probe_random -- random-access probe after the coalescing
 * micro-benchmark of Section 5.1 (Figure 9): `lanes` threads in groups of
 * `group` neighbouring lanes; in each of `steps` steps every group reads
 * `group` consecutive 64-bit words of `buf` at a random group-aligned
 * position, with 8 independent streams per lane, so one launch performs
 * lanes * steps * 8 word loads.  It measures the random granule throughput
 * of the memory system (the ceiling a dependent-load search approaches).
 *
 *   buf    device array of `words` uint64 (contents irrelevant)
 *   group  power of two in [1, 64]; lanes a multiple of 256
 *   sink   device uint64 written only to keep the loads alive
 * Enqueued on `stream`.  Errors: IDX_ERR_ARG, IDX_ERR_HIP.
 */
int idx_probe_random(const void *buf, uint64_t words, uint32_t group, uint64_t lanes, uint32_t steps,
                     uint64_t seed, uint64_t *sink, idx_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* IDX_H */
