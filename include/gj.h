/*
 * gj: radix-partitioned joins and grouped aggregations on one AMD Instinct
 * MI355X (gfx950). C ABI of libgj.so.
 *
 * Conventions for every entry point:
 *   - Return value: GJ_OK (0) or a negative GJ_E* code. On error the
 *     thread-local message from gj_last_error() says what failed, and no
 *     output is left allocated.
 *   - Column data pointers are HIP device pointers. They are borrowed for the
 *     duration of the call and never retained.
 *   - `stream` is a hipStream_t (NULL = the default stream). All device work
 *     is enqueued on it in order. Calls that must size their outputs read one
 *     count back to the host and so synchronize with the stream.
 *   - Memory: outputs and scratch come from the caller's gj_allocator, called
 *     on the calling thread. Scratch is released through allocator->free
 *     before the call returns, in stream order (the caller's allocator must be
 *     stream-ordered, as a caching device allocator on `stream` is). A NULL
 *     allocator means hipMallocAsync/hipFreeAsync on `stream`.
 *   - Row counts are at most 2^31 - 1 per relation (row identifiers are
 *     32-bit); larger inputs return GJ_EOVERFLOW.
 *   - Calls on different streams may run concurrently; calls that share a
 *     stream are serialized by it.
 */
#ifndef GJ_H
#define GJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GJ_OK 0
#define GJ_EINVAL (-1)       /* null pointer, negative size, mismatched dtypes, bad option */
#define GJ_ENOMEM (-2)       /* the allocator returned NULL */
#define GJ_EHIP (-3)         /* a HIP runtime error; text in gj_last_error() */
#define GJ_EUNSUPPORTED (-4) /* a valid request the library does not implement */
#define GJ_ECAPACITY (-5)    /* a caller-sized output is too small */
#define GJ_EOVERFLOW (-6)    /* more than 2^31 - 1 rows in one relation, or join work units */

typedef enum { GJ_I32 = 1, GJ_I64 = 2 } gj_dtype;

/* One column: `data` points to n_rows elements of `dtype` in device memory. */
typedef struct {
    const void *data;
    int32_t dtype; /* gj_dtype */
} gj_col;

/* A relation R(key, p_1, .., p_n) stored column-wise (Section 3 assumes
 * relations are device-resident columns, one array each). */
typedef struct {
    gj_col key;
    const gj_col *payloads; /* n_payloads columns, may be NULL when n_payloads = 0 */
    int32_t n_payloads;     /* 0..8 */
    int64_t n_rows;
} gj_rel;

typedef struct {
    void *(*alloc)(size_t bytes, void *ctx); /* device memory, >= 256-byte aligned; NULL on failure */
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} gj_allocator;

/* Materialization pattern (Section 4.1): GFTR partitions every payload column
 * together with the key and gathers from the partitioned copies; GFUR
 * partitions (key, row id) only and gathers from the original columns. */
typedef enum { GJ_MAT_AUTO = 0, GJ_MAT_GFTR = 1, GJ_MAT_GFUR = 2 } gj_mat;

/* Join algorithm: the partitioned hash join of Section 4.1.4 (PHJ) or the
 * sort-merge join of Section 3.1.1 (SMJ: full-key radix sort of both
 * relations, Merge Path match finding; its output comes in ascending key
 * order). Either takes GFTR or GFUR materialization. */
typedef enum { GJ_JOIN_AUTO = 0, GJ_JOIN_PHJ = 1, GJ_JOIN_SMJ = 2 } gj_join_algo;

/* Join options; 0 in any field means "choose automatically". Options change
 * speed, never results (SMJ additionally fixes the output order). */
typedef struct {
    int32_t mat;               /* gj_mat */
    int32_t unique_build_keys; /* accepted and ignored: the count pass already detects, on the
                                  device, whether any S row matches twice, and picks the
                                  streaming write pass when none does */
    int32_t radix_bits;        /* total partition bits, 1..16 */
    int32_t passes;            /* 1 or 2 (each pass uses at most 8 bits) */
    int32_t block_size;        /* reserved; must be 0 or 256 */
    float ht_occupancy;        /* ignored by joins (the LDS table has at least as many buckets
                                  as rows of its build block) */
    int32_t lds_budget;        /* max R rows per build block, 64..16384 (8-byte keys: 64..8192);
                                  0: 4096 below |R| = 2^24; from there 16384 for GFTR with
                                  4-byte keys and at most 18 bytes of R payload per row,
                                  else 8192; the LDS table
                                  has 4096, 8192 or 16384 rows, the smallest that holds it */
    uint64_t flags;            /* reserved, must be 0 */
    int32_t algo;              /* gj_join_algo */
    float match_ratio_hint;    /* expected share of S rows with a match, for automatic choices
                                  (0: unknown, taken as 1) */
    float skew_hint;           /* expected Zipf factor of S.key (0: unknown, taken as uniform) */
} gj_join_opts;

/* Join output T(key, r_1..r_cR, s_1..s_cS). The library allocates every column
 * separately through the allocator; the caller owns them. r_payloads and
 * s_payloads are caller-provided arrays with room for R.n_payloads and
 * S.n_payloads pointers. Column dtypes equal the input columns' dtypes. */
typedef struct {
    void *key;
    void **r_payloads;
    void **s_payloads;
    int64_t n_rows;
} gj_join_out;

/*
 * Inner equi-join T = R |><| S on key (Section 2.2), by the partitioned hash
 * join of Section 4.1.4: stable radix partitioning of both relations into
 * contiguous partitions, a hash build on each R partition in LDS probed by the
 * co-partition of S, and materialization of the payload columns under GFTR or
 * GFUR. Many-to-many inputs are supported (every matching pair is emitted).
 * R and S keys must share a dtype (GJ_I32 or GJ_I64); payload columns may be
 * GJ_I32 or GJ_I64. Output row order is unspecified but deterministic for a
 * given input and options. Empty inputs give n_rows = 0 and NULL columns.
 * Default radix_bits: partitions of about lds_budget / 2 R rows (at least 1 bit).
 * Partition digits are the low key bits; when the largest R partition holds more
 * than four times the mean plus a build block (keys whose low bits barely vary),
 * both relations are partitioned again on the MurmurHash3 finalizer of the key.
 * More than 2^31 - 1 work units (partitions far beyond the build block, as with
 * very many duplicate keys and a tiny lds_budget) return GJ_EOVERFLOW before any
 * match is sought. Synchronizes with `stream` twice (unit count and output size).
 */
int gj_join(const gj_rel *R, const gj_rel *S, const gj_join_opts *opts,
            const gj_allocator *alloc, void *stream, gj_join_out *out);

/* A batch of independent relations stored back to back ("ragged" layout):
 * instance i owns rows [offsets[i], offsets[i+1]) of every column. */
typedef struct {
    gj_col key;
    const gj_col *payloads; /* n_payloads concatenated columns */
    int32_t n_payloads;     /* 0..8 */
    const int64_t *offsets; /* host array of n_instances + 1 row offsets, offsets[0] = 0 */
    int32_t n_instances;
} gj_rel_batch;

/*
 * Many independent joins T_i = R_i |><| S_i in one call (no counterpart in the
 * paper; the method of gj_join applied to every instance at once). Instance i is
 * a segment of one partitioning pass with its own partition bits (at most 8), and
 * one count pass, one scan and one write pass serve all instances, so the number
 * of kernel launches does not grow with the number of instances.
 * R and S must have the same n_instances, key dtype, and payload column counts
 * and dtypes per side across the batch. The output T is concatenated in instance
 * order; out_offsets (host, n_instances + 1 entries) receives where each
 * instance's rows begin. Each side's total row count must be below 2^31
 * (GJ_EOVERFLOW otherwise). Synchronizes with `stream` twice.
 */
int gj_join_batch(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts,
                  const gj_allocator *alloc, void *stream, gj_join_out *out, int64_t *out_offsets);

/* ---- Batch plans: persistent kernels replayed as one HIP graph ----------------
 * A plan fixes the shape of a batch (row counts per instance, column types,
 * options), borrows its input columns (their addresses are baked in) and owns
 * every block of device memory the batch needs: scratch, per-instance device
 * parameters and output columns of a capacity fixed at creation. Running a plan
 * enqueues kernels only: no allocation, no host synchronization, no copy, no
 * memset. Every data-dependent size (work units, output rows) stays in device
 * memory, and the kernels that depend on it are persistent workgroups looping
 * over the device count. So the run can be captured once into a HIP graph and
 * replayed with one hipGraphLaunch per batch; refilling the input columns in
 * place and launching again processes new data of the same shape.
 * Calls on one plan must not overlap (its scratch is shared); different plans
 * are independent. Plan memory comes from `alloc` (hipMalloc when NULL) and is
 * returned by gj_plan_destroy; `alloc` must stay valid until then.
 */
typedef struct gj_plan gj_plan;

/* Tuning of a join plan per size class c = floor(log2 |R_i|) (0..31). A zero
 * field selects the built-in rule. Tuning changes speed, never results. */
#define GJ_TUNE_CLASSES 32
typedef struct {
    int8_t part_log2[GJ_TUNE_CLASSES];    /* target rows per partition 2^v, v in 6..12 (rule: 11); the
                                             instance gets clamp(ceil(log2 |R_i|) - v, 0, 8) bits */
    int8_t bucket_shift[GJ_TUNE_CLASSES]; /* LDS hash buckets per build block: 2^(ceil(log2 rows) + shift),
                                             shift 0 or 1, capped at 2048 for 4096-row blocks (rule: 0) */
    int32_t scatter_variant;              /* partition scatter shape, 1..13 (rule: 0 = built-in) */
} gj_join_tuning;

/*
 * Plan for the batch of gj_join_batch (same layout and rules), with one
 * difference: instances are grouped into consecutive runs of at most 2^30 rows
 * per side, each run partitioned and joined as one segment, so the batch itself
 * may exceed 2^31 rows (each instance may not). Output columns hold
 * out_capacity rows (0 = the sum of |S_i|, which bounds every PK-FK batch);
 * rows past the capacity are dropped and reported by gj_join_plan_result.
 * mat must be GJ_MAT_GFTR or GJ_MAT_GFUR (GJ_MAT_AUTO picks GFTR). tuning may
 * be NULL (built-in rules). Work-unit room per instance assumes that no R
 * partition of it exceeds twice the build block (always true for unique R keys
 * and the default rules); otherwise the result reports GJ_ECAPACITY.
 * Synchronizes with `stream` once, to upload the per-instance parameters.
 */
int gj_join_plan_create(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts,
                        const gj_join_tuning *tuning, int64_t out_capacity, const gj_allocator *alloc,
                        void *stream, gj_plan **plan);

/* Enqueue one run of the plan on `stream` (kernels only). */
int gj_plan_run(gj_plan *plan, void *stream);

/* Capture one run into a HIP graph and instantiate it (once per plan; the
 * capture itself runs nothing). */
int gj_plan_capture(gj_plan *plan);

/* Launch the captured graph on `stream` (one hipGraphLaunch). */
int gj_plan_launch(gj_plan *plan, void *stream);

/* Synchronizes with `stream` and reports the last run of a join plan: out
 * receives the plan's output columns (owned by the plan, valid until
 * gj_plan_destroy) and n_rows = |T|; out_offsets (host, n_instances + 1) the
 * first output row of each instance. Returns GJ_ECAPACITY, with n_rows set to
 * the required output rows, when the output or the work-unit room was too
 * small; the columns then hold a truncated result. */
int gj_join_plan_result(gj_plan *plan, void *stream, gj_join_out *out, int64_t *out_offsets);

typedef struct {
    int64_t launches_per_run; /* kernels one run enqueues */
    int64_t groups;           /* consecutive instance runs of the plan */
    int64_t scratch_bytes;    /* device scratch the plan holds */
    int64_t output_bytes;     /* device output the plan holds */
    int64_t unit_capacity;    /* work units the plan has room for */
} gj_plan_info;
int gj_plan_get_info(const gj_plan *plan, gj_plan_info *info);

/* Releases the graph and every block of device memory of the plan. */
int gj_plan_destroy(gj_plan *plan);

/*
 * Autotuner for join plans: for each size class present in the batch, copies up
 * to 64 of its instances into a staging batch and times plan runs (graph
 * launches, median of `reps`) over the candidates part_log2 in {9, 10, 11, 12}
 * x bucket_shift in {0, 1}; then times the 13 scatter variants with the chosen
 * table on the staging batch of the class with the most rows. Writes the best
 * table to *out. Allocates and synchronizes freely; results never change.
 */
int gj_join_autotune(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts, int32_t reps,
                     const gj_allocator *alloc, void *stream, gj_join_tuning *out);

typedef enum { GJ_SUM = 1, GJ_COUNT = 2, GJ_MIN = 3, GJ_MAX = 4 } gj_agg_op;
typedef struct {
    int32_t col; /* value column index (ignored for GJ_COUNT) */
    int32_t op;  /* gj_agg_op */
} gj_agg;

/* Group-by algorithm: hash (Section 4.2, Algorithm 1), sort (Section 4.1.3),
 * partition (Section 4.3), or sort on dictionary-encoded keys (Section 4.4:
 * the distinct keys get codes 0..g-1 in key order from a global hash table,
 * rows are sorted on the code bytes that vary, then reduced; always GFTR). */
typedef enum {
    GJ_GB_AUTO = 0,
    GJ_GB_HASH = 1,
    GJ_GB_SORT = 2,
    GJ_GB_PARTITION = 3,
    GJ_GB_SORT_DE = 4
} gj_gb_algo;
typedef struct {
    int32_t algo;       /* gj_gb_algo */
    int32_t mat;        /* gj_mat, for sort and partition */
    int32_t radix_bits; /* partition group-by: total partition bits, 1..16 */
    int32_t block_size; /* reserved; 0 or 256 */
    float ht_occupancy; /* hash: target load of the global table, sized from the HyperLogLog
                           estimate of the group count (0: 0.45; at most 64). A table that turns
                           out too small (a row finds no slot within 4096 probes, as loads above 1
                           make sure of) is replaced by one of 1.5 slots per row and the insert
                           runs again; the result does not depend on it. */
    int32_t lds_budget; /* hash: bytes of LDS per workgroup for aggregation records (0: 160 KB,
                           a compute unit's LDS). When the group ids, cut into at most 64
                           consecutive ranges, fit that budget per range, every group
                           aggregates in LDS (one workgroup per row chunk and id range);
                           otherwise the ids that fit min(budget, 64 KiB) aggregate in LDS
                           and the rest with global atomics */
    float skew_hint;    /* expected Zipf factor of the keys, for automatic choices (0: unknown) */
} gj_groupby_opts;

/* Group-by output A(k, a_1..a_n): one row per distinct key. aggs[i] is the
 * aggregate requested by the i-th gj_agg: SUM and COUNT as int64, MIN and MAX
 * in the value column's dtype. The caller provides aggs with room for n_aggs
 * pointers; the library allocates each column. */
typedef struct {
    void *key;
    void **aggs;
    int64_t n_groups;
} gj_groupby_out;

/*
 * Grouped aggregation with one group key and reducible aggregates
 * (Section 2.2): for each distinct key, COUNT(*) and SUM/MIN/MAX of value
 * columns. Keys are GJ_I32 or GJ_I64; value columns GJ_I32 or GJ_I64 (Section
 * 5.2 evaluates 8-byte payloads), mixed freely. SUM is int64: exact for int32
 * values (at most 2^31 rows), modulo 2^64 for int64 values; MIN and MAX keep
 * the value column's dtype. Group order: ascending key for the sort algorithms (with or without
 * dictionary encoding); unspecified (but deterministic) for partition;
 * unspecified for hash.
 * Synchronizes with `stream` to read the group count.
 */
int gj_groupby(gj_col key, const gj_col *vals, int32_t n_vals, int64_t n_rows,
               const gj_agg *aggs, int32_t n_aggs, const gj_groupby_opts *opts,
               const gj_allocator *alloc, void *stream, gj_groupby_out *out);

/* A batch of independent group-by inputs stored back to back: instance i owns
 * rows [offsets[i], offsets[i+1]) of the key and of every value column. */
typedef struct {
    gj_col key;
    const gj_col *vals;     /* n_vals GJ_I32 columns */
    int32_t n_vals;         /* 0..8 */
    const int64_t *offsets; /* host array of n_instances + 1 row offsets, offsets[0] = 0 */
    int32_t n_instances;
} gj_gb_batch;

/*
 * Plan (see gj_join_plan_create) for the partition group-by of Section 4.3 on
 * every instance of a batch: one hashed, segmented partitioning pass (instance i
 * with its own bits: radix_bits of opts, or clamp(ceil(log2 N_i) - 10, 0, 8)),
 * group discovery in LDS, and a persistent aggregation over all instances'
 * partitions (per partition: one group in registers, records in LDS when they
 * fit, else global atomics). Output groups are dense over the batch, instance by
 * instance, in the order of gj_groupby's partition algorithm; the output columns
 * hold sum(N_i) groups. opts->algo must be GJ_GB_AUTO or GJ_GB_PARTITION; mat
 * GFTR (default) or GFUR. A partition with more than 4096 distinct keys cannot
 * be discovered in LDS: the result then reports GJ_ECAPACITY (use gj_groupby
 * for such instances; keeping N_i <= 2^20 makes this practically impossible
 * unless the keys are chosen to collide). Runs, capture, launch and destroy are
 * the gj_plan_* calls.
 */
int gj_groupby_plan_create(const gj_gb_batch *B, const gj_agg *aggs, int32_t n_aggs,
                           const gj_groupby_opts *opts, const gj_allocator *alloc, void *stream,
                           gj_plan **plan);

/* Synchronizes with `stream` and reports the last run of a group-by plan: out
 * receives the plan's key and aggregate columns (owned by the plan) and n_groups
 * the total; group_offsets (host, n_instances + 1) the first group of each
 * instance. GJ_ECAPACITY when a partition overflowed its LDS table. */
int gj_groupby_plan_result(gj_plan *plan, void *stream, gj_groupby_out *out, int64_t *group_offsets);

/*
 * Eager form of the group-by plan (no counterpart in the paper; the partition
 * group-by of Section 4.3 applied to every instance at once): plans the batch,
 * runs it once on `stream` and returns columns of exactly n_groups rows
 * allocated through `alloc` (owned by the caller; out->aggs has room for n_aggs
 * pointers; SUM and COUNT are int64, MIN and MAX int32). group_offsets (host,
 * n_instances + 1) receives the first group of each instance. Same inputs,
 * options and errors as gj_groupby_plan_create and gj_groupby_plan_result; on
 * error nothing stays allocated. Synchronizes with `stream`.
 */
int gj_groupby_batch(const gj_gb_batch *B, const gj_agg *aggs, int32_t n_aggs, const gj_groupby_opts *opts,
                     const gj_allocator *alloc, void *stream, gj_groupby_out *out, int64_t *group_offsets);

/* Digit source of the partition primitive. */
typedef enum {
    GJ_DIGIT_BITS = 0,   /* the key's unsigned two's-complement bit pattern */
    GJ_DIGIT_HASH = 1,   /* MurmurHash3 32-bit finalizer of the key (8-byte keys: of lo ^ hi) */
    GJ_DIGIT_ORDERED = 2 /* the key with its sign bit flipped (unsigned order = signed order) */
} gj_digit_mode;

/*
 * The radix-partition primitive of Section 2.3, on a key column plus up to 8
 * value columns: rows are reordered stably by digit = bits
 * [bit_lo, bit_lo + bits) of the digit source, in `passes` passes (MSD, at
 * most 8 bits each). bits is 1..16; passes is 0 (auto), 1 or 2.
 * out_key / out_cols[i] receive the reordered columns (device, n_rows each,
 * caller-allocated). If out_rowid is not NULL it receives, as int32, the input
 * row index of each output row. If out_offsets is not NULL it receives 2^bits+1
 * int32 partition offsets (device). Scratch comes from `alloc`.
 */
int gj_partition(gj_col key, const gj_col *cols, int32_t n_cols, int64_t n_rows,
                 int32_t bit_lo, int32_t bits, int32_t passes, int32_t mode,
                 void *out_key, void *const *out_cols, void *out_rowid, int32_t *out_offsets,
                 const gj_allocator *alloc, void *stream);

/*
 * gj_partition without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. One pass only (bits 1..8, so passes is implied); otherwise
 * the arguments, the output layout and the result are those of gj_partition,
 * except that out_offsets (2^bits + 1 int32, device) is required. The caller
 * owns every input and output buffer. The scratch of the pass (chunk table,
 * per-chunk digit histograms, scan partials: about 4.2 MB at most, for any row
 * count) lives in one statically allocated device array of
 * gj_partition_noalloc_scratch_bytes() bytes per device, which the library
 * holds until the process ends. A request needing more returns GJ_ECAPACITY.
 * All calls on one device share that array: calls that overlap on a device
 * (concurrent streams or threads) race and must not be issued; calls in
 * sequence on any streams of the device are fine. Enqueues kernels only (no
 * allocation, copy, memset or synchronization); the first call on a device
 * looks up the array's device address.
 */
int gj_partition_noalloc(gj_col key, const gj_col *cols, int32_t n_cols, int64_t n_rows,
                         int32_t bit_lo, int32_t bits, int32_t mode, void *out_key,
                         void *const *out_cols, void *out_rowid, int32_t *out_offsets, void *stream);

/* Size in bytes of the static scratch array of gj_partition_noalloc (per device). */
size_t gj_partition_noalloc_scratch_bytes(void);

/* ---- Machine measurements ----------------------------------------------------
 * The two kernels behind the cost model's constants (Section 4.1.1, Table 1).
 *
 * gj_stream_copy: dst[0..bytes) = src[0..bytes) with 16-byte loads and stores
 * (both buffers device memory, 16-byte aligned, not overlapping): the plain
 * streaming rate that bounds every pass over HBM.
 *
 * gj_gather_i32: out[i] = values[map[i]] for i < n (device buffers): map and
 * out are streamed, values is read where map points. A map that walks
 * partition-local rows (clustered) reads values in few cache lines; a random
 * permutation (unclustered) reads one line per value. Their time ratio s gives
 * B_G / B_R = (12 s - 8) / 4 (Section 4.1.1). Entries of map outside
 * [0, n_values) give 0. Returns GJ_EOVERFLOW for n_values > 2^31 - 1.
 */
int gj_stream_copy(const void *src, void *dst, size_t bytes, void *stream);
int gj_gather_i32(const int32_t *map, const int32_t *values, int64_t n_values, int32_t *out, int64_t n,
                  void *stream);

/* ---- Algorithm selection -----------------------------------------------------
 * Workload features (12 floats, each scaled to about [0, 1]):
 *   [0] 1 for a join, 0 for a group-by
 *   [1] log2 |R| / 32 (group-by: log2 N / 32)
 *   [2] log2 |S| / 32 (group-by: 0)
 *   [3] log2 g / 32 (join: log2 |R| / 32; group-by: the HyperLogLog estimate)
 *   [4] key bytes / 8
 *   [5] R payload columns / 8 (group-by: value columns / 8)
 *   [6] S payload columns / 8 (group-by: key bytes that vary between rows / 8)
 *   [7] Zipf factor of the foreign keys or group keys / 1.2 (the hint; 0 without)
 *   [8] match ratio (the hint, else 1; group-by: 1)
 *   [9] log2(|S| / |R|) / 32 (group-by: log2(N / g) / 32)
 *   [10] log2 expected output rows / 32 (group-by: log2 of the LDS bytes the hash
 *        group-by's records of all groups take, estimate x record bytes / 32)
 *   [11] log2 input bytes / 48
 * Classes: 0 partitioned-hash join GFTR, 1 partitioned-hash join GFUR,
 * 2 hash, 3 sort, 4 partition group-by, 5 sort group-by on dictionary-encoded
 * keys, 6 sort-merge join GFTR. op_kind 0 = join (classes 0, 1, 6 valid),
 * 1 = group-by (classes 2-5 valid). */
#define GJ_SELECT_CLASSES 7

/* The analytical model: predicted seconds per class (infinity for invalid
 * classes), built on the paper's bandwidth models (Sections 4.1.3, 4.1.4) over
 * this implementation's passes, with MI355X constants. */
int gj_cost_model(const float features[12], int32_t op_kind, double predicted_seconds[GJ_SELECT_CLASSES]);

/* The class to run: the learned network's argmax when weights are loaded and its
 * output is finite, else the cost model's argmin. probs (may be NULL) receives
 * the network's probabilities, or a one-hot of the cost model's choice. The
 * choice never changes a result. */
int gj_select(const float features[12], int32_t op_kind, int32_t *choice, float probs[GJ_SELECT_CLASSES]);

/* The feature vector an automatic join choice (mat or algo GJ_*_AUTO) uses for
 * these relations and options (host only; no device access). */
int gj_join_features(const gj_rel *R, const gj_rel *S, const gj_join_opts *opts, float features[12]);

/* The feature vector an automatic group-by choice uses for these columns and
 * aggregates (value columns and aggregates as gj_groupby takes them; only the
 * value widths are read): reads the keys once on `stream` (group-count estimate
 * and varying key bytes) and synchronizes.
 * The estimate comes from the sketch kernel gj_groupby runs for the same
 * opts->algo and opts->radix_bits (automatic and partition choices also count a
 * per-chunk hash histogram there); both kernels give the same estimate.
 * Scratch from `alloc` (NULL: hipMallocAsync). */
int gj_groupby_features(gj_col key, const gj_col *vals, int32_t n_vals, const gj_agg *aggs, int32_t n_aggs,
                        int64_t n_rows, const gj_groupby_opts *opts, const gj_allocator *alloc, void *stream,
                        float features[12]);

/* Load trained network weights (host array of GJ_MLP_PARAMS floats; NULL or n = 0
 * unloads them). Thread-safe. */
int gj_selector_set_weights(const float *params, int32_t n);

/* Override the cost model's constants (bytes/s of streaming, B_G/B_R of 4-byte
 * gathers, scattered global atomics per second). */
int gj_set_cost_constants(double seq_bytes_per_s, double rand_ratio, double atomic_rate);

/* The cost model's current constants (host pointers). */
int gj_get_cost_constants(double *seq_bytes_per_s, double *rand_ratio, double *atomic_rate);

/* ---- Selector network ------------------------------------------------------
 * 12 workload features -> 64 -> 64 (ReLU) -> 7 logits over the classes above,
 * softmax over the classes valid for the sample (mask), loss = batch mean of
 * -log p[label]. FP32; parameters are one flat device vector of GJ_MLP_PARAMS
 * floats: W1 (64x12 row-major), b1, W2 (64x64), b2, W3 (7x64), b3. X is
 * [batch x 12], mask [batch x 7] (1 = valid class), labels [batch], all device
 * arrays. Results are deterministic (fixed summation order). */
#define GJ_MLP_PARAMS 5447

/* probs [batch x 7] = masked softmax of the network's logits. */
int gj_mlp_forward(const float *params, const float *X, const float *mask, int32_t batch, float *probs,
                   const gj_allocator *alloc, void *stream);

/* grad [GJ_MLP_PARAMS] = gradient of the batch-mean cross-entropy; *loss (device,
 * may be NULL) = that loss. */
int gj_mlp_grad(const float *params, const float *X, const float *mask, const int32_t *labels,
                int32_t batch, float *grad, float *loss, const gj_allocator *alloc, void *stream);

/* One Adam step (Kingma and Ba, 2015) with bias correction at step t >= 1,
 * updating params, m and v in place (device arrays of GJ_MLP_PARAMS). */
int gj_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                float beta2, float eps, void *stream);

/* Per-kernel timing of this thread's launches (for benchmarks and phase
 * breakdowns). */
typedef struct {
    char name[48];     /* kernel name */
    int64_t launches;  /* launches recorded */
    double total_ms;   /* sum of event-measured durations on the launch stream */
    double alg_bytes;  /* sum of algorithmic bytes: compulsory reads + writes */
} gj_kernel_stat;

/* Start recording: every later launch made by this thread is bracketed by two
 * HIP events on its stream. Adds two event records per launch. */
int gj_profile_start(void);

/* Stop recording, wait for the recorded events, and write up to `cap` per-kernel
 * aggregates to `stats` (host memory); *n_out receives the number of distinct
 * kernels. Returns GJ_EHIP if an event could not be read. */
int gj_profile_stop(gj_kernel_stat *stats, int32_t cap, int32_t *n_out);

/* Thread-local text of the last error on this thread ("" if none). */
const char *gj_last_error(void);

/* Library version string. */
const char *gj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GJ_H */
