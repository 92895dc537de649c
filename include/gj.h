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
#define GJ_EUNSUPPORTED (-4) /* a valid request this build does not implement */
#define GJ_ECAPACITY (-5)    /* a caller-sized output is too small */
#define GJ_EOVERFLOW (-6)    /* more than 2^31 - 1 rows in one relation */

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

/* Join options; 0 in any field means "choose automatically". Options change
 * speed, never results. */
typedef struct {
    int32_t mat;               /* gj_mat */
    int32_t unique_build_keys; /* hint that R.key is unique; results stay exact if wrong */
    int32_t radix_bits;        /* total partition bits, 1..16 */
    int32_t passes;            /* 1 or 2 (each pass uses at most 8 bits) */
    int32_t block_size;        /* reserved; must be 0 or 256 */
    float ht_occupancy;        /* reserved */
    int32_t lds_budget;        /* max R rows per build block, 64..4096 */
    uint64_t flags;            /* reserved, must be 0 */
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
 * Synchronizes with `stream` twice (unit count and output size).
 */
int gj_join(const gj_rel *R, const gj_rel *S, const gj_join_opts *opts,
            const gj_allocator *alloc, void *stream, gj_join_out *out);

typedef enum { GJ_SUM = 1, GJ_COUNT = 2, GJ_MIN = 3, GJ_MAX = 4 } gj_agg_op;
typedef struct {
    int32_t col; /* value column index (ignored for GJ_COUNT) */
    int32_t op;  /* gj_agg_op */
} gj_agg;

/* Group-by algorithm: hash (Section 4.2, Algorithm 1), sort (Section 4.1.3)
 * or partition (Section 4.3). */
typedef enum { GJ_GB_AUTO = 0, GJ_GB_HASH = 1, GJ_GB_SORT = 2, GJ_GB_PARTITION = 3 } gj_gb_algo;
typedef struct {
    int32_t algo;       /* gj_gb_algo */
    int32_t mat;        /* gj_mat, for sort and partition */
    int32_t radix_bits; /* partition group-by: total partition bits, 1..16 */
    int32_t block_size; /* reserved; 0 or 256 */
    float ht_occupancy; /* reserved */
    int32_t lds_budget; /* bytes of LDS for the aggregation buffer; forces global fallback when small */
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
 * columns. Keys are GJ_I32 or GJ_I64; value columns GJ_I32. SUM is exact in
 * int64. Group order: ascending key for the sort algorithm; unspecified (but
 * deterministic) for partition; unspecified for hash.
 * Synchronizes with `stream` to read the group count.
 */
int gj_groupby(gj_col key, const gj_col *vals, int32_t n_vals, int64_t n_rows,
               const gj_agg *aggs, int32_t n_aggs, const gj_groupby_opts *opts,
               const gj_allocator *alloc, void *stream, gj_groupby_out *out);

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
