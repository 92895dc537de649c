// Host-side internals of libgj: error model, scratch and output memory, and
// the launchers each kernel file exports to the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/gj.h"
#include "common.hpp"

namespace gj {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define GJ_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::gj::Error(GJ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GJ_LAUNCHED(name)                                                                   \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess)                                                               \
            throw ::gj::Error(GJ_EHIP, std::string("launch ") + name + ": " + hipGetErrorString(e_)); \
    } while (0)

inline void require(bool ok, const std::string &msg, int code = GJ_EINVAL) {
    if (!ok) throw Error(code, msg);
}

// The thread's message for gj_last_error() (capi.hip): fail() sets it and returns code.
int fail(int code, const std::string &msg);
void clear_error();

// ---- prof.hip: optional per-launch event timing ------------------------------------
// When profiling is on for the calling thread, every launch made through GJ_LAUNCH
// is bracketed by two HIP events on its stream and tagged with its algorithmic
// byte count (the compulsory reads and writes of the method, no re-reads).
void prof_before(const char *name, double alg_bytes, hipStream_t s);
void prof_after(hipStream_t s);

// While a plan measures the memory of its run (plan.hip), launches are counted
// and skipped: no kernel runs and no placeholder address is touched.
extern thread_local bool g_dry_run;
extern thread_local int64_t g_dry_launches;

#define GJ_LAUNCH(name, alg_bytes, kernel, grid, block, shm, stream, ...)              \
    do {                                                                                \
        if (::gj::g_dry_run) {                                                          \
            ++::gj::g_dry_launches;                                                     \
            break;                                                                      \
        }                                                                               \
        ::gj::prof_before(name, (double)(alg_bytes), stream);                           \
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);              \
        GJ_LAUNCHED(name);                                                              \
        ::gj::prof_after(stream);                                                       \
    } while (0)

// Pauses the per-launch profiler for a scope (HIP graph capture records no events).
struct ProfPause {
    ProfPause();
    ~ProfPause();
    bool was;
};

// Bump allocation over one preallocated device block (a plan's scratch). With
// base == nullptr it only measures: addresses are placeholders, never used.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0, peak = 0;
};

// Memory for one C-ABI call. Scratch is released at the end of the call;
// outputs are released only if the call fails. Over an arena, nothing is released.
class Ctx {
  public:
    Ctx(const gj_allocator *a, hipStream_t s) : alloc_(a), stream(s) {}
    Ctx(Arena *ar, hipStream_t s) : alloc_(nullptr), stream(s), arena_(ar) {}
    ~Ctx() {
        for (void *p : scratch_) release(p);
        if (!committed_)
            for (void *p : outputs_) release(p);
    }
    void *scratch(size_t bytes) {
        void *p = get(bytes);
        scratch_.push_back(p);
        return p;
    }
    template <typename T>
    T *scratch_n(size_t n) { return static_cast<T *>(scratch(n * sizeof(T))); }
    void *output(size_t bytes) {
        void *p = get(bytes);
        outputs_.push_back(p);
        return p;
    }
    void commit() { committed_ = true; }
    const gj_allocator *alloc_;
    hipStream_t stream;

  private:
    void *get(size_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (arena_) {
            const size_t off = arena_->used;
            arena_->used += bytes;
            if (arena_->used > arena_->peak) arena_->peak = arena_->used;
            if (!arena_->base) return reinterpret_cast<char *>(uintptr_t(1) << 44) + off;
            if (arena_->used > arena_->size) throw Error(GJ_ENOMEM, "plan scratch exhausted");
            return arena_->base + off;
        }
        void *p = nullptr;
        if (alloc_ && alloc_->alloc) {
            p = alloc_->alloc(bytes, alloc_->ctx);
        } else {
            if (hipMallocAsync(&p, bytes, stream) != hipSuccess) p = nullptr;
        }
        if (!p) throw Error(GJ_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes failed");
        return p;
    }
    void release(void *p) {
        if (!p || arena_) return;
        if (alloc_ && alloc_->alloc) {
            if (alloc_->free) alloc_->free(p, alloc_->ctx);
        } else {
            (void)hipFreeAsync(p, stream);
        }
    }
    std::vector<void *> scratch_, outputs_;
    bool committed_ = false;
    Arena *arena_ = nullptr;
};

template <typename T>
inline T read_back(const T *dev, hipStream_t s) {
    T v{};
    GJ_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    GJ_HIP(hipStreamSynchronize(s));
    return v;
}

// ---- scan.hip ---------------------------------------------------------------------
// Exclusive prefix sum of n elements (in == out allowed). If total != nullptr the
// grand total is written there (device). Scratch comes from ctx.
void scan_exclusive_u32(Ctx &ctx, const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total);
void scan_exclusive_u64(Ctx &ctx, const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *total);
// The same over min(nmax, *n_dev * mult) elements, the count read on the device
// (launch sizes depend on nmax only).
void scan_exclusive_u64_dev(Ctx &ctx, const uint64_t *in, uint64_t *out, uint64_t nmax, const uint32_t *n_dev,
                            uint32_t mult, uint64_t *total);
void fill_u32(hipStream_t s, uint32_t *p, uint32_t v, uint64_t n);
void fill_u64(hipStream_t s, uint64_t *p, uint64_t v, uint64_t n);

// ---- partition.hip ------------------------------------------------------------------
struct PartCols {
    int n = 0;                   // payload columns moved with the key
    const void *in[kMaxCols];
    void *out[kMaxCols];
    int width[kMaxCols];     // 4 or 8 bytes
    bool gen_rowid = false;      // append an int32 row-id column (output only, slot n)
    void *rowid_out = nullptr;
};

// Stable radix partition of n rows on digit bits [bit_lo, bit_lo + bits) of the
// digit source `mode`, in `passes` MSD passes. Writes 2^bits + 1 uint32 offsets to
// poff (device). n == 0 is allowed.
// hist8 (optional, one pass at bit_lo 0): per chunk of pass_chunk_rows(n) rows,
// the rows per value of the digit source's low 8 bits (chunk-major, 256 counts
// each), read by an earlier kernel; the pass then folds it to its own digit
// instead of reading the keys for a histogram.
void partition_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                   uint32_t n, int bit_lo, int bits, int passes, int mode, uint32_t *poff,
                   const uint32_t *hist8 = nullptr);
// Rows per chunk of a single-segment pass over n rows with the current scatter shape.
uint32_t pass_chunk_rows(uint32_t n);

// One stable pass over nseg segments (device offsets seg_off[0..nseg]), the digit of
// segment s being the low seg_bits[s] (<= 8) bits of the digit source `mode` (the key
// bits, or its hash): partition (s, d) gets index s * 256 + d in poff (nseg * 256 + 1
// entries). Used for batches of instances.
void partition_run_segments(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                            uint32_t n, const uint32_t *seg_off, uint32_t nseg, const uint8_t *seg_bits,
                            uint32_t *poff, int mode = kDigitBits);

// Stable LSD radix sort of n rows by the signed key (8 bits per pass; bytes that are
// equal in every key are skipped). Moves the columns of `cols` along.
void sort_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols, uint32_t n);

// Scatter tile shape for the calling thread: 0 = default (or GJ_SCATTER_SHAPE),
// 1..kScatterVariants = a compiled (block, rows per thread, column group) shape.
constexpr int kScatterVariants = 14;
void set_scatter_variant(int v);

// ---- groupby.hip ----------------------------------------------------------------------
// Value columns of a group-by: device pointers and widths (4 or 8 bytes).
struct ValCols {
    int n = 0;
    const void *col[8] = {};
    int width[8] = {};
};
// Each returns the number of groups and allocates the key and aggregate outputs
// through ctx.output(). groupby_partition returns -1 with *fell_back = 1 when a
// partition holds more distinct keys than its LDS table.
// Estimated number of distinct keys (HyperLogLog, about 3% standard error);
// synchronizes with the stream.
// varying_bytes (optional) receives how many bytes of the order-preserving key
// differ between rows (the passes a radix sort of the raw keys takes).
// hist8 (optional): also count, per chunk of pass_chunk_rows(n) rows, the rows
// per low 8 bits of the key's hash (the partition group-by's digit), in the same
// read; *hist8 receives the scratch array.
double estimate_groups(Ctx &ctx, int key_bytes, const void *key, uint32_t n, int *varying_bytes = nullptr,
                       const uint32_t **hist8 = nullptr);
// hist8 (optional): the counts estimate_groups made for a single pass.
int64_t groupby_partition(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc,
                          uint32_t n, const gj_agg *aggs, int n_aggs, bool gfur, int bits, void **out_key,
                          void **out_aggs, int *fell_back, const uint32_t *hist8 = nullptr);
// g_est > 0 sizes the global table for about that many groups at load `occupancy`
// (<= 0: 0.45); a table found too small is replaced by one of 1.5 slots per row.
int64_t groupby_hash(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                     const gj_agg *aggs, int n_aggs, int lds_budget, double g_est, float occupancy, void **out_key,
                     void **out_aggs);
int64_t groupby_sort(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                     const gj_agg *aggs, int n_aggs, bool gfur, void **out_key, void **out_aggs);
// Sort-based group-by with dictionary-encoded keys (SGB-DE-TR): Algorithm 1's
// table assigns ids, the sorted distinct keys give each id its rank, rows are
// sorted on 4-byte codes over the code bytes that vary, then reduced in order.
int64_t groupby_sort_de(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                        const gj_agg *aggs, int n_aggs, double g_est, float occupancy, void **out_key,
                        void **out_aggs);

// Partition group-by of a batch of instances (segments seg_off[0..nseg] of the
// columns) without any host read: one hashed segmented partition pass (instance i
// with seg_bits[i] bits), discovery, a persistent aggregation over the device unit
// count, outputs at group rows *pl.out_base + (dense position over the batch).
struct PgbPlanned {
    uint32_t cap_units;          // aggregation units room (an exact bound)
    const uint64_t *out_base;    // device: first output group of this call
    uint64_t *next_base;         // device: receives out_base + groups
    uint32_t *status;            // device: [0] LDS table overflow flag, [1] units
    void *out_key;
    void *out_aggs[16];
    uint64_t out_cap;            // rows of the output columns past out_base
    uint32_t lds_bytes;          // dynamic LDS of the aggregation kernel
    uint64_t *inst_goff;         // device: nseg + 1 first output groups per instance
};
void groupby_partition_segments(Ctx &ctx, int key_bytes, const void *key, const int32_t *const *vals, int n_vals,
                                uint32_t n, const gj_agg *aggs, int n_aggs, bool gfur, const uint32_t *seg_off,
                                uint32_t nseg, const uint8_t *seg_bits, const PgbPlanned &pl);
uint32_t pgb_plan_lds_bytes(int key_bytes);

// ---- select.hip -----------------------------------------------------------------------
// Class 0..4 for the features (see gj.h); the network when loaded, else the cost model.
int select_algorithm(const float *features, int op_kind, float *probs_out);
// The feature vectors the automatic choices use (gj.h lists the features):
// hints <= 0 mean unknown (join: every S row matches, uniform keys).
void features_join(float *f, double nr, double ns, int key_bytes, int cr, int cs, float mr_hint, float skew_hint);
void features_groupby(float *f, double n, int key_bytes, int nv, double g_est, int varying_bytes, float skew_hint,
                      double rec_bytes);
// Bytes of one group's LDS record in the hash group-by (padded to whole 64-bit words).
size_t hgb_record_bytes(const gj_agg *aggs, int n_aggs, const int *val_w);

// ---- join.hip -------------------------------------------------------------------------
// Work-unit geometry. An R build block of at most r_block rows runs in one of
// three kernel shapes, 4096, 8192 or 16384 table rows (16 rows per thread), and
// a work unit probes an S piece of twice the table rows. 8-byte keys stop at 8192
// (their 16384-row table would not fit in one compute unit's LDS).
constexpr uint32_t kJoinMaxBuild = 16384;
inline uint32_t join_table_rows(int r_block) { return r_block <= 4096 ? 4096u : r_block <= 8192 ? 8192u : 16384u; }
inline uint32_t join_s_piece(int r_block) { return 2u * join_table_rows(r_block); }
inline int join_max_r_block(int key_bytes) { return key_bytes == 4 ? 16384 : 8192; }
inline void check_join_lds_budget(int lds_budget, int key_bytes) {
    require(lds_budget == 0 || (lds_budget >= 64 && lds_budget <= join_max_r_block(key_bytes)),
            key_bytes == 8 ? "lds_budget must be 64..8192 for 8-byte keys" : "lds_budget must be 64..16384");
}
// LDS the staged streaming write pass may use for one partition's R payloads.
constexpr size_t kJoinStagedLds = 144 * 1024;
// Default R build block and partition bits of a single join: partitions of
// about r_block / 2 rows leave room for variance. R relations of 2^24 rows and
// more use larger blocks, so that fewer partition bits (fewer, longer scatter
// runs per pass) suffice: 16384-row blocks (partitions of about 8192 rows) for
// GFTR with 4-byte keys when such a partition's R payload fits the staged
// write pass's LDS, else 8192-row blocks, whose 4096-row partitions keep the
// write pass's R gathers mostly in L2.
inline int join_default_r_block(uint64_t n_r, int key_bytes, bool gfur, int r_pay_bytes) {
    if (n_r < (1ull << 24)) return 4096;
    if (!gfur && key_bytes == 4 && (size_t)8192 * (size_t)r_pay_bytes <= kJoinStagedLds) return 16384;
    return 8192;
}
inline int join_default_bits(uint64_t n_r, int r_block) {
    const uint64_t target = (uint64_t)(r_block / 2 > 1 ? r_block / 2 : 1);
    const uint64_t parts = (n_r + target - 1) / target;
    int b = 0;
    while ((1ull << b) < parts) ++b;
    return b < 1 ? 1 : (b > 16 ? 16 : b);
}

struct JoinSide {
    const void *key;          // partitioned keys
    const void *pay[8];       // GFTR: partitioned payload columns; GFUR: original columns
    int width[8];
    int n_pay;
    const int32_t *rowid;     // GFUR: partitioned row ids; GFTR: nullptr
    const uint32_t *poff;     // partition offsets (2^bits + 1)
    uint32_t rows;            // rows of the relation
};
struct JoinOut {
    void *key;
    void *r[8];
    void *s[8];
};
// Runs work-unit generation, the count pass and, after sizing, the write pass on
// partitioned R and S. Output columns are allocated through ctx.output() with the
// key width and the payload widths of R and S. Returns the number of output rows.
// Batches (seg_bits != nullptr): partitions are (instance, digit) with index
// instance * 256 + digit, instance i using seg_bits[i] partition bits; inst_off
// (device, n_inst + 1) receives each instance's first output row.
//
// Planned runs (pl != nullptr) never read device memory from the host: the count
// and write passes are launched for pl->cap_units units and loop over the device
// count; output goes to the preallocated pl->out columns at rows *pl->out_base +
// (scanned position), stores at or past pl->out_cap are dropped; the output row
// count is written to pl->total, and *pl->out_base + total to pl->next_base when
// that is set. Returns 0 in that mode.
struct JoinPlanned {
    uint32_t cap_units;
    uint64_t out_cap;
    const uint64_t *out_base;
    uint64_t *total;
    uint64_t *next_base;
    JoinOut out;
    const uint8_t *seg_bshift;  // per instance extra LDS bucket bits (0 or 1)
    uint64_t expect_rows;       // for the profiler's byte count only
    uint32_t *units_out;        // device: receives the unit count
};
// Eager single joins only: what the unit count found, and the spread check. With
// check_spread set, a largest R partition beyond spread_limit rows returns -1
// before any pass runs (nothing was written, the caller may partition again).
// hashed_digits: the partitions come from hashed keys, so the LDS bucket hash
// uses every key bit (with key-bit digits it skips the partition bits).
// Sort-merge join (Section 3.1.1) on R and S already sorted by key (sort_run):
// Merge Path lower bounds, counts, scan and write. JoinSide::poff is unused.
// Output allocated through ctx.output(); returns the output rows (in key order).
int64_t join_sort_merge(Ctx &ctx, int key_bytes, const JoinSide &R, const JoinSide &S, bool gfur, JoinOut *out);

struct JoinStats {
    bool check_spread = false;
    uint32_t spread_limit = 0;
    bool hashed_digits = false;
    uint32_t max_r_rows = 0;
    bool multi_block = false;
};
int64_t join_partitioned(Ctx &ctx, int key_bytes, const JoinSide &R, const JoinSide &S, int bits,
                         int r_block, bool gfur, JoinOut *out, const uint8_t *seg_bits = nullptr,
                         uint32_t n_inst = 0, uint64_t *inst_off = nullptr, const JoinPlanned *pl = nullptr,
                         JoinStats *stats = nullptr);

}  // namespace gj
