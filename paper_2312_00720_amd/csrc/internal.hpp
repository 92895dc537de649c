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

// ---- prof.hip: optional per-launch event timing ------------------------------------
// When profiling is on for the calling thread, every launch made through GJ_LAUNCH
// is bracketed by two HIP events on its stream and tagged with its algorithmic
// byte count (the compulsory reads and writes of the method, no re-reads).
void prof_before(const char *name, double alg_bytes, hipStream_t s);
void prof_after(hipStream_t s);

#define GJ_LAUNCH(name, alg_bytes, kernel, grid, block, shm, stream, ...)              \
    do {                                                                                \
        ::gj::prof_before(name, (double)(alg_bytes), stream);                           \
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);              \
        GJ_LAUNCHED(name);                                                              \
        ::gj::prof_after(stream);                                                       \
    } while (0)

// Memory for one C-ABI call. Scratch is released at the end of the call;
// outputs are released only if the call fails.
class Ctx {
  public:
    Ctx(const gj_allocator *a, hipStream_t s) : alloc_(a), stream(s) {}
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
        if (!p) return;
        if (alloc_ && alloc_->alloc) {
            if (alloc_->free) alloc_->free(p, alloc_->ctx);
        } else {
            (void)hipFreeAsync(p, stream);
        }
    }
    std::vector<void *> scratch_, outputs_;
    bool committed_ = false;
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
void partition_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                   uint32_t n, int bit_lo, int bits, int passes, int mode, uint32_t *poff);

// One stable pass over nseg segments (device offsets seg_off[0..nseg]), the digit of
// segment s being the low seg_bits[s] (<= 8) bits of the key: partition (s, d) gets
// index s * 256 + d in poff (nseg * 256 + 1 entries). Used for batches of instances.
void partition_run_segments(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                            uint32_t n, const uint32_t *seg_off, uint32_t nseg, const uint8_t *seg_bits,
                            uint32_t *poff);

// Stable LSD radix sort of n rows by the signed key (8 bits per pass; bytes that are
// equal in every key are skipped). Moves the columns of `cols` along.
void sort_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols, uint32_t n);

// ---- groupby.hip ----------------------------------------------------------------------
// Each returns the number of groups and allocates the key and aggregate outputs
// through ctx.output(). groupby_partition returns -1 with *fell_back = 1 when a
// partition holds more distinct keys than its LDS table.
int64_t groupby_partition(Ctx &ctx, int key_bytes, const void *key, const int32_t *const *vals, int n_vals,
                          uint32_t n, const gj_agg *aggs, int n_aggs, bool gfur, int bits, void **out_key,
                          void **out_aggs, int *fell_back);
int64_t groupby_hash(Ctx &ctx, int key_bytes, const void *key, const int32_t *const *vals, int n_vals, uint32_t n,
                     const gj_agg *aggs, int n_aggs, int lds_budget, void **out_key, void **out_aggs);
int64_t groupby_sort(Ctx &ctx, int key_bytes, const void *key, const int32_t *const *vals, int n_vals, uint32_t n,
                     const gj_agg *aggs, int n_aggs, bool gfur, void **out_key, void **out_aggs);

// ---- select.hip -----------------------------------------------------------------------
// Class 0..4 for the features (see gj.h); the network when loaded, else the cost model.
int select_algorithm(const float *features, int op_kind, float *probs_out);
void features_join(float *f, double nr, double ns, int key_bytes, int cr, int cs);
void features_groupby(float *f, double n, int key_bytes, int nv);

// ---- join.hip -------------------------------------------------------------------------
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
int64_t join_partitioned(Ctx &ctx, int key_bytes, const JoinSide &R, const JoinSide &S, int bits,
                         int r_block, bool gfur, JoinOut *out, const uint8_t *seg_bits = nullptr,
                         uint32_t n_inst = 0, uint64_t *inst_off = nullptr);

}  // namespace gj
