// Grouped aggregation: partition-based (Section 4.3), hash-based (Section 4.2,
// Algorithm 1) and sort-based (Sections 3.2.2 and 4.1.3), the last also on
// dictionary-encoded keys (Section 4.4).
//
// Aggregates: COUNT, and SUM / MIN / MAX of int32 or int64 value columns. While
// a group is being aggregated in LDS, its record holds the 64-bit fields first
// (sums, and minima and maxima of 8-byte columns), then 32-bit counts, minima
// and maxima, padded to an even number of words. Outputs: SUM and COUNT as
// int64 (a sum of 8-byte values is taken modulo 2^64), MIN and MAX in the value
// column's type. Kernels hold a row's values as int when every column is 4
// bytes, else as long long.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace gj {

namespace {

constexpr int kMaxAggs = 16;
constexpr int kMaxVals = 8;
constexpr uint32_t kDiscoverCap = 4096;  // LDS table slots of the discover pass

// Bytes per slot of a partition's aggregation table in LDS: 4-byte keys share one
// 8-byte word with their group id (one read finds both), 8-byte keys keep the ids
// in a 16-bit array beside the keys.
constexpr uint32_t agg_slot_bytes(int key_bytes) { return key_bytes == 4 ? 8u : (uint32_t)key_bytes + 2u; }

// Slots (log2) of the aggregation table for a partition of g groups: a power of
// two of at least 1.5 g (load at most 2/3, short linear probes) and 64. At most
// kDiscoverCap keys go in; the key equal to the empty marker, when present, is
// counted in g but kept apart.
__host__ __device__ inline int agg_table_log2(uint32_t g) {
    const uint32_t keys = g < kDiscoverCap ? g : kDiscoverCap;
    int l = 6;
    while ((1u << l) * 2u < 3u * keys) ++l;
    return l;
}
constexpr uint32_t kUnitRows = 8192;     // rows per aggregation work unit
constexpr uint32_t kDiscoverUnit = 65536; // partitions above this size are discovered by several workgroups

struct AggSpec {
    int n;
    int op[kMaxAggs];   // GJ_SUM / GJ_COUNT / GJ_MIN / GJ_MAX
    int col[kMaxAggs];  // value column
    int word[kMaxAggs]; // word offset in an LDS record at an even word
    int word_odd[kMaxAggs];  // word offset in a record at an odd word (odd record sizes)
    int w8[kMaxAggs];   // MIN / MAX of an 8-byte column: a 64-bit field and output
    int words;          // record size in 4-byte words
    void *out[kMaxAggs];
};

struct ValSrc {
    int n;
    const void *col[kMaxVals];     // GFTR: partitioned/sorted columns; GFUR: original columns
    int w8[kMaxVals];              // 1 for an 8-byte column
    const int32_t *rowid;          // GFUR: row ids aligned with the keys; else nullptr
};

// MIN and MAX fields start at the identity of their width; a 4-byte field
// narrows a 64-bit running value, whose identity lies beyond int32.
__device__ __forceinline__ int narrow_min(long long x) { return (int)(x < INT32_MAX ? x : INT32_MAX); }
__device__ __forceinline__ int narrow_max(long long x) { return (int)(x > INT32_MIN ? x : INT32_MIN); }

// Word offset of field j in a record starting `at` words past an 8-byte aligned
// base. The hash group-by's records (ODD) take an odd number of words when any
// field is 32 bits wide (no padding word, so one more group fits every 9 or so):
// a record at an odd word shifts its first 32-bit field in front of the 64-bit
// ones, which then stay 8-byte aligned. Other records are padded to an even
// size (the partition group-by's aggregation keeps one more wave per SIMD
// without the per-field parity test).
template <bool ODD>
__device__ __forceinline__ int field_at(const AggSpec &s, int j, uint32_t at) {
    if constexpr (ODD) return (at & 1u) ? s.word_odd[j] : s.word[j];
    else return s.word[j];
}
template <bool ODD>
__device__ __forceinline__ uint32_t word_parity(const uint32_t *rec) {
    if constexpr (ODD) return (uint32_t)((uintptr_t)rec >> 2) & 1u;
    else return 0u;
}

template <bool ODD = false>
__device__ __forceinline__ void rec_init(uint32_t *rec, const AggSpec &s) {
    const uint32_t par = word_parity<ODD>(rec);
    for (int j = 0; j < s.n; ++j) {
        uint32_t *p = rec + field_at<ODD>(s, j, par);
        switch (s.op[j]) {
            case GJ_SUM: p[0] = 0; p[1] = 0; break;
            case GJ_COUNT: p[0] = 0; break;
            case GJ_MIN:
                if (s.w8[j]) *reinterpret_cast<long long *>(p) = INT64_MAX;
                else p[0] = (uint32_t)INT32_MAX;
                break;
            default:
                if (s.w8[j]) *reinterpret_cast<long long *>(p) = INT64_MIN;
                else p[0] = (uint32_t)INT32_MIN;
                break;
        }
    }
}

// Write (plain) or fold (atomic) an LDS record into output group o.
template <bool ODD = false>
__device__ __forceinline__ void rec_flush(const uint32_t *rec, const AggSpec &s, uint64_t o, bool atomic) {
    const uint32_t par = word_parity<ODD>(rec);
    for (int j = 0; j < s.n; ++j) {
        const uint32_t *p = rec + field_at<ODD>(s, j, par);
        switch (s.op[j]) {
            case GJ_SUM: {
                const unsigned long long x = *reinterpret_cast<const unsigned long long *>(p);
                unsigned long long *q = static_cast<unsigned long long *>(s.out[j]) + o;
                if (atomic) atomicAdd(q, x);
                else *q = x;
                break;
            }
            case GJ_COUNT: {
                unsigned long long *q = static_cast<unsigned long long *>(s.out[j]) + o;
                if (atomic) atomicAdd(q, (unsigned long long)p[0]);
                else *q = p[0];
                break;
            }
            case GJ_MIN: {
                if (s.w8[j]) {
                    const long long x = *reinterpret_cast<const long long *>(p);
                    long long *q = static_cast<long long *>(s.out[j]) + o;
                    if (atomic) atomicMin(q, x);
                    else *q = x;
                } else {
                    int *q = static_cast<int *>(s.out[j]) + o;
                    if (atomic) atomicMin(q, (int)p[0]);
                    else *q = (int)p[0];
                }
                break;
            }
            default: {
                if (s.w8[j]) {
                    const long long x = *reinterpret_cast<const long long *>(p);
                    long long *q = static_cast<long long *>(s.out[j]) + o;
                    if (atomic) atomicMax(q, x);
                    else *q = x;
                } else {
                    int *q = static_cast<int *>(s.out[j]) + o;
                    if (atomic) atomicMax(q, (int)p[0]);
                    else *q = (int)p[0];
                }
                break;
            }
        }
    }
}

// Values of one row for value columns 0..NV-1 (NV >= the number of columns in
// use), held as V: int when every column is 4 bytes, long long otherwise.
template <int NV, typename V = int>
struct Row {
    V v[NV];
};

template <int NV, typename V = int>
__device__ __forceinline__ Row<NV, V> load_row(const ValSrc &vs, uint32_t row) {
    Row<NV, V> r;
    const uint32_t src = vs.rowid ? (uint32_t)vs.rowid[row] : row;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        if constexpr (sizeof(V) == 4) {
            r.v[c] = c < vs.n ? static_cast<const int32_t *>(vs.col[c])[src] : 0;
        } else {
            r.v[c] = c < vs.n ? (vs.w8[c] ? static_cast<const long long *>(vs.col[c])[src]
                                          : (long long)static_cast<const int32_t *>(vs.col[c])[src])
                              : 0ll;
        }
    }
    return r;
}

// Value of column c (uniform over the wave) of a row held in registers. A
// branch on c == cc would let the optimizer index the row by c, which sends the
// row to scratch memory; masks keep every access at a constant index.
template <int NV, typename V>
__device__ __forceinline__ V pick(const Row<NV, V> &r, int c) {
    V x = 0;
#pragma unroll
    for (int cc = 0; cc < NV; ++cc) x |= r.v[cc] & -(V)(cc == c);
    return x;
}

template <int NV, typename V>
__device__ __forceinline__ void row_add_global_r(const AggSpec &s, const Row<NV, V> &r, uint64_t o) {
    for (int j = 0; j < s.n; ++j) {
        const V x = pick(r, s.col[j]);
        switch (s.op[j]) {
            case GJ_SUM:
                atomicAdd(static_cast<unsigned long long *>(s.out[j]) + o, (unsigned long long)(long long)x);
                break;
            case GJ_COUNT: atomicAdd(static_cast<unsigned long long *>(s.out[j]) + o, 1ull); break;
            case GJ_MIN:
                if (sizeof(V) == 8 && s.w8[j]) atomicMin(static_cast<long long *>(s.out[j]) + o, (long long)x);
                else atomicMin(static_cast<int *>(s.out[j]) + o, (int)x);
                break;
            default:
                if (sizeof(V) == 8 && s.w8[j]) atomicMax(static_cast<long long *>(s.out[j]) + o, (long long)x);
                else atomicMax(static_cast<int *>(s.out[j]) + o, (int)x);
                break;
        }
    }
}

// Spare words after the real records, for lanes whose row adds nothing: lane l
// points its record at spare word 2l, so that no two lanes of one atomic share an
// address. The spare "records" overlap and nothing reads them; with one record's
// worth of words beyond the last lane's start they take kSpareWords + words.
constexpr uint32_t kSpareWords = 2 * kWave;
__device__ __forceinline__ uint32_t spare_off(uint32_t rec_end) { return rec_end + 2u * lane_id(); }

// LDS atomic MIN / MAX on a record field of T (int, or long long for an 8-byte
// column); with `skewed`, a row that cannot change the field (checked against a
// possibly stale read) skips the atomic.
template <typename T, int RB, bool IS_MIN, bool ODD>
__device__ __forceinline__ void rec_minmax(uint32_t *recs, const uint32_t (&off)[RB], int w0, int w1,
                                           const T (&x)[RB], int nact, bool skewed) {
    if (!skewed) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (r < nact) {
                T *p = reinterpret_cast<T *>(recs + off[r] + ((ODD && (off[r] & 1u)) ? w1 : w0));
                if (IS_MIN) atomicMin(p, x[r]);
                else atomicMax(p, x[r]);
            }
        }
        return;
    }
    // skewed keys: a minimum only falls (a maximum only rises), so a row no lower
    // (higher) than what the record holds, even a stale read of it, cannot change
    // it; the frequent groups' extremes settle early and most rows skip the
    // atomic that many lanes of a wave would contend for. Uniform keys skip the
    // read: it would wait behind the atomics issued before it.
    T cur[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (r < nact)
            cur[r] = __atomic_load_n(reinterpret_cast<T *>(recs + off[r] + ((ODD && (off[r] & 1u)) ? w1 : w0)), __ATOMIC_RELAXED);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (r < nact && (IS_MIN ? x[r] < cur[r] : x[r] > cur[r])) {
            T *p = reinterpret_cast<T *>(recs + off[r] + ((ODD && (off[r] & 1u)) ? w1 : w0));
            if (IS_MIN) atomicMin(p, x[r]);
            else atomicMax(p, x[r]);
        }
    }
}

// Accumulate rows 0..nact-1 of RB (values in registers) into LDS records: row r
// goes to the record at word off[r]. nact is uniform over the wave (rows past it
// are empty for every lane), and lanes with nothing to add in an active row point
// at a spare, so the atomics need no divergent branch. The loop runs over the
// aggregates outside the rows: each aggregate's atomics issue back to back, and
// the aggregate list is read once per batch of rows rather than once per row.
template <int NV, int RB, typename V, bool ODD = false>
__device__ __forceinline__ void rec_add_rows(uint32_t *recs, const AggSpec &s, const uint32_t (&off)[RB],
                                             const Row<NV, V> (&rr)[RB], int nact, bool skewed) {
    for (int j = 0; j < s.n; ++j) {
        const int c = s.col[j], w = s.word[j], wo = s.word_odd[j];
        switch (s.op[j]) {
            case GJ_SUM:
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nact)
                        atomicAdd(reinterpret_cast<unsigned long long *>(recs + off[r] + ((ODD && (off[r] & 1u)) ? wo : w)),
                                  (unsigned long long)(long long)pick(rr[r], c));
                break;
            case GJ_COUNT:
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nact) atomicAdd(recs + off[r] + ((ODD && (off[r] & 1u)) ? wo : w), 1u);
                break;
            case GJ_MIN:
            default: {
                const bool is_min = s.op[j] == GJ_MIN;
                if constexpr (sizeof(V) == 8) {
                    if (s.w8[j]) {
                        long long x[RB];
#pragma unroll
                        for (int r = 0; r < RB; ++r) x[r] = pick(rr[r], c);
                        if (is_min) rec_minmax<long long, RB, true, ODD>(recs, off, w, wo, x, nact, skewed);
                        else rec_minmax<long long, RB, false, ODD>(recs, off, w, wo, x, nact, skewed);
                        break;
                    }
                }
                int x[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) x[r] = (int)pick(rr[r], c);
                if (is_min) rec_minmax<int, RB, true, ODD>(recs, off, w, wo, x, nact, skewed);
                else rec_minmax<int, RB, false, ODD>(recs, off, w, wo, x, nact, skewed);
                break;
            }
        }
    }
}

// Rows base + r * stride + (first lane of the wave) for r < RB: how many of them
// start below end, i.e. the rows in which some lane of the wave has a row.
template <int RB>
__device__ __forceinline__ int wave_active_rows(uint32_t base, uint32_t stride, uint32_t end) {
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(base + (threadIdx.x & ~(uint32_t)(kWave - 1)));
    if (w0 >= end) return 0;
    return (int)min((uint32_t)RB, (end - w0 + stride - 1) / stride);
}

// Running aggregate of a set of rows: count, and per value column sum / min / max.
template <int NV, typename V = int>
struct Acc {
    uint32_t cnt;
    long long sum[NV];
    V mn[NV], mx[NV];
};

template <typename V>
__device__ __forceinline__ V v_max() { return sizeof(V) == 4 ? (V)INT32_MAX : (V)INT64_MAX; }
template <typename V>
__device__ __forceinline__ V v_min() { return sizeof(V) == 4 ? (V)INT32_MIN : (V)INT64_MIN; }

template <int NV, typename V>
__device__ __forceinline__ void acc_clear(Acc<NV, V> &x) {
    x.cnt = 0;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        x.sum[c] = 0;
        x.mn[c] = v_max<V>();
        x.mx[c] = v_min<V>();
    }
}
template <int NV, typename V>
__device__ __forceinline__ void acc_merge(Acc<NV, V> &x, const Acc<NV, V> &y) {
    x.cnt += y.cnt;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        x.sum[c] = (long long)((unsigned long long)x.sum[c] + (unsigned long long)y.sum[c]);  // wraps mod 2^64
        x.mn[c] = min(x.mn[c], y.mn[c]);
        x.mx[c] = max(x.mx[c], y.mx[c]);
    }
}
template <int NV, typename V>
__device__ __forceinline__ void acc_row(Acc<NV, V> &x, const Row<NV, V> &r) {
    x.cnt += 1;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        x.sum[c] = (long long)((unsigned long long)x.sum[c] + (unsigned long long)(long long)r.v[c]);
        x.mn[c] = min(x.mn[c], r.v[c]);
        x.mx[c] = max(x.mx[c], r.v[c]);
    }
}
// Acc of the lane `src` (all lanes call).
template <int NV, typename V>
__device__ __forceinline__ Acc<NV, V> acc_shfl(const Acc<NV, V> &x, int src) {
    Acc<NV, V> y;
    y.cnt = __shfl(x.cnt, src, kWave);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        y.sum[c] = __shfl(x.sum[c], src, kWave);
        y.mn[c] = __shfl(x.mn[c], src, kWave);
        y.mx[c] = __shfl(x.mx[c], src, kWave);
    }
    return y;
}
template <int NV, typename V>
__device__ __forceinline__ Acc<NV, V> acc_wave_reduce(Acc<NV, V> x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        Acc<NV, V> y;
        y.cnt = __shfl_xor(x.cnt, d, kWave);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            y.sum[c] = __shfl_xor(x.sum[c], d, kWave);
            y.mn[c] = __shfl_xor(x.mn[c], d, kWave);
            y.mx[c] = __shfl_xor(x.mx[c], d, kWave);
        }
        acc_merge(x, y);
    }
    return x;
}

// Column c of an Acc in registers, selected by masks as pick() does.
template <int NV, typename V>
__device__ __forceinline__ void acc_pick(const Acc<NV, V> &x, int c, long long &sum, V &mn, V &mx) {
    sum = 0;
    mn = 0;
    mx = 0;
#pragma unroll
    for (int cc = 0; cc < NV; ++cc) {
        sum |= x.sum[cc] & -(long long)(cc == c);
        mn |= x.mn[cc] & -(V)(cc == c);
        mx |= x.mx[cc] & -(V)(cc == c);
    }
}

template <int NV, typename V>
__device__ __forceinline__ void acc_flush(const Acc<NV, V> &x, const AggSpec &s, uint64_t o, bool atomic) {
    for (int j = 0; j < s.n; ++j) {
        long long sum;
        V mn, mx;
        acc_pick(x, s.col[j], sum, mn, mx);
        switch (s.op[j]) {
            case GJ_SUM: {
                unsigned long long *q = static_cast<unsigned long long *>(s.out[j]) + o;
                if (atomic) atomicAdd(q, (unsigned long long)sum);
                else *q = (unsigned long long)sum;
                break;
            }
            case GJ_COUNT: {
                unsigned long long *q = static_cast<unsigned long long *>(s.out[j]) + o;
                if (atomic) atomicAdd(q, (unsigned long long)x.cnt);
                else *q = x.cnt;
                break;
            }
            case GJ_MIN: {
                if (sizeof(V) == 8 && s.w8[j]) {
                    long long *q = static_cast<long long *>(s.out[j]) + o;
                    if (atomic) atomicMin(q, (long long)mn);
                    else *q = (long long)mn;
                } else {
                    int *q = static_cast<int *>(s.out[j]) + o;
                    if (atomic) atomicMin(q, narrow_min(mn));
                    else *q = narrow_min(mn);
                }
                break;
            }
            default: {
                if (sizeof(V) == 8 && s.w8[j]) {
                    long long *q = static_cast<long long *>(s.out[j]) + o;
                    if (atomic) atomicMax(q, (long long)mx);
                    else *q = (long long)mx;
                } else {
                    int *q = static_cast<int *>(s.out[j]) + o;
                    if (atomic) atomicMax(q, narrow_max(mx));
                    else *q = narrow_max(mx);
                }
                break;
            }
        }
    }
}

// Fold an Acc into an LDS record (leader lane of a wave-aggregated update).
template <int NV, typename V, bool ODD = false>
__device__ __forceinline__ void rec_add_acc(uint32_t *rec, const AggSpec &s, const Acc<NV, V> &x) {
    const uint32_t par = word_parity<ODD>(rec);
    for (int j = 0; j < s.n; ++j) {
        uint32_t *p = rec + field_at<ODD>(s, j, par);
        long long sum;
        V mn, mx;
        acc_pick(x, s.col[j], sum, mn, mx);
        switch (s.op[j]) {
            case GJ_SUM: atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)sum); break;
            case GJ_COUNT: atomicAdd(p, x.cnt); break;
            case GJ_MIN:
                if (sizeof(V) == 8 && s.w8[j]) atomicMin(reinterpret_cast<long long *>(p), (long long)mn);
                else atomicMin(reinterpret_cast<int *>(p), narrow_min(mn));
                break;
            default:
                if (sizeof(V) == 8 && s.w8[j]) atomicMax(reinterpret_cast<long long *>(p), (long long)mx);
                else atomicMax(reinterpret_cast<int *>(p), narrow_max(mx));
                break;
        }
    }
}

// Rows of one wave round with group ids: lanes sharing an id are combined in
// registers first, so each distinct id costs one set of LDS atomics per wave
// instead of one per lane (the case of few groups, where lanes collide).
template <int NV, typename V, bool ODD = false>
__device__ __forceinline__ void wave_aggregate(uint32_t *recs, const AggSpec &s, bool valid, uint32_t id,
                                               const Row<NV, V> &r) {
    uint64_t todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t lid = __shfl(id, leader, kWave);
        const bool mine = valid && id == lid;
        const uint64_t peers = __ballot(mine);
        Acc<NV, V> x;
        acc_clear(x);
        if (mine) acc_row(x, r);
        x = acc_wave_reduce(x);
        if (lane_id() == leader) rec_add_acc<NV, V, ODD>(recs + (uint64_t)lid * s.words, s, x);
        todo &= ~peers;
    }
}

__device__ __forceinline__ void out_identity(const AggSpec &s, uint64_t i) {
    for (int j = 0; j < s.n; ++j) {
        switch (s.op[j]) {
            case GJ_SUM:
            case GJ_COUNT: static_cast<long long *>(s.out[j])[i] = 0; break;
            case GJ_MIN:
                if (s.w8[j]) static_cast<long long *>(s.out[j])[i] = INT64_MAX;
                else static_cast<int *>(s.out[j])[i] = INT32_MAX;
                break;
            default:
                if (s.w8[j]) static_cast<long long *>(s.out[j])[i] = INT64_MIN;
                else static_cast<int *>(s.out[j])[i] = INT32_MIN;
                break;
        }
    }
}

// Identity values for every output column over groups [0, g).
__global__ void k_out_init(AggSpec s, uint64_t g) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g; i += (uint64_t)gridDim.x * blockDim.x)
        out_identity(s, i);
}

// The same for groups [base, base + min(g, cap)), base and g read on the device.
__global__ void k_out_init_dev(AggSpec s, const uint64_t *__restrict__ base, const uint32_t *__restrict__ g_dev,
                               uint64_t cap) {
    const uint64_t b = base ? *base : 0ull, g = min((uint64_t)*g_dev, cap);
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < g; k += (uint64_t)gridDim.x * blockDim.x)
        out_identity(s, b + k);
}

// Batches: first output group of each instance (partitions are instance * 256 + digit).
__global__ void k_pgb_inst_offsets(const uint32_t *__restrict__ goff, uint32_t nseg,
                                   const uint64_t *__restrict__ base, uint64_t *__restrict__ out) {
    const uint64_t b = base ? *base : 0ull;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nseg; i += gridDim.x * blockDim.x)
        out[i] = b + goff[(uint64_t)i << 8];
}

// Plan bookkeeping: next group base, the overflow flag and the unit count.
__global__ void k_pgb_status(const uint64_t *__restrict__ base, const uint32_t *__restrict__ g_dev,
                             uint64_t *__restrict__ next, const uint32_t *__restrict__ stat,
                             const uint32_t *__restrict__ nunits, uint32_t *__restrict__ status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *next = (base ? *base : 0ull) + *g_dev;
        status[0] = stat[1];
        status[1] = *nunits;
    }
}

template <typename K>
__device__ __forceinline__ K empty_key() {
    if constexpr (sizeof(K) == 4) return (K)INT32_MIN;
    else return (K)INT64_MIN;
}

// Slot hash for LDS tables: the top bits of the MurmurHash3 finalizer. The
// partition digit of the partition-based group-by takes the low bits of the
// same hash, so keys of one partition still spread over the table.
template <typename K>
__device__ __forceinline__ uint32_t slot_hash(K key, int log2cap) {
    uint32_t x;
    if constexpr (sizeof(K) == 4) x = (uint32_t)key;
    else x = (uint32_t)(uint64_t)key ^ (uint32_t)((uint64_t)key >> 32);
    return log2cap == 0 ? 0u : fmix32(x) >> (32 - log2cap);
}

// Insert-or-find in an LDS open-addressing table (linear probing). The key equal
// to the empty marker never reaches here. Returns the slot, or -1 if full.
template <typename K>
__device__ __forceinline__ int lds_insert(K *tab, int log2cap, K key) {
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t h = slot_hash<K>(key, log2cap);
    const K e = empty_key<K>();
    for (uint32_t step = 0; step <= mask; ++step) {
        K cur = tab[h];  // a plain read first: keys already present need no atomic
        if (cur == key) return (int)h;
        if (cur != e) {
            h = (h + 1) & mask;
            continue;
        }
        if constexpr (sizeof(K) == 4) cur = (K)atomicCAS(reinterpret_cast<int *>(&tab[h]), (int)e, (int)key);
        else
            cur = (K)atomicCAS(reinterpret_cast<unsigned long long *>(&tab[h]), (unsigned long long)e,
                               (unsigned long long)key);
        if (cur == e || cur == key) return (int)h;
        h = (h + 1) & mask;
    }
    return -1;
}

template <typename K>
__device__ __forceinline__ int lds_find(const K *tab, int log2cap, K key) {
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t h = slot_hash<K>(key, log2cap);
    for (uint32_t step = 0; step <= mask; ++step) {
        if (tab[h] == key) return (int)h;
        if (tab[h] == empty_key<K>()) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

// ---------------------------------------------------------------------------------
// Group-count estimate before any group-by runs (the count is unknown up front,
// Section 2.2): a HyperLogLog sketch (Flajolet, Fusy, Gandouet, Meunier 2007)
// over the 32-bit MurmurHash3 finalizer of the keys, 2^10 registers. One read of
// the key column; it picks the partition passes and feeds the selector.

constexpr int kHllBits = 10;

// The same read also ORs and ANDs the key bits (bits[0], bits[1]): their xor
// marks the key bytes that vary, i.e. the passes a radix sort of the raw keys
// needs. With hist8, workgroup b reads chunk b (chunk_rows rows) and also
// counts its rows per low 8 bits of the hash, the digit a single partition pass
// of the partition-based group-by takes, so that pass reads no keys for its
// histogram.
// U keys of the sketch read: their hash digits counted, their registers raised,
// their bits ORed and ANDed. A register only grows, so a key whose rank does
// not exceed the value read now cannot change it: the U registers are read
// first and only larger ranks take an atomic (with few distinct keys nearly
// none do, where atomics on one address would serialize a wave).
template <typename K, bool HIST, typename B, int U>
__device__ __forceinline__ void hll_keys(const K (&k)[U], uint32_t valid, uint32_t *s_reg, uint32_t *s_cnt, B &o,
                                         B &x) {
    uint32_t ir[U], cur[U];  // register index | rank << 16
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = (valid >> u) & 1u;
        const uint32_t h = (uint32_t)digit_source<K>(k[u], kDigitHash);
        const uint32_t wv = (h << kHllBits) | (1u << (kHllBits - 1));  // the bits below the index
        ir[u] = (h >> (32 - kHllBits)) | (ok ? ((uint32_t)__clz((int)wv) + 1u) << 16 : 0u);
        if constexpr (HIST) {
            // a wave whose rows all share one digit (few distinct keys) adds once
            const uint32_t d = h & 0xFFu, d0 = __builtin_amdgcn_readfirstlane(d);
            const uint32_t lanes = (uint32_t)__popcll(__ballot(ok));  // taken by the whole wave
            if (__all(ok && d == d0)) {
                if (lane_id() == 0) atomicAdd(&s_cnt[d0], lanes);
            } else if (ok) {
                atomicAdd(&s_cnt[d], 1u);
            }
        }
        if (ok) {
            o |= (B)k[u];
            x &= (B)k[u];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = s_reg[ir[u] & 0xFFFFu];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if ((ir[u] >> 16) > cur[u]) atomicMax(&s_reg[ir[u] & 0xFFFFu], ir[u] >> 16);
}

template <typename K, bool HIST>
__global__ __launch_bounds__(kBlock) void k_hll(const K *__restrict__ keys, uint32_t n, uint32_t *__restrict__ regs,
                                                unsigned long long *__restrict__ bits, uint32_t chunk_rows,
                                                uint32_t *__restrict__ hist8) {
    constexpr int U = sizeof(K) == 4 ? 16 : 8;  // keys per thread and round
    constexpr int V = 16 / (int)sizeof(K);  // keys per 16-byte load
    using B = std::conditional_t<sizeof(K) == 4, uint32_t, unsigned long long>;
    __shared__ uint32_t s_reg[1 << kHllBits];
    __shared__ uint32_t s_cnt[HIST ? kWaves : 1][HIST ? 256 : 1];
    for (int i = threadIdx.x; i < (1 << kHllBits); i += kBlock) s_reg[i] = 0;
    if constexpr (HIST)
        for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    B o = 0, x = ~B(0);
    uint32_t *cnt = &s_cnt[HIST ? threadIdx.x / kWave : 0][0];
    uint32_t lo, hi, stride;
    if constexpr (HIST) {
        lo = blockIdx.x * chunk_rows;
        hi = (uint32_t)min<uint64_t>((uint64_t)lo + chunk_rows, n);
        stride = kBlock * U;
    } else {
        lo = blockIdx.x * kBlock * U;
        hi = n;
        stride = gridDim.x * kBlock * U;
    }
    uint32_t base = lo;
    if ((reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
        // whole rounds: a wave's 16-byte loads cover 1 KB of consecutive keys
        // (rounds start at multiples of kBlock * U rows, so every load is aligned)
        for (; (uint64_t)base + kBlock * U <= hi; base += stride) {
            const uint4 *__restrict__ q = reinterpret_cast<const uint4 *>(keys + base) + threadIdx.x;
            uint4 v[U / V];
#pragma unroll
            for (int j = 0; j < U / V; ++j) v[j] = q[j * kBlock];
            // the keys in two halves keep the register count down
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                K k[U / 2];
#pragma unroll
                for (int e = 0; e < U / 2; ++e)
                    k[e] = reinterpret_cast<const K *>(&v[0])[half * (U / 2) + e];
                hll_keys<K, HIST, B, U / 2>(k, (1u << (U / 2)) - 1u, s_reg, cnt, o, x);
            }
        }
    }
    // the rest (a partial round, or keys that are not 16-byte aligned), row by row
    for (; base < hi; base += stride) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            K k[U / 2];
            uint32_t valid = 0;
#pragma unroll
            for (int u = 0; u < U / 2; ++u) {
                const uint32_t i = base + (half * (U / 2) + u) * kBlock + threadIdx.x;
                k[u] = i < hi ? keys[i] : K(0);
                valid |= (i < hi ? 1u : 0u) << u;
            }
            hll_keys<K, HIST, B, U / 2>(k, valid, s_reg, cnt, o, x);
        }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        o |= __shfl_xor(o, d, kWave);
        x &= __shfl_xor(x, d, kWave);
    }
    if (lane_id() == 0) {
        // 4-byte keys leave the upper word alone (set in the AND, clear in the OR)
        atomicOr(&bits[0], (unsigned long long)o);
        atomicAnd(&bits[1], (unsigned long long)x | (sizeof(K) == 4 ? 0xFFFFFFFF00000000ull : 0ull));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << kHllBits); i += kBlock)
        if (s_reg[i]) atomicMax(&regs[i], s_reg[i]);
    if constexpr (HIST) {
        for (int d = threadIdx.x; d < 256; d += kBlock) {
            uint32_t t = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) t += s_cnt[q][d];
            hist8[(size_t)blockIdx.x * 256u + d] = t;
        }
    }
}

// ---------------------------------------------------------------------------------
// Partition-based group-by (Section 4.3). After partitioning on the hashed key,
// the discover pass inserts every key of a partition into an LDS table before any
// aggregation, which gives the partition's group count and hence dense output
// offsets. Local group ids follow the first occurrence of each key in the
// (stable) partitioned order, so the output order is deterministic.

struct PgbArgs {
    const void *keys;       // partitioned keys
    const uint32_t *poff;   // partition offsets (np + 1)
    uint32_t np;
    void *tmp_keys;         // per partition: its distinct keys in id order, at the partition's row offset
    uint32_t *gcnt;         // groups per partition (np + 1; scanned into offsets later)
    uint32_t *stat;         // [0] = max groups in one partition, [1] = overflow flag
    // aggregation pass
    const uint32_t *goff;   // exclusive prefix of gcnt
    const uint32_t *ubase;  // exclusive prefix of units per partition
    void *out_key;
    AggSpec spec;
    ValSrc vals;
    int log2cap;            // LDS table size of the aggregation pass
    int lds_records;        // 1: aggregate in LDS records; 0: global atomics
    // discovery of oversized partitions by several workgroups
    const uint32_t *dubase; // exclusive prefix of discovery units per partition (np + 1)
    uint32_t *dcount;       // distinct keys found by each discovery unit
    // persistent aggregation (plans): unit count in device memory, output offset
    const uint32_t *nunits; // device: aggregation units
    uint32_t cap_units;     // units beyond this are not processed
    const uint64_t *out_base; // device: first output group of this call (nullptr = 0)
    uint32_t lds_bytes;     // > 0: table size and records chosen per partition within this LDS
    uint32_t g_lo, g_hi;    // plans: only partitions with g_lo <= groups <= g_hi (two launches share them)
};

template <typename K>
__global__ __launch_bounds__(kBlock) void k_pgb_discover(PgbArgs a) {
    __shared__ K s_key[kDiscoverCap];
    __shared__ uint32_t s_first[kDiscoverCap];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_sent;  // first row holding the key equal to the empty marker
    __shared__ int s_over;
    constexpr int log2cap = 12;
    static_assert((1u << log2cap) == kDiscoverCap, "table size");
    const uint32_t p = blockIdx.x;
    const uint32_t p0 = a.poff[p], p1 = a.poff[p + 1];
    const int tid = threadIdx.x;
    if (p0 == p1) {
        if (tid == 0) a.gcnt[p] = 0;
        return;
    }
    if (p1 - p0 > kDiscoverUnit) return;  // discovered by k_pgb_discover_unit + k_pgb_merge
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    const K e = empty_key<K>();
    for (uint32_t i = tid; i < kDiscoverCap; i += kBlock) {
        s_key[i] = e;
        s_first[i] = 0xFFFFFFFFu;
    }
    if (tid == 0) {
        s_sent = 0xFFFFFFFFu;
        s_over = 0;
    }
    __syncthreads();
    constexpr int RB = 16;  // keys loaded per thread before they are inserted
    for (uint32_t base = p0; base < p1; base += kBlock * RB) {
        K kk[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + tid;
            kk[r] = i < p1 ? keys[i] : e;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + tid;
            if (i >= p1) continue;
            const uint32_t local = i - p0;
            if (kk[r] == e) {
                atomicMin(&s_sent, local);
            } else if (!__atomic_load_n(&s_over, __ATOMIC_RELAXED)) {  // once full, stop probing
                const int slot = lds_insert<K>(s_key, log2cap, kk[r]);
                if (slot < 0) s_over = 1;
                else if (s_first[slot] > local) atomicMin(&s_first[slot], local);
            }
        }
    }
    __syncthreads();
    if (s_over) {
        if (tid == 0) {
            a.gcnt[p] = 0;
            atomicOr(&a.stat[1], 1u);
        }
        return;
    }
    // ids in order of first occurrence. Rows are read coalesced: round r of a
    // 4096-row chunk is rows c0 + 256 r + tid, so row order is (round, wave, lane).
    // Every (round, wave) counts its heads by ballot; one barrier later each thread
    // knows how many heads come before its row from those counts and its rank.
    K *__restrict__ tk = static_cast<K *>(a.tmp_keys);
    constexpr int HB = 16;
    __shared__ uint32_t s_rw[HB][kWaves];
    const int w = tid / kWave;
    uint32_t ids = 0;
    for (uint32_t c0 = p0; c0 < p1; c0 += kBlock * HB) {
        K kk[HB];
#pragma unroll
        for (int r = 0; r < HB; ++r) {
            const uint32_t i = c0 + r * kBlock + tid;
            kk[r] = i < p1 ? keys[i] : e;
        }
        uint32_t hmask = 0, rk[HB];
#pragma unroll
        for (int r = 0; r < HB; ++r) {
            const uint32_t i = c0 + r * kBlock + tid;
            bool head = false;
            if (i < p1) {
                const uint32_t local = i - p0;
                head = (kk[r] == e) ? (s_sent == local) : (s_first[lds_find<K>(s_key, log2cap, kk[r])] == local);
            }
            const uint64_t m = __ballot(head);
            rk[r] = rank_below(m);
            if (head) hmask |= 1u << r;
            if (lane_id() == 0) s_rw[r][w] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        uint32_t before = 0, tot = 0;  // heads before (round r, this wave), and in the chunk
#pragma unroll
        for (int r = 0; r < HB; ++r) {
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                const uint32_t c = s_rw[r][q];
                if (q < w) before += c;
                tot += c;
            }
            if (hmask & (1u << r)) tk[p0 + ids + before + rk[r]] = kk[r];
            // the rest of round r (this and later waves) precedes round r + 1
#pragma unroll
            for (int q = 0; q < kWaves; ++q)
                if (q >= w) before += s_rw[r][q];
        }
        ids += tot;
        __syncthreads();  // the counts are rewritten by the next chunk
    }
    if (tid == 0) {
        a.gcnt[p] = ids;
        atomicMax(&a.stat[0], ids);
    }
}

__global__ void k_pgb_dunits(const uint32_t *__restrict__ poff, uint32_t np, uint32_t *__restrict__ du) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
        const uint32_t n = poff[p + 1] - poff[p];
        du[p] = n > kDiscoverUnit ? ceil_div_u32(n, kDiscoverUnit) : 0u;
    }
}

// One slice of an oversized partition: its distinct keys (in table order) are
// written over the slice's own rows of tmp_keys, their number to dcount.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_pgb_discover_unit(PgbArgs a) {
    __shared__ K s_key[kDiscoverCap];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_unit[3];
    __shared__ int s_sent, s_over;
    constexpr int log2cap = 12;
    const int tid = threadIdx.x;
    const uint32_t u = blockIdx.x;
    const uint32_t total = a.dubase[a.np];
    if (u >= total) return;
    if (tid == 0) {
        uint32_t lo = 0, hi = a.np;  // dubase[lo] <= u < dubase[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.dubase[mid] <= u) lo = mid;
            else hi = mid;
        }
        const uint32_t p0 = a.poff[lo], p1 = a.poff[lo + 1];
        const uint32_t j = u - a.dubase[lo];
        s_unit[0] = p0 + j * kDiscoverUnit;
        s_unit[1] = min(p0 + (j + 1) * kDiscoverUnit, p1);
        s_sent = 0;
        s_over = 0;
    }
    const K e = empty_key<K>();
    for (uint32_t i = tid; i < kDiscoverCap; i += kBlock) s_key[i] = e;
    __syncthreads();
    const uint32_t r0 = s_unit[0], r1 = s_unit[1];
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    constexpr int RB = 16;
    for (uint32_t base = r0; base < r1; base += kBlock * RB) {
        K kk[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + tid;
            kk[r] = i < r1 ? keys[i] : e;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (base + r * kBlock + tid >= r1) continue;
            if (kk[r] == e) s_sent = 1;
            else if (!__atomic_load_n(&s_over, __ATOMIC_RELAXED) && lds_insert<K>(s_key, log2cap, kk[r]) < 0)
                s_over = 1;  // once full, the remaining keys are not probed
        }
    }
    __syncthreads();
    if (s_over) {
        if (tid == 0) {
            a.dcount[u] = 0;  // the merge reads every slice's count
            atomicOr(&a.stat[1], 1u);
        }
        return;
    }
    K *__restrict__ tk = static_cast<K *>(a.tmp_keys);
    uint32_t cnt = 0;
    for (uint32_t c0 = 0; c0 < kDiscoverCap; c0 += kBlock) {
        const K k = s_key[c0 + tid];
        const uint32_t f = k != e;
        uint32_t tot;
        const uint32_t pre = block_exclusive_sum<uint32_t>(f, s_tmp, &tot);
        if (f) tk[r0 + cnt + pre] = k;
        cnt += tot;
    }
    if (tid == 0) {
        if (s_sent) tk[r0 + cnt++] = e;
        a.dcount[u] = cnt;
    }
}

// Union of the slices' key lists of an oversized partition, sorted by key (a
// deterministic group order), written to the partition's tmp_keys range.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_pgb_merge(PgbArgs a) {
    __shared__ K s_key[kDiscoverCap];
    __shared__ K s_sort[kDiscoverCap];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ int s_sent, s_over;
    constexpr int log2cap = 12;
    const uint32_t p = blockIdx.x;
    const int tid = threadIdx.x;
    const uint32_t u0 = a.dubase[p], u1 = a.dubase[p + 1];
    if (u0 == u1) return;  // not an oversized partition
    // a slice overflowed (here or in another partition): the result is discarded
    // (hash group-by takes over, or a plan reports the overflow), so nothing is
    // merged; the group count is still defined for the kernels that follow
    if (__atomic_load_n(&a.stat[1], __ATOMIC_RELAXED)) {
        if (tid == 0) a.gcnt[p] = 0;
        return;
    }
    const uint32_t p0 = a.poff[p], p1 = a.poff[p + 1];
    const K e = empty_key<K>();
    for (uint32_t i = tid; i < kDiscoverCap; i += kBlock) s_key[i] = e;
    if (tid == 0) {
        s_sent = 0;
        s_over = 0;
    }
    __syncthreads();
    K *__restrict__ tk = static_cast<K *>(a.tmp_keys);
    for (uint32_t u = u0; u < u1; ++u) {
        // a slice's distinct keys sit over its own rows: never more than the rows
        // of the slice or the slots of its table
        const uint32_t r0 = p0 + (u - u0) * kDiscoverUnit;
        const uint32_t d = min(a.dcount[u], min(kDiscoverCap + 1u, p1 - r0));
        for (uint32_t i = tid; i < d; i += kBlock) {
            const K k = tk[r0 + i];
            if (k == e) s_sent = 1;
            else if (!__atomic_load_n(&s_over, __ATOMIC_RELAXED) && lds_insert<K>(s_key, log2cap, k) < 0)
                s_over = 1;
        }
    }
    __syncthreads();
    if (s_over) {
        if (tid == 0) {
            a.gcnt[p] = 0;
            atomicOr(&a.stat[1], 1u);
        }
        return;
    }
    // compact, pad with the largest key, bitonic sort ascending
    uint32_t cnt = 0;
    for (uint32_t c0 = 0; c0 < kDiscoverCap; c0 += kBlock) {
        const K k = s_key[c0 + tid];
        const uint32_t f = k != e;
        uint32_t tot;
        const uint32_t pre = block_exclusive_sum<uint32_t>(f, s_tmp, &tot);
        if (f) s_sort[cnt + pre] = k;
        cnt += tot;
    }
    uint32_t n2 = 1;
    while (n2 < cnt) n2 <<= 1;
    const K big = sizeof(K) == 4 ? (K)INT32_MAX : (K)INT64_MAX;
    for (uint32_t i = cnt + tid; i < n2; i += kBlock) s_sort[i] = big;
    __syncthreads();
    for (uint32_t k2 = 2; k2 <= n2; k2 <<= 1) {
        for (uint32_t j = k2 >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < n2; i += kBlock) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const K x = s_sort[i], y = s_sort[l];
                    const bool up = (i & k2) == 0;
                    if ((x > y) == up) {
                        s_sort[i] = y;
                        s_sort[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    // the key equal to the empty marker is the smallest key of all
    const uint32_t off = s_sent ? 1u : 0u;
    if (tid == 0 && s_sent) tk[p0] = e;
    for (uint32_t i = tid; i < cnt; i += kBlock) tk[p0 + off + i] = s_sort[i];
    if (tid == 0) {
        a.gcnt[p] = cnt + off;
        atomicMax(&a.stat[0], cnt + off);
    }
}

// Rows per aggregation unit of a partition with g groups: at least 128 rows per
// group (at most 2^20), so that folding a unit's records into the output (g
// atomic updates per aggregate) stays small next to the rows the unit aggregated.
// (256 rows per group left a last round of a few units on a nearly idle GPU at
// 2^16-2^18 groups: 3-5% slower; 64 and 96 measured like 128.)
__device__ __forceinline__ uint32_t unit_rows_for(uint32_t g) {
    const uint32_t r = min(max(kUnitRows, g * 128u), 1u << 20);
    return ceil_div_u32(r, kUnitRows) * kUnitRows;
}

__global__ void k_pgb_units(const uint32_t *__restrict__ poff, const uint32_t *__restrict__ goff, uint32_t np,
                            uint32_t *__restrict__ ucnt, uint32_t *__restrict__ max_units) {
    uint32_t mx = 0;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
        const uint32_t u = ceil_div_u32(poff[p + 1] - poff[p], unit_rows_for(goff[p + 1] - goff[p]));
        ucnt[p] = u;
        mx = max(mx, u);
    }
    atomicMax(max_units, mx);
}

template <typename K, int NV, int BT, bool SKEW, typename V>
__device__ __forceinline__ void pgb_unit(const PgbArgs &a, uint32_t u, uint64_t out_base, uint32_t *s_dyn,
                                         uint32_t *s_unit, uint32_t &s_sent_id) {
    constexpr int RB = NV <= 2 ? 8 : 16 / NV;  // rows loaded per thread before they are aggregated
    const int tid = threadIdx.x, lane = lane_id();
    if (tid == 0) {
        uint32_t lo = 0, hi = a.np;  // ubase[lo] <= u < ubase[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.ubase[mid] <= u) lo = mid;
            else hi = mid;
        }
        const uint32_t p = lo;
        const uint32_t p0 = a.poff[p], p1 = a.poff[p + 1];
        const uint32_t j = u - a.ubase[p];
        const uint32_t ur = unit_rows_for(a.goff[p + 1] - a.goff[p]);
        s_unit[0] = p;
        s_unit[1] = p0 + j * ur;
        s_unit[2] = min(p0 + (j + 1) * ur, p1);
        s_unit[3] = (a.ubase[p + 1] - a.ubase[p]) > 1;  // several units share the partition
        s_unit[4] = j;
        s_sent_id = 0xFFFFFFFFu;
    }
    __syncthreads();
    const uint32_t p = s_unit[0], r0 = s_unit[1], r1 = s_unit[2];
    const bool multi = s_unit[3] != 0;
    const uint32_t j = s_unit[4];
    const uint32_t p0 = a.poff[p];
    const uint32_t g = a.goff[p + 1] - a.goff[p];  // group counts were scanned in place into offsets
    const uint64_t gb = out_base + a.goff[p];
    if (g == 0) return;
    if (a.lds_bytes && (g < a.g_lo || g > a.g_hi)) return;  // the other launch of a plan takes it
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    const K *__restrict__ tk = static_cast<const K *>(a.tmp_keys);
    if (j == 0) {
        K *ok = static_cast<K *>(a.out_key);
        for (uint32_t i = tid; i < g; i += BT) ok[gb + i] = tk[p0 + i];
    }
    const AggSpec &s = a.spec;
    if (g == 1) {
        // one group (case 1): registers, then a block-wide reduction
        Acc<NV, V> x;
        acc_clear(x);
        for (uint32_t base = r0; base < r1; base += BT * RB) {
            Row<NV, V> rr[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t i = base + r * BT + tid;
                if (i < r1) rr[r] = load_row<NV, V>(a.vals, i);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (base + r * BT + tid < r1) acc_row(x, rr[r]);
        }
        x = acc_wave_reduce(x);
        Acc<NV, V> *s_acc = reinterpret_cast<Acc<NV, V> *>(s_dyn);
        if (lane == 0) s_acc[tid / kWave] = x;
        __syncthreads();
        if (tid == 0) {
            Acc<NV, V> t = s_acc[0];
            for (int w = 1; w < (BT / kWave); ++w) acc_merge(t, s_acc[w]);
            acc_flush(t, s, gb, multi);
        }
        return;
    }
    int log2cap = a.log2cap;
    bool lds_records = a.lds_records != 0;
    if (a.lds_bytes) {
        // the table holds at least 1.5 slots per group; records (and the spare
        // words) stay in LDS when they fit beside it. The plan's LDS is fixed, so
        // the table then grows into what is left, up to 4 slots per group: fewer
        // lookups probe past their first slot.
        const auto tab_bytes = [](int l) { return (1u << l) * agg_slot_bytes(sizeof(K)) + 8u; };
        const uint32_t rec = ((g + 1) * (uint32_t)a.spec.words + kSpareWords) * 4u;
        log2cap = agg_table_log2(g);
        lds_records = tab_bytes(log2cap) + rec <= a.lds_bytes;
        const uint32_t keys = max(min(g, kDiscoverCap), 16u), need = lds_records ? rec : 0u;
        while ((2u << log2cap) <= 4u * keys && tab_bytes(log2cap + 1) + need <= a.lds_bytes) ++log2cap;
    }
    const uint32_t cap = 1u << log2cap;
    K *tab = reinterpret_cast<K *>(s_dyn);                      // 8-byte keys
    uint16_t *id_of = reinterpret_cast<uint16_t *>(tab + cap);  // 8-byte keys: slot -> group id
    unsigned long long *tab64 = reinterpret_cast<unsigned long long *>(s_dyn);  // 4-byte keys: id << 32 | key
    const K e = empty_key<K>();
    const unsigned long long e64 = (0xFFFFFFFFull << 32) | (uint32_t)e;
    // records from the first 8-byte boundary after the table; an index into s_dyn
    // (not integer pointer arithmetic) keeps them addressed as LDS, so the record
    // updates compile to LDS atomics rather than flat ones
    uint32_t *recs = s_dyn + ((cap * agg_slot_bytes(sizeof(K)) + 7u) & ~7u) / 4u;
    if constexpr (sizeof(K) == 4) {
        for (uint32_t i = tid; i < cap; i += BT) tab64[i] = e64;
    } else {
        for (uint32_t i = tid; i < cap; i += BT) tab[i] = e;
    }
    if (lds_records)
        for (uint32_t i = tid; i < g; i += BT) rec_init(recs + (uint64_t)i * s.words, s);
    __syncthreads();
    for (uint32_t i = tid; i < g; i += BT) {
        const K k = tk[p0 + i];
        if (k == e) {
            s_sent_id = i;
        } else if constexpr (sizeof(K) == 4) {
            // the partition's keys are distinct: the first empty slot of the probe takes it
            uint32_t h = slot_hash<K>(k, log2cap);
            for (uint32_t step = 0; step < cap; ++step) {
                if (atomicCAS(&tab64[h], e64, ((unsigned long long)i << 32) | (uint32_t)k) == e64) break;
                h = (h + 1) & (cap - 1);
            }
        } else {
            const int slot = lds_insert<K>(tab, log2cap, k);
            id_of[slot] = (uint16_t)i;
        }
    }
    __syncthreads();
    // case 2 (records in LDS) or case 3 (global atomics); few groups per
    // partition means colliding lanes, which are combined per wave first
    const bool few = g <= 2;
    for (uint32_t base = r0; base < r1; base += BT * RB) {
        K kk[RB];
        Row<NV, V> rr[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * BT + tid;
            kk[r] = i < r1 ? keys[i] : e;
            if (i < r1) rr[r] = load_row<NV, V>(a.vals, i);
        }
        // group ids: every row's first probe is read before any is resolved (the
        // table is at most half full, so most rows stop there)
        bool ok[RB];
        uint32_t hs[RB], ids[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ok[r] = base + r * BT + tid < r1;
            hs[r] = slot_hash<K>(kk[r], log2cap);
        }
        if constexpr (sizeof(K) == 4) {
            unsigned long long v[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) v[r] = tab64[hs[r]];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (ok[r] && kk[r] != e && (uint32_t)v[r] != (uint32_t)kk[r]) {
                    // the key is in the table: probe on until it turns up
                    uint32_t h = hs[r];
                    for (uint32_t step = 1; step < cap; ++step) {
                        h = (h + 1) & (cap - 1);
                        v[r] = tab64[h];
                        if ((uint32_t)v[r] == (uint32_t)kk[r]) break;
                    }
                }
                ids[r] = ok[r] && kk[r] != e ? (uint32_t)(v[r] >> 32) : 0u;
            }
        } else {
            K t0[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) t0[r] = tab[hs[r]];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (ok[r] && kk[r] != e && t0[r] != kk[r]) hs[r] = (uint32_t)lds_find<K>(tab, log2cap, kk[r]);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) ids[r] = ok[r] && kk[r] != e ? (uint32_t)id_of[hs[r]] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (ok[r] && kk[r] == e) ids[r] = s_sent_id;
        if (lds_records && !few) {
            uint32_t off[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) off[r] = ok[r] ? ids[r] * (uint32_t)s.words : spare_off(g * s.words);
            rec_add_rows<NV, RB>(recs, s, off, rr, wave_active_rows<RB>(base, BT, r1), SKEW);
        } else {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (lds_records) wave_aggregate<NV>(recs, s, ok[r], ids[r], rr[r]);
                else if (ok[r]) row_add_global_r<NV>(s, rr[r], gb + ids[r]);
            }
        }
    }
    if (lds_records) {
        __syncthreads();
        for (uint32_t i = tid; i < g; i += BT) rec_flush(recs + (uint64_t)i * s.words, s, gb + i, multi);
    }
}

// BT threads per workgroup: 256, or 1024 when a partition's table and records
// take so much LDS that only one or two workgroups fit a compute unit (many
// groups per partition), so that the unit still runs 16 or more waves.
template <typename K, int NV, int BT = kBlock, bool SKEW = false, typename V = int>
__global__ __launch_bounds__(BT) void k_pgb_aggregate(PgbArgs a) {
    extern __shared__ __align__(16) uint32_t s_dyn[];
    __shared__ uint32_t s_unit[5];
    __shared__ uint32_t s_sent_id;
    const uint32_t n_units = min(*a.nunits, a.cap_units);
    const uint64_t out_base = a.out_base ? *a.out_base : 0ull;
    // persistent: a workgroup takes units blockIdx.x, blockIdx.x + gridDim.x, ...
    for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        pgb_unit<K, NV, BT, SKEW, V>(a, u, out_base, s_dyn, s_unit, s_sent_id);
        __syncthreads();  // the unit's LDS state is rebuilt by the next one
    }
}

template <typename K, int NV, typename V = int>
void launch_pgb_aggregate(bool wide, bool skewed, uint32_t units, size_t lds, hipStream_t st, const PgbArgs &a,
                          double bytes) {
    if constexpr (NV <= 2) {
        if (wide) {
            if (skewed)
                GJ_LAUNCH("k_pgb_aggregate", bytes, (k_pgb_aggregate<K, NV, 1024, true, V>), dim3(units), dim3(1024),
                          lds, st, a);
            else
                GJ_LAUNCH("k_pgb_aggregate", bytes, (k_pgb_aggregate<K, NV, 1024, false, V>), dim3(units), dim3(1024),
                          lds, st, a);
            return;
        }
    }
    (void)wide;
    if (skewed)
        GJ_LAUNCH("k_pgb_aggregate", bytes, (k_pgb_aggregate<K, NV, kBlock, true, V>), dim3(units), dim3(kBlock), lds,
                  st, a);
    else
        GJ_LAUNCH("k_pgb_aggregate", bytes, (k_pgb_aggregate<K, NV, kBlock, false, V>), dim3(units), dim3(kBlock), lds,
                  st, a);
}

// ---------------------------------------------------------------------------------
// Hash-based group-by (Algorithm 1). Stage 1 inserts (key, row) into a global
// open-addressing table; the inserting row takes the next dense group id from an
// atomic counter and every row records the row its key was inserted with. Stage 2
// aggregates into a dense buffer: LDS records when all groups fit, else global.

struct HgbArgs {
    const void *keys;
    uint32_t n;
    void *table;          // 4-byte keys: packed (key << 32 | row); 8-byte keys: row index
    int log2cap;
    uint32_t max_probe;   // slots a row probes before it flags the table as too small
    uint32_t *gid;        // group id of inserting rows
    uint32_t *gid_loc;    // row with which the key was inserted
    uint32_t *ngroups;    // [0] groups so far, [1] set when a row found no slot
    void *tmp_keys;       // key of each group id
    // stage 2
    AggSpec spec;
    ValSrc vals;
    void *out_key;
    uint32_t g;
    uint32_t lds_groups;  // groups 0..lds_groups-1 aggregate in LDS records, the rest with global atomics
    // sliced stage 2 (every group in LDS): consecutive id ranges of slice_groups
    // groups, rows cut into `chunks` chunks of chunk_rows rows; gid_row: every
    // row's group id (resolved once when several slices read it), else nullptr
    uint32_t slices, slice_groups, chunks, chunk_rows;
    const uint32_t *gid_row;
};

// Workgroups are dispatched to the 8 XCDs of the chip round robin by index.
constexpr uint32_t kXcds = 8;
// Most id slices of the sliced hash aggregation: every slice re-reads the rows'
// group ids (mostly from L2), so beyond this the global-atomic stage 2 is used.
constexpr uint32_t kHgbMaxSlices = 64;

// Every row's group id, gid[gid_loc[i]], for the slices to stream.
__global__ void k_hgb_resolve(const uint32_t *__restrict__ gid_loc, const uint32_t *__restrict__ gid, uint32_t n,
                              uint32_t *__restrict__ out) {
    constexpr int RB = 16;
    for (uint32_t base = blockIdx.x * kBlock * RB; base < n; base += gridDim.x * kBlock * RB) {
        uint32_t loc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            loc[r] = i < n ? gid_loc[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            if (i < n) out[i] = gid[loc[r]];
        }
    }
}

template <typename K>
__device__ __forceinline__ uint64_t global_slot_hash(K key) {
    uint64_t u = (uint64_t)key;
    if constexpr (sizeof(K) == 4) u &= 0xFFFFFFFFull;
    // splitmix64 output function (Steele, Lea, Flood 2014)
    u += 0x9E3779B97F4A7C15ull;
    u = (u ^ (u >> 30)) * 0xBF58476D1CE4E5B9ull;
    u = (u ^ (u >> 27)) * 0x94D049BB133111EBull;
    return u ^ (u >> 31);
}

// Inserts row i (key k) from slot h on and returns the row whose insert holds
// the key (gid_loc); STORE also writes it to gid_loc[i] where it is found (in
// the row-by-row kernel, one store after the probe loop instead measured twice
// as slow from 2^24 groups up). The first row to claim a slot for its key takes
// the next group id.
template <typename K, bool STORE>
__device__ __forceinline__ uint32_t hgb_insert_from(const HgbArgs &a, const K *keys, uint32_t i, K k, uint64_t h) {
    const uint64_t mask = (1ull << a.log2cap) - 1ull;
    for (uint64_t step = 0; step <= mask && step < a.max_probe; ++step) {
        if constexpr (sizeof(K) == 4) {
            unsigned long long *t = static_cast<unsigned long long *>(a.table);
            // A filled slot never changes again, so a plain (cacheable) read that
            // shows a key is final; only an empty read may be stale, and the CAS
            // below settles it.
            unsigned long long cur = t[h];
            if (cur == ~0ull) {
                const unsigned long long mine = ((unsigned long long)(uint32_t)k << 32) | i;
                cur = atomicCAS(&t[h], ~0ull, mine);
                if (cur == ~0ull) {
                    const uint32_t g = atomicAdd(a.ngroups, 1u);
                    a.gid[i] = g;
                    static_cast<K *>(a.tmp_keys)[g] = k;
                    if constexpr (STORE) a.gid_loc[i] = i;
                    return i;
                }
            }
            if ((uint32_t)(cur >> 32) == (uint32_t)k) {
                if constexpr (STORE) a.gid_loc[i] = (uint32_t)cur;
                return (uint32_t)cur;
            }
        } else {
            uint32_t *t = static_cast<uint32_t *>(a.table);
            uint32_t cur = t[h];  // as above: only an empty read may be stale
            if (cur == 0xFFFFFFFFu) {
                cur = atomicCAS(&t[h], 0xFFFFFFFFu, i);
                if (cur == 0xFFFFFFFFu) {
                    const uint32_t g = atomicAdd(a.ngroups, 1u);
                    a.gid[i] = g;
                    static_cast<K *>(a.tmp_keys)[g] = k;
                    if constexpr (STORE) a.gid_loc[i] = i;
                    return i;
                }
            }
            if (keys[cur] == k) {
                if constexpr (STORE) a.gid_loc[i] = cur;
                return cur;
            }
        }
        h = (h + 1) & mask;
    }
    atomicOr(&a.ngroups[1], 1u);  // no slot within the probe limit: the table is too small
    return i;
}

// Algorithm 1, stage 1: every row in turn probes the global table from its
// home slot. (Reading a round's home slots together first was faster with a
// few dozen groups but 10-20% slower from 2^14 groups up; the cached kernel
// below serves the small counts.)
template <typename K>
__global__ __launch_bounds__(kBlock) void k_hgb_insert(HgbArgs a) {
    constexpr int RB = 16;
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    const uint64_t mask = (1ull << a.log2cap) - 1ull;
    const uint32_t stride = gridDim.x * kBlock * RB;
    for (uint32_t base = blockIdx.x * kBlock * RB; base < a.n; base += stride) {
        K kk[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            kk[r] = i < a.n ? keys[i] : K(0);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            if (i < a.n) hgb_insert_from<K, true>(a, keys, i, kk[r], global_slot_hash<K>(kk[r]) & mask);
        }
    }
}

// Stage 1 for 4-byte keys and a few thousand groups: each workgroup keeps the
// keys it has resolved, with their gid_loc, in an LDS table (Fibonacci hashing,
// linear probing over at most kCacheProbe slots), so that a row whose key the
// workgroup has met before never touches the global table. Rows the cache does
// not hold go to the global table exactly as in k_hgb_insert and are then
// entered in the cache; the cache only remembers what the global table
// answered, so the ids are the same. Entries are key << 32 | gid_loc
// (gid_loc < 2^31, so no entry equals the empty ~0). Whole rounds move keys and
// gid_loc as 16-byte runs of 4 rows (both arrays 16-byte aligned).
constexpr int kInsBlock = 1024;
constexpr int kInsRows = 8;  // rows per thread and round
constexpr int kCacheProbe = 8;

template <int LOG2C>
__device__ __forceinline__ uint32_t cache_home(int32_t k) {
    return ((uint32_t)k * 0x9E3779B1u) >> (32 - LOG2C);
}

template <int LOG2C, int RB>
__device__ __forceinline__ void insert_cached_rows(const HgbArgs &a, unsigned long long *s_c, const int32_t (&kk)[RB],
                                                   const uint32_t (&row)[RB], uint32_t valid, uint32_t (&loc)[RB]) {
    constexpr uint32_t CM = (1u << LOG2C) - 1u;
    uint32_t ch[RB];
    uint32_t open = valid;  // bit r: row r still looks for its key in the cache
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        ch[r] = cache_home<LOG2C>(kk[r]);
        loc[r] = 0xFFFFFFFFu;
    }
    for (int p = 0; p < kCacheProbe && open; ++p) {
        unsigned long long e[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) e[r] = ((open >> r) & 1u) ? s_c[(ch[r] + p) & CM] : 0ull;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (!((open >> r) & 1u)) continue;
            if (e[r] == ~0ull) {
                open &= ~(1u << r);  // an empty slot: the key is not cached
            } else if ((uint32_t)(e[r] >> 32) == (uint32_t)kk[r]) {
                loc[r] = (uint32_t)e[r];
                open &= ~(1u << r);
            }
        }
    }
    uint32_t miss = 0;
#pragma unroll
    for (int r = 0; r < RB; ++r) miss |= (((valid >> r) & 1u) && loc[r] == 0xFFFFFFFFu ? 1u : 0u) << r;
    if (!miss) return;
    // misses (a workgroup's first rows of each key) one at a time
    const int32_t *keys = static_cast<const int32_t *>(a.keys);
    const uint64_t mask = (1ull << a.log2cap) - 1ull;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (!((miss >> r) & 1u)) continue;
        loc[r] = hgb_insert_from<int32_t, false>(a, keys, row[r], kk[r], global_slot_hash<int32_t>(kk[r]) & mask);
        const unsigned long long ent = ((unsigned long long)(uint32_t)kk[r] << 32) | loc[r];
        for (int p = 0; p < kCacheProbe; ++p) {
            const unsigned long long old = atomicCAS(&s_c[(ch[r] + p) & CM], ~0ull, ent);
            if (old == ~0ull || (uint32_t)(old >> 32) == (uint32_t)kk[r]) break;
        }
    }
}

template <int LOG2C>
__global__ __launch_bounds__(kInsBlock, 8) void k_hgb_insert_cached(HgbArgs a) {
    constexpr int RB = kInsRows;
    constexpr uint32_t kRound = (uint32_t)kInsBlock * RB;
    __shared__ unsigned long long s_c[1u << LOG2C];
    for (uint32_t j = threadIdx.x; j < (1u << LOG2C); j += kInsBlock) s_c[j] = ~0ull;
    __syncthreads();
    const int32_t *__restrict__ keys = static_cast<const int32_t *>(a.keys);
    const uint32_t stride = gridDim.x * kRound;
    uint32_t base = blockIdx.x * kRound;
    for (; (uint64_t)base + kRound <= a.n; base += stride) {
        // thread t: rows base + (j * kInsBlock + t) * 4 .. + 3, j < RB / 4
        int32_t kk[RB];
        uint32_t row[RB], loc[RB];
#pragma unroll
        for (int j = 0; j < RB / 4; ++j) {
            const uint32_t r0 = base + (uint32_t)(j * kInsBlock + threadIdx.x) * 4u;
            const int4 v = *reinterpret_cast<const int4 *>(keys + r0);
            kk[4 * j] = v.x;
            kk[4 * j + 1] = v.y;
            kk[4 * j + 2] = v.z;
            kk[4 * j + 3] = v.w;
#pragma unroll
            for (int e = 0; e < 4; ++e) row[4 * j + e] = r0 + e;
        }
        insert_cached_rows<LOG2C, RB>(a, s_c, kk, row, (1u << RB) - 1u, loc);
#pragma unroll
        for (int j = 0; j < RB / 4; ++j)
            *reinterpret_cast<uint4 *>(a.gid_loc + row[4 * j]) =
                make_uint4(loc[4 * j], loc[4 * j + 1], loc[4 * j + 2], loc[4 * j + 3]);
    }
    // the last, partial round of this workgroup (if any), row by row
    if (base < a.n) {
        int32_t kk[RB];
        uint32_t row[RB], loc[RB];
        uint32_t valid = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            row[r] = base + (uint32_t)r * kInsBlock + threadIdx.x;
            kk[r] = row[r] < a.n ? keys[row[r]] : 0;
            valid |= (row[r] < a.n ? 1u : 0u) << r;
        }
        insert_cached_rows<LOG2C, RB>(a, s_c, kk, row, valid, loc);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (row[r] < a.n) a.gid_loc[row[r]] = loc[r];
    }
}

// Stage 2 for at most G groups: every thread folds its rows into one
// accumulator per group in registers, and only at the end do the waves reduce
// them into the workgroup's LDS records, which are then folded into the output.
// (LDS records updated per row would have every lane of a wave contend for the
// same few addresses.)
// The same for 8-byte keys, whose entries do not fit one 64-bit word: a key
// array and a gid_loc array. A slot is claimed by a 64-bit CAS of its key from
// the sentinel kCacheNoKey (rows with that key bypass the cache), and its
// gid_loc, written once afterwards, reads as empty until then: a reader that
// sees the key before its gid_loc treats the row as a miss. So a gid_loc read
// in a slot always belongs to the key there.
constexpr long long kCacheNoKey = (long long)0x8000000000000001ull;
constexpr int kInsRows8 = 4;  // rows per thread and round, 8-byte keys

template <int LOG2C>
__device__ __forceinline__ uint32_t cache_home8(long long k) {
    const uint64_t u = (uint64_t)k;
    return ((uint32_t)(u ^ (u >> 32)) * 0x9E3779B1u) >> (32 - LOG2C);
}

template <int LOG2C, int RB>
__device__ __forceinline__ void insert_cached_rows8(const HgbArgs &a, long long *s_k, uint32_t *s_l,
                                                    const long long (&kk)[RB], const uint32_t (&row)[RB],
                                                    uint32_t valid, uint32_t (&loc)[RB]) {
    constexpr uint32_t CM = (1u << LOG2C) - 1u;
    uint32_t ch[RB];
    uint32_t open = 0;  // bit r: row r still looks for its key in the cache
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        ch[r] = cache_home8<LOG2C>(kk[r]);
        loc[r] = 0xFFFFFFFFu;
        open |= (((valid >> r) & 1u) && kk[r] != kCacheNoKey ? 1u : 0u) << r;
    }
    for (int p = 0; p < kCacheProbe && open; ++p) {
        long long e[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) e[r] = ((open >> r) & 1u) ? s_k[(ch[r] + p) & CM] : kCacheNoKey;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (!((open >> r) & 1u)) continue;
            if (e[r] == kCacheNoKey) {
                open &= ~(1u << r);  // an empty slot: the key is not cached
            } else if (e[r] == kk[r]) {
                loc[r] = s_l[(ch[r] + p) & CM];  // still empty while its writer is between the two stores
                open &= ~(1u << r);
            }
        }
    }
    uint32_t miss = 0;
#pragma unroll
    for (int r = 0; r < RB; ++r) miss |= (((valid >> r) & 1u) && loc[r] == 0xFFFFFFFFu ? 1u : 0u) << r;
    if (!miss) return;
    const long long *keys = static_cast<const long long *>(a.keys);
    const uint64_t mask = (1ull << a.log2cap) - 1ull;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (!((miss >> r) & 1u)) continue;
        loc[r] = hgb_insert_from<long long, false>(a, keys, row[r], kk[r], global_slot_hash<long long>(kk[r]) & mask);
        if (kk[r] == kCacheNoKey) continue;
        for (int p = 0; p < kCacheProbe; ++p) {
            const uint32_t slot = (ch[r] + p) & CM;
            const long long old = (long long)atomicCAS(reinterpret_cast<unsigned long long *>(&s_k[slot]),
                                                       (unsigned long long)kCacheNoKey, (unsigned long long)kk[r]);
            if (old == kCacheNoKey) s_l[slot] = loc[r];
            if (old == kCacheNoKey || old == kk[r]) break;
        }
    }
}

template <int LOG2C>
__global__ __launch_bounds__(kInsBlock, 8) void k_hgb_insert_cached8(HgbArgs a) {
    constexpr int RB = kInsRows8;
    constexpr uint32_t kRound = (uint32_t)kInsBlock * RB;
    __shared__ long long s_k[1u << LOG2C];
    __shared__ uint32_t s_l[1u << LOG2C];
    for (uint32_t j = threadIdx.x; j < (1u << LOG2C); j += kInsBlock) {
        s_k[j] = kCacheNoKey;
        s_l[j] = 0xFFFFFFFFu;
    }
    __syncthreads();
    const long long *__restrict__ keys = static_cast<const long long *>(a.keys);
    const uint32_t stride = gridDim.x * kRound;
    uint32_t base = blockIdx.x * kRound;
    for (; (uint64_t)base + kRound <= a.n; base += stride) {
        // thread t: rows base + t * 4 .. + 3 (two 16-byte loads, one 16-byte store)
        long long kk[RB];
        uint32_t row[RB], loc[RB];
        const uint32_t r0 = base + (uint32_t)threadIdx.x * 4u;
        const longlong2 v0 = *reinterpret_cast<const longlong2 *>(keys + r0);
        const longlong2 v1 = *reinterpret_cast<const longlong2 *>(keys + r0 + 2);
        kk[0] = v0.x;
        kk[1] = v0.y;
        kk[2] = v1.x;
        kk[3] = v1.y;
#pragma unroll
        for (int e = 0; e < RB; ++e) row[e] = r0 + e;
        insert_cached_rows8<LOG2C, RB>(a, s_k, s_l, kk, row, (1u << RB) - 1u, loc);
        *reinterpret_cast<uint4 *>(a.gid_loc + r0) = make_uint4(loc[0], loc[1], loc[2], loc[3]);
    }
    // the last, partial round of this workgroup (if any), row by row
    if (base < a.n) {
        long long kk[RB];
        uint32_t row[RB], loc[RB];
        uint32_t valid = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            row[r] = base + (uint32_t)r * kInsBlock + threadIdx.x;
            kk[r] = row[r] < a.n ? keys[row[r]] : 0;
            valid |= (row[r] < a.n ? 1u : 0u) << r;
        }
        insert_cached_rows8<LOG2C, RB>(a, s_k, s_l, kk, row, valid, loc);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (row[r] < a.n) a.gid_loc[row[r]] = loc[r];
    }
}

template <int NV, typename V, int G>
__global__ __launch_bounds__(kBlock) void k_hgb_aggregate_few(HgbArgs a) {
    constexpr int RB = NV <= 2 ? 8 : 16 / NV;
    extern __shared__ __align__(16) uint32_t s_dyn[];
    const AggSpec &s = a.spec;
    for (uint32_t i = threadIdx.x; i < a.g; i += kBlock) rec_init(s_dyn + (uint64_t)i * s.words, s);
    __syncthreads();
    Acc<NV, V> acc[G];
#pragma unroll
    for (int q = 0; q < G; ++q) acc_clear(acc[q]);
    const uint32_t stride = gridDim.x * kBlock * RB;
    for (uint32_t base = blockIdx.x * kBlock * RB; base < a.n; base += stride) {
        uint32_t loc[RB], gid[RB];
        Row<NV, V> rr[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            loc[r] = i < a.n ? a.gid_loc[i] : 0u;
            if (i < a.n) rr[r] = load_row<NV, V>(a.vals, i);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) gid[r] = base + r * kBlock + threadIdx.x < a.n ? a.gid[loc[r]] : (uint32_t)G;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (gid[r] == (uint32_t)q) acc_row(acc[q], rr[r]);
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
        if ((uint32_t)q < a.g) {
            const Acc<NV, V> x = acc_wave_reduce(acc[q]);
            if (lane_id() == 0) rec_add_acc<NV, V>(s_dyn + (uint64_t)q * s.words, s, x);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < a.g; i += kBlock) rec_flush(s_dyn + (uint64_t)i * s.words, s, i, true);
}

template <int NV, typename V = int>
__global__ __launch_bounds__(kBlock) void k_hgb_aggregate(HgbArgs a) {
    constexpr int RB = NV <= 2 ? 8 : 16 / NV;
    extern __shared__ __align__(16) uint32_t s_dyn[];
    const AggSpec &s = a.spec;
    const uint32_t L = a.lds_groups;
    if (L) {
        for (uint32_t i = threadIdx.x; i < L; i += kBlock) rec_init(s_dyn + (uint64_t)i * s.words, s);
        __syncthreads();
    }
    const uint32_t stride = gridDim.x * kBlock * RB;
    for (uint32_t base = blockIdx.x * kBlock * RB; base < a.n; base += stride) {
        uint32_t loc[RB], gid[RB];
        Row<NV, V> rr[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            loc[r] = i < a.n ? a.gid_loc[i] : 0u;
            if (i < a.n) rr[r] = load_row<NV, V>(a.vals, i);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) gid[r] = a.gid[loc[r]];
        uint32_t off[RB];  // rows that do not use LDS point at the spare words
        bool any = false;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool in_lds = base + r * kBlock + threadIdx.x < a.n && gid[r] < L;
            off[r] = in_lds ? gid[r] * (uint32_t)s.words : spare_off(L * s.words);
            any |= in_lds;
        }
        if (__any(any)) rec_add_rows<NV, RB>(s_dyn, s, off, rr, wave_active_rows<RB>(base, kBlock, a.n), false);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (base + r * kBlock + threadIdx.x < a.n && gid[r] >= L) row_add_global_r<NV>(s, rr[r], gid[r]);
    }
    if (L) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < L; i += kBlock) rec_flush(s_dyn + (uint64_t)i * s.words, s, i, true);
    }
}

// Stage 2 with every group's record in LDS (is_smem_enough once the groups are
// cut into id ranges): workgroup (chunk, slice) aggregates the rows of its chunk
// whose group id falls in its slice of at most slice_groups consecutive ids, then
// folds its records into the output with global atomics. All slices of a chunk
// run on one XCD, so the chunk's group ids come from HBM once and from that
// XCD's L2 for the other slices; value columns are read only for rows in the
// slice.
//
// With several slices only about one row in `slices` belongs to a workgroup, so
// a wave first queues its slice's rows in LDS (ballot + rank, a ring of 128
// entries per wave) and updates records 64 queued rows at a time: every lane of
// every record atomic then carries a row, where updating in place would spend a
// full wave of atomics on a handful of rows. A queue entry is the record offset
// and the row's values when they fit two words, else the row index (its values
// are read when the entry is taken).
template <int NV, typename V>
struct HgbQueue {
    static constexpr bool kVals = NV * sizeof(V) <= 8;      // values kept in the entry
    static constexpr uint32_t kWords = kVals ? 1 + NV * sizeof(V) / 4 : 2;  // per entry
    static constexpr uint32_t kEntries = 2 * kWave;         // ring size per wave
};

__host__ __device__ constexpr uint32_t hgb_queue_bytes(int nv_tier, int value_bytes, uint32_t threads) {
    return (nv_tier * value_bytes <= 8 ? 1u + (uint32_t)(nv_tier * value_bytes) / 4u : 2u) * 4u *
           (2u * kWave) * (threads / kWave);
}

template <int NV, int BT, typename V, bool ODD>
__device__ __forceinline__ void hgb_queue_take(const HgbArgs &a, uint32_t *recs, const uint32_t *q, uint32_t head,
                                               uint32_t cnt, uint32_t spare) {
    using Q = HgbQueue<NV, V>;
    const uint32_t lane = lane_id();
    const uint32_t e = (head + lane) & (Q::kEntries - 1);
    const bool on = lane < cnt;
    uint32_t off[1];
    Row<NV, V> rr[1];
    off[0] = on ? q[e] : spare;
    if constexpr (Q::kVals) {
        const V *qv = reinterpret_cast<const V *>(q + Q::kEntries);
#pragma unroll
        for (int c = 0; c < NV; ++c) rr[0].v[c] = on ? qv[(uint32_t)c * Q::kEntries + e] : V(0);
    } else {
        rr[0] = on ? load_row<NV, V>(a.vals, q[Q::kEntries + e]) : Row<NV, V>{};
    }
    rec_add_rows<NV, 1, V, ODD>(recs, a.spec, off, rr, 1, false);
}

template <int NV, int BT, typename V, bool ODD>
__global__ __launch_bounds__(BT) void k_hgb_aggregate_sliced(HgbArgs a) {
    constexpr int RB = NV <= 2 ? 8 : 16 / NV;
    using Q = HgbQueue<NV, V>;
    extern __shared__ __align__(16) uint32_t s_dyn[];
    const AggSpec &s = a.spec;
    const uint32_t b = blockIdx.x, qi = b / kXcds;
    const uint32_t slice = qi % a.slices, chunk = (qi / a.slices) * kXcds + b % kXcds;
    if (chunk >= a.chunks) return;
    const uint32_t g0 = slice * a.slice_groups;
    if (g0 >= a.g) return;
    const uint32_t L = min(a.slice_groups, a.g - g0);
    for (uint32_t i = threadIdx.x; i < L; i += BT) rec_init<ODD>(s_dyn + (uint64_t)i * s.words, s);
    __syncthreads();
    const uint32_t row0 = chunk * a.chunk_rows;
    const uint32_t row1 = (uint32_t)min<uint64_t>((uint64_t)row0 + a.chunk_rows, a.n);
    const uint32_t spare = spare_off(L * s.words);
    if (!a.gid_row) {
        // one slice: every row of the chunk updates a record in place
        for (uint32_t base = row0; base < row1; base += BT * RB) {
            uint32_t id[RB], off[RB];
            Row<NV, V> rr[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t i = base + r * BT + threadIdx.x;
                id[r] = i < row1 ? a.gid_loc[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) id[r] = a.gid[id[r]];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t i = base + r * BT + threadIdx.x;
                const bool in = i < row1 && id[r] - g0 < L;
                off[r] = in ? (id[r] - g0) * (uint32_t)s.words : spare;
                rr[r] = in ? load_row<NV, V>(a.vals, i) : Row<NV, V>{};
            }
            rec_add_rows<NV, RB, V, ODD>(s_dyn, s, off, rr, wave_active_rows<RB>(base, BT, row1), false);
        }
    } else {
        // queue of this wave, after the records and their spare words
        const uint32_t rec_words = ((L + 1) * s.words + kSpareWords + 3u) & ~3u;
        uint32_t *q = s_dyn + rec_words + (threadIdx.x / kWave) * (Q::kWords * Q::kEntries);
        const uint32_t lane = lane_id();
        uint32_t head = 0, cnt = 0;  // wave-uniform: first queued entry, entries queued
        for (uint32_t base = row0; base < row1; base += BT * RB) {
            uint32_t id[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t i = base + r * BT + threadIdx.x;
                id[r] = i < row1 ? a.gid_row[i] : 0xFFFFFFFFu;
            }
            Row<NV, V> rr[RB];
            if constexpr (Q::kVals) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const uint32_t i = base + r * BT + threadIdx.x;
                    rr[r] = id[r] - g0 < L ? load_row<NV, V>(a.vals, i) : Row<NV, V>{};
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t i = base + r * BT + threadIdx.x;
                const bool in = id[r] - g0 < L;  // rows past the chunk carry no id in range
                const uint64_t m = __ballot(in);
                if (in) {
                    const uint32_t e = (head + cnt + rank_below(m)) & (Q::kEntries - 1);
                    q[e] = (id[r] - g0) * (uint32_t)s.words;
                    if constexpr (Q::kVals) {
                        V *qv = reinterpret_cast<V *>(q + Q::kEntries);
#pragma unroll
                        for (int c = 0; c < NV; ++c) qv[(uint32_t)c * Q::kEntries + e] = rr[r].v[c];
                    } else {
                        q[Q::kEntries + e] = i;
                    }
                }
                cnt += (uint32_t)__popcll(m);
                if (cnt >= kWave) {
                    // the entries written above by other lanes of this wave
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    hgb_queue_take<NV, BT, V, ODD>(a, s_dyn, q, head, kWave, spare);
                    head = (head + kWave) & (Q::kEntries - 1);
                    cnt -= kWave;
                    // the taken entries are read before later rows reuse them
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            (void)lane;
        }
        if (cnt) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            hgb_queue_take<NV, BT, V, ODD>(a, s_dyn, q, head, cnt, spare);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < L; i += BT) rec_flush<ODD>(s_dyn + (uint64_t)i * s.words, s, g0 + i, true);
}

template <typename K>
__global__ void k_copy_keys(const K *__restrict__ in, K *__restrict__ out, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

// ---------------------------------------------------------------------------------
// Sort-based group-by: keys sorted (with the value columns under GFTR, with row
// ids under GFUR); a head marks the first row of each run of equal keys. The
// reduction walks rows in tiles of kBlock x 16: each thread reduces its 16 rows
// sequentially, a block-level segmented scan carries each run across threads,
// and the thread holding the last row of a run writes it. Runs that start
// before the tile or reach past it are folded in with atomics.

constexpr int kSgbItems = 16;
constexpr uint32_t kSgbTile = kBlock * kSgbItems;

struct SgbArgs {
    const void *keys;     // sorted keys
    uint32_t n;
    uint32_t *tile_heads; // heads per tile -> exclusive prefix
    AggSpec spec;
    ValSrc vals;
    void *out_key;
};

template <typename K>
__global__ __launch_bounds__(kBlock) void k_sgb_heads(SgbArgs a) {
    __shared__ uint32_t s_tmp[kWaves];
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    const uint32_t t0 = blockIdx.x * kSgbTile;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kSgbItems; ++k) {
        const uint32_t i = t0 + k * kBlock + threadIdx.x;
        if (i < a.n) c += (i == 0 || keys[i] != keys[i - 1]);
    }
    uint32_t tot;
    block_exclusive_sum<uint32_t>(c, s_tmp, &tot);
    if (threadIdx.x == 0) a.tile_heads[blockIdx.x] = tot;
}

template <int NV, typename V>
__device__ __forceinline__ Acc<NV, V> acc_shfl_up(const Acc<NV, V> &x, int d) {
    Acc<NV, V> y;
    y.cnt = __shfl_up(x.cnt, d, kWave);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        y.sum[c] = __shfl_up(x.sum[c], d, kWave);
        y.mn[c] = __shfl_up(x.mn[c], d, kWave);
        y.mx[c] = __shfl_up(x.mx[c], d, kWave);
    }
    return y;
}

// Segmented combine: (f1, A1) then (f2, A2) = (f1 | f2, f2 ? A2 : A1 + A2).
template <typename K, int NV, typename V = int>
__global__ __launch_bounds__(kBlock) void k_sgb_reduce(SgbArgs a) {
    constexpr int IT = kSgbItems;
    __shared__ Acc<NV, V> s_wacc[kWaves];
    __shared__ uint32_t s_wf[kWaves];
    __shared__ uint32_t s_tmp[kWaves];
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t t0 = blockIdx.x * kSgbTile;
    const uint32_t first = t0 + tid * IT;  // this thread's rows: [first, first + IT)
    K kk[IT];
    Row<NV, V> rr[IT];
    if (first + IT <= a.n && !a.vals.rowid) {
        // a full run of consecutive rows: 16-byte loads (each lane's rows are
        // contiguous, so a wave's 4-byte loads would touch 64 lines per instruction)
        load_run16<K>(keys + first, kk);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            if (c < a.vals.n) {
                if (sizeof(V) == 8 && a.vals.w8[c]) {
                    long long t[IT];
                    load_run16<long long>(static_cast<const long long *>(a.vals.col[c]) + first, t);
#pragma unroll
                    for (int k = 0; k < IT; ++k) rr[k].v[c] = (V)t[k];
                } else {
                    int t[IT];
                    load_run16<int>(static_cast<const int *>(a.vals.col[c]) + first, t);
#pragma unroll
                    for (int k = 0; k < IT; ++k) rr[k].v[c] = (V)t[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < IT; ++k) rr[k].v[c] = V(0);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const uint32_t i = first + k;
            kk[k] = K(0);
            if (i < a.n) {
                kk[k] = keys[i];
                rr[k] = load_row<NV, V>(a.vals, i);
            }
        }
    }
    K prev = (first > 0 && first <= a.n) ? keys[first - 1] : K(0);
    uint32_t hmask = 0, hc = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const uint32_t i = first + k;
        if (i < a.n) {
            if (i == 0 || kk[k] != prev) {
                hmask |= 1u << k;
                ++hc;
            }
            prev = kk[k];
        }
    }
    const uint32_t hpre = block_exclusive_sum<uint32_t>(hc, s_tmp, (uint32_t *)nullptr);
    // this thread's tail: rows after its last head (all rows if it has none)
    Acc<NV, V> A;
    acc_clear(A);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (first + k < a.n) {
            if (hmask & (1u << k)) acc_clear(A);
            acc_row(A, rr[k]);
        }
    }
    uint32_t f = hc != 0;
    // inclusive segmented scan over the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t fo = __shfl_up(f, d, kWave);
        Acc<NV, V> Ao = acc_shfl_up(A, d);
        if (lane >= d) {
            if (!f) {
                acc_merge(Ao, A);
                A = Ao;
            }
            f |= fo;
        }
    }
    if (lane == kWave - 1) {
        s_wacc[w] = A;
        s_wf[w] = f;
    }
    uint32_t fx = __shfl_up(f, 1, kWave);
    Acc<NV, V> Ax = acc_shfl_up(A, 1);
    if (lane == 0) {
        fx = 0;
        acc_clear(Ax);
    }
    __syncthreads();
    // carry into this thread = (earlier waves) then (earlier lanes of this wave)
    Acc<NV, V> carry;
    if (fx) {
        carry = Ax;
    } else {
        acc_clear(carry);
        for (int q = 0; q < w; ++q) {
            if (s_wf[q]) carry = s_wacc[q];
            else acc_merge(carry, s_wacc[q]);
        }
        acc_merge(carry, Ax);
    }
    // Group id of a row = heads before the tile + heads of the tile up to the row - 1.
    // A run that began before this thread began inside the tile iff an earlier
    // thread of the tile had a head; only runs inside the tile are written plainly.
    const uint64_t gbase = a.tile_heads[blockIdx.x];
    Acc<NV, V> cur = carry;
    bool cur_in_tile = hpre > 0;
    uint64_t cur_gid = gbase + hpre - 1;  // wraps only before row 0, where cur is empty
    K *ok = static_cast<K *>(a.out_key);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const uint32_t i = first + k;
        if (i < a.n) {
            if (hmask & (1u << k)) {
                if (cur.cnt > 0) acc_flush(cur, a.spec, cur_gid, !cur_in_tile);
                acc_clear(cur);
                cur_gid += 1;
                cur_in_tile = true;
                if (ok) ok[cur_gid] = kk[k];
            }
            acc_row(cur, rr[k]);
        }
    }
    // the thread holding the tile's last row flushes the run that reaches it
    const uint32_t tile_end = min(t0 + kSgbTile, a.n);
    if (first < tile_end && first + IT >= tile_end && cur.cnt > 0) acc_flush(cur, a.spec, cur_gid, true);
}

// ---------------------------------------------------------------------------------
// Dictionary encoding for the sort-based group-by (Section 4.4). The dictionary
// is the global table of Algorithm 1 (ids in first-come order); sorting its g
// distinct keys gives every id its rank, so that codes follow key order and the
// group-by of the codes comes out in key order, as a sort-based group-by does.

// rank[id[p]] = p for the sorted dictionary (id[p]: the id of the p-th smallest key).
__global__ void k_de_rank(const int32_t *__restrict__ sorted_id, uint32_t g, uint32_t *__restrict__ rank) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < g; p += gridDim.x * blockDim.x)
        rank[sorted_id[p]] = p;
}

// code[i] = rank of row i's group: its key's position among the distinct keys.
__global__ void k_de_encode(const uint32_t *__restrict__ gid_loc, const uint32_t *__restrict__ gid,
                            const uint32_t *__restrict__ rank, uint32_t n, int32_t *__restrict__ code) {
    constexpr int RB = 16;
    for (uint32_t base = blockIdx.x * kBlock * RB; base < n; base += gridDim.x * kBlock * RB) {
        uint32_t loc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            loc[r] = i < n ? gid_loc[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t i = base + r * kBlock + threadIdx.x;
            if (i < n) code[i] = (int32_t)rank[gid[loc[r]]];
        }
    }
}

}  // namespace

// ---- host drivers ------------------------------------------------------------------

namespace {

// Register tier for the value columns: kernels are built for 1, 2, 4 and 8.
int nv_tier(int n_vals) { return n_vals <= 1 ? 1 : n_vals <= 2 ? 2 : n_vals <= 4 ? 4 : 8; }

// Record layout: 64-bit fields first (sums, and MIN / MAX of 8-byte columns),
// then 32-bit ones, so that every 64-bit field is 8-byte aligned. val_w: value
// column widths (nullptr: all 4 bytes).
AggSpec make_spec(const gj_agg *aggs, int n_aggs, void *const *outs, const int *val_w = nullptr,
                  bool odd_records = false) {
    AggSpec s{};
    s.n = n_aggs;
    // even-word records: 64-bit fields first, then 32-bit ones
    int w = 0, n64 = 0, first32 = -1;
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < n_aggs; ++j) {
            const int op = aggs[j].op;
            const bool w8 = (op == GJ_MIN || op == GJ_MAX) && val_w && val_w[aggs[j].col] == 8;
            const bool is64 = op == GJ_SUM || w8;
            if ((pass == 0) != is64) continue;
            s.op[j] = op;
            s.col[j] = op == GJ_COUNT ? 0 : aggs[j].col;
            s.w8[j] = w8 ? 1 : 0;
            s.word[j] = w;
            w += is64 ? 2 : 1;
            n64 += is64 ? 1 : 0;
            if (!is64 && first32 < 0) first32 = j;
            s.out[j] = outs[j];
        }
    }
    // odd-word records (an odd size needs a 32-bit field): that field first, the
    // 64-bit fields from word 1, the other 32-bit fields after them
    if (!odd_records) w = (w + 1) & ~1;  // padded to an even size
    for (int j = 0; j < n_aggs; ++j) {
        if (w % 2 == 0) s.word_odd[j] = s.word[j];
        else if (j == first32) s.word_odd[j] = 0;
        else if (s.word[j] < 2 * n64) s.word_odd[j] = s.word[j] + 1;
        else s.word_odd[j] = s.word[j] < s.word[first32] ? s.word[j] + 1 : s.word[j];
    }
    s.words = w > 0 ? w : 2;
    return s;
}

// Value source over the caller's columns (GFUR, or no transformation).
ValSrc val_src(const ValCols &vc) {
    ValSrc vs{};
    vs.n = vc.n;
    for (int c = 0; c < vc.n; ++c) {
        vs.col[c] = vc.col[c];
        vs.w8[c] = vc.width[c] == 8;
    }
    vs.rowid = nullptr;
    return vs;
}

bool any_wide(const ValCols &vc) {
    for (int c = 0; c < vc.n; ++c)
        if (vc.width[c] == 8) return true;
    return false;
}

double val_bytes(const ValCols &vc) {
    double b = 0;
    for (int c = 0; c < vc.n; ++c) b += vc.width[c];
    return b;
}

// Output column of aggregate j: SUM and COUNT int64, MIN and MAX the column's width.
size_t agg_out_width(const gj_agg &a, const ValCols &vc) {
    if (a.op == GJ_SUM || a.op == GJ_COUNT) return 8;
    return (size_t)vc.width[a.col];
}

// GFTR: value columns move with the keys into scratch columns of the same widths.
void val_transform(Ctx &ctx, const ValCols &vc, uint32_t n, PartCols &pc, ValSrc &vs) {
    pc.n = vc.n;
    vs = val_src(vc);
    for (int c = 0; c < vc.n; ++c) {
        pc.in[c] = vc.col[c];
        pc.width[c] = vc.width[c];
        pc.out[c] = ctx.scratch((size_t)n * vc.width[c]);
        vs.col[c] = pc.out[c];
    }
}

void init_outputs(hipStream_t st, const AggSpec &s, uint64_t g) {
    if (g == 0) return;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((g + 255) / 256, 4096);
    GJ_LAUNCH("k_out_init", (double)g * 4.0 * s.words, k_out_init, dim3(blocks), dim3(256), 0, st, s, g);
}

}  // namespace

size_t hgb_record_bytes(const gj_agg *aggs, int n_aggs, const int *val_w) {
    std::vector<void *> no_outs(n_aggs, nullptr);
    return (size_t)make_spec(aggs, n_aggs, no_outs.data(), val_w, false).words * 4;
}

double estimate_groups(Ctx &ctx, int key_bytes, const void *key, uint32_t n, int *varying_bytes,
                       const uint32_t **hist8) {
    if (varying_bytes) *varying_bytes = 0;
    if (hist8) *hist8 = nullptr;
    if (n == 0) return 0.0;
    hipStream_t st = ctx.stream;
    constexpr int m = 1 << kHllBits;
    uint32_t *regs = ctx.scratch_n<uint32_t>(m + 4);
    unsigned long long *bits = reinterpret_cast<unsigned long long *>(regs + m);
    fill_u32(st, regs, 0u, m + 2);
    fill_u32(st, regs + m + 2, 0xFFFFFFFFu, 2);
    if (hist8) {
        // one workgroup per chunk of the partition pass that may follow
        const uint32_t crows = pass_chunk_rows(n), chunks = ceil_div_u32(n, crows);
        uint32_t *h8 = ctx.scratch_n<uint32_t>((size_t)chunks * 256);
        *hist8 = h8;
        if (key_bytes == 4)
            GJ_LAUNCH("k_hll", 4.0 * n, (k_hll<int32_t, true>), dim3(chunks), dim3(kBlock), 0, st,
                      static_cast<const int32_t *>(key), n, regs, bits, crows, h8);
        else
            GJ_LAUNCH("k_hll", 8.0 * n, (k_hll<int64_t, true>), dim3(chunks), dim3(kBlock), 0, st,
                      static_cast<const int64_t *>(key), n, regs, bits, crows, h8);
    } else {
        const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(ceil_div_u32(n, kBlock * 16), 2048));
        if (key_bytes == 4)
            GJ_LAUNCH("k_hll", 4.0 * n, (k_hll<int32_t, false>), dim3(grid), dim3(kBlock), 0, st,
                      static_cast<const int32_t *>(key), n, regs, bits, 0u, nullptr);
        else
            GJ_LAUNCH("k_hll", 8.0 * n, (k_hll<int64_t, false>), dim3(grid), dim3(kBlock), 0, st,
                      static_cast<const int64_t *>(key), n, regs, bits, 0u, nullptr);
    }
    std::vector<uint32_t> h(m + 4);
    GJ_HIP(hipMemcpyAsync(h.data(), regs, 4ull * (m + 4), hipMemcpyDeviceToHost, st));
    GJ_HIP(hipStreamSynchronize(st));
    if (varying_bytes) {
        const uint64_t o = (uint64_t)h[m] | ((uint64_t)h[m + 1] << 32), a = (uint64_t)h[m + 2] | ((uint64_t)h[m + 3] << 32);
        for (int b = 0; b < key_bytes; ++b) *varying_bytes += (((o ^ a) >> (8 * b)) & 0xFF) != 0;
    }
    h.resize(m);
    double sum = 0.0;
    int zeros = 0;
    for (uint32_t r : h) {
        sum += std::ldexp(1.0, -(int)r);
        zeros += (r == 0);
    }
    const double alpha = 0.7213 / (1.0 + 1.079 / m);
    double e = alpha * m * (double)m / sum;
    if (e <= 2.5 * m && zeros > 0) e = m * std::log((double)m / zeros);  // small-range correction
    return std::min(e, (double)n);
}

int64_t groupby_partition(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc,
                          uint32_t n, const gj_agg *aggs, int n_aggs, bool gfur, int bits, void **out_key,
                          void **out_aggs, int *fell_back, const uint32_t *hist8) {
    hipStream_t st = ctx.stream;
    *fell_back = 0;
    const int passes = bits > 8 ? 2 : 1;
    const int n_vals = vc.n;
    // transformation: partition keys (and, under GFTR, the value columns) on the hashed key
    void *pkey = ctx.scratch((size_t)n * key_bytes);
    PartCols pc;
    ValSrc vs{};
    if (!gfur) {
        val_transform(ctx, vc, n, pc, vs);
    } else {
        vs = val_src(vc);
        pc.n = 0;
        pc.gen_rowid = true;
        pc.rowid_out = ctx.scratch((size_t)n * 4);
        vs.rowid = static_cast<const int32_t *>(pc.rowid_out);
    }
    const uint32_t np = 1u << bits;
    uint32_t *poff = ctx.scratch_n<uint32_t>(np + 1);
    partition_run(ctx, key_bytes, key, pkey, pc, n, 0, bits, passes, kDigitHash, poff, passes == 1 ? hist8 : nullptr);

    // discover: groups per partition, distinct keys in first-occurrence order
    PgbArgs a{};
    a.keys = pkey;
    a.poff = poff;
    a.np = np;
    a.tmp_keys = ctx.scratch((size_t)n * key_bytes);
    uint32_t *gcnt = ctx.scratch_n<uint32_t>(np + 1);
    uint32_t *stat = ctx.scratch_n<uint32_t>(4);
    fill_u32(st, stat, 0u, 4);
    a.gcnt = gcnt;
    a.stat = stat;
    // oversized partitions (skew, few groups) are discovered in slices by many workgroups
    uint32_t *du = ctx.scratch_n<uint32_t>(np + 1);
    GJ_LAUNCH("k_pgb_dunits", 12.0 * np, k_pgb_dunits, dim3(std::min<uint32_t>((np + 255) / 256, 1024)), dim3(256),
              0, st, poff, np, du);
    scan_exclusive_u32(ctx, du, du, np, du + np);
    a.dubase = du;
    const uint32_t max_du = 2 * ceil_div_u32(n, kDiscoverUnit) + 1;
    a.dcount = ctx.scratch_n<uint32_t>(max_du);
    // the two discovery kernels (partitions up to kDiscoverUnit rows, and slices of
    // larger ones) share one tag: together they read the keys twice
    if (key_bytes == 4) {
        GJ_LAUNCH("k_pgb_discover", 8.0 * n, k_pgb_discover<int32_t>, dim3(np), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_discover", 0.0, k_pgb_discover_unit<int32_t>, dim3(max_du), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_merge", 8.0 * np, k_pgb_merge<int32_t>, dim3(np), dim3(kBlock), 0, st, a);
    } else {
        GJ_LAUNCH("k_pgb_discover", 16.0 * n, k_pgb_discover<int64_t>, dim3(np), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_discover", 0.0, k_pgb_discover_unit<int64_t>, dim3(max_du), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_merge", 16.0 * np, k_pgb_merge<int64_t>, dim3(np), dim3(kBlock), 0, st, a);
    }
    scan_exclusive_u32(ctx, gcnt, gcnt, np, gcnt + np);
    uint32_t *ucnt = ctx.scratch_n<uint32_t>(np + 1);
    GJ_LAUNCH("k_pgb_units", 16.0 * np, k_pgb_units, dim3(std::min<uint32_t>((np + 255) / 256, 1024)), dim3(256),
              0, st, poff, (const uint32_t *)gcnt, np, ucnt, stat + 2);
    scan_exclusive_u32(ctx, ucnt, ucnt, np, ucnt + np);
    uint32_t host[5];
    GJ_HIP(hipMemcpyAsync(&host[0], gcnt + np, 4, hipMemcpyDeviceToHost, st));
    GJ_HIP(hipMemcpyAsync(&host[1], stat, 12, hipMemcpyDeviceToHost, st));
    GJ_HIP(hipMemcpyAsync(&host[4], ucnt + np, 4, hipMemcpyDeviceToHost, st));
    GJ_HIP(hipStreamSynchronize(st));
    const uint32_t g = host[0], maxg = host[1], over = host[2], max_units = host[3], units = host[4];
    if (over) {
        *fell_back = 1;  // some partition holds more distinct keys than its LDS table
        return -1;
    }
    // outputs
    *out_key = ctx.output((size_t)std::max<uint32_t>(g, 1) * key_bytes);
    std::vector<void *> outs(n_aggs);
    for (int j = 0; j < n_aggs; ++j) {
        outs[j] = ctx.output((size_t)std::max<uint32_t>(g, 1) * agg_out_width(aggs[j], vc));
        out_aggs[j] = outs[j];
    }
    if (g == 0) return 0;
    a.spec = make_spec(aggs, n_aggs, outs.data(), vc.width);
    a.vals = vs;
    a.goff = gcnt;
    a.ubase = ucnt;
    a.out_key = *out_key;
    a.nunits = ucnt + np;
    a.cap_units = units;
    a.out_base = nullptr;
    a.lds_bytes = 0;
    // LDS: the aggregation table (key and group id per slot), then maxg records and
    // the spare words
    const auto tab_bytes = [&](int l) { return ((size_t)1 << l) * agg_slot_bytes(key_bytes) + 8; };
    const size_t rec_bytes = (((size_t)maxg + 1) * a.spec.words + kSpareWords) * 4;
    int log2cap = agg_table_log2(maxg);
    size_t lds = tab_bytes(log2cap) + rec_bytes;
    a.lds_records = 1;
    if (lds > 120 * 1024 || log2cap > 16) {
        a.lds_records = 0;  // too many groups per partition for LDS records: global atomics
        lds = tab_bytes(log2cap);
    }
    require(lds <= 150 * 1024, "partition group-by: too many groups per partition", GJ_EUNSUPPORTED);
    // fewer than three 256-thread workgroups per compute unit (by LDS): 1024-thread
    // ones (one or two value columns; more would spill registers)
    const bool wide = lds > 160 * 1024 / 3 && nv_tier(n_vals) <= 2;
    // The table starts at 1.5 slots per group and grows, up to 4 per group (fewer
    // lookups probe past their first slot), within the LDS that the workgroups
    // the registers allow per compute unit leave: 32 KB for 256-thread ones (five
    // per compute unit), the whole budget for a 1024-thread one.
    {
        const size_t room = wide ? (size_t)150 * 1024 : std::max<size_t>((size_t)32 * 1024, lds);
        const size_t keys = std::max<size_t>(std::min(maxg, kDiscoverCap), 16), need = a.lds_records ? rec_bytes : 0;
        while (((size_t)2 << log2cap) <= 4 * keys && tab_bytes(log2cap + 1) + need <= room) ++log2cap;
        lds = tab_bytes(log2cap) + need;
    }
    a.log2cap = log2cap;
    lds = std::max<size_t>(lds, (size_t)16 * 256 + 16);  // the one-group path keeps a per-wave total
    // outputs of partitions split over several units are folded with atomics
    if (max_units > 1 || !a.lds_records) init_outputs(st, a.spec, g);
    // skew: the largest partition holds at least twice the mean partition's units
    const bool skewed = (uint64_t)max_units * np >= 2ull * units && max_units >= 4;
    const double bytes = (double)n * (key_bytes + val_bytes(vc) + (gfur ? 4.0 : 0.0)) +
                         (double)g * (key_bytes + 4.0 * a.spec.words);
    const int nvt = nv_tier(n_vals);
#define GJ_PGB(K, NV, V) launch_pgb_aggregate<K, NV, V>(wide, skewed, units, lds, st, a, bytes)
#define GJ_PGB_NV(K, V) \
    if (nvt == 1) GJ_PGB(K, 1, V); else if (nvt == 2) GJ_PGB(K, 2, V); else if (nvt == 4) GJ_PGB(K, 4, V); else GJ_PGB(K, 8, V)
    if (any_wide(vc)) {
        if (key_bytes == 4) { GJ_PGB_NV(int32_t, long long); } else { GJ_PGB_NV(int64_t, long long); }
    } else {
        if (key_bytes == 4) { GJ_PGB_NV(int32_t, int); } else { GJ_PGB_NV(int64_t, int); }
    }
#undef GJ_PGB_NV
#undef GJ_PGB
    return g;
}

uint32_t pgb_plan_lds_bytes(int key_bytes) {
    // room for the largest per-partition table (2 x kDiscoverCap slots of key and
    // group id), and at least 64 KiB so that records of ~1000 groups fit beside
    // a small table
    return std::max<uint32_t>(2u * kDiscoverCap * agg_slot_bytes(key_bytes) + 8, 65536u);
}

void groupby_partition_segments(Ctx &ctx, int key_bytes, const void *key, const int32_t *const *vals, int n_vals,
                                uint32_t n, const gj_agg *aggs, int n_aggs, bool gfur, const uint32_t *seg_off,
                                uint32_t nseg, const uint8_t *seg_bits, const PgbPlanned &pl) {
    hipStream_t st = ctx.stream;
    void *pkey = ctx.scratch((size_t)n * key_bytes);
    PartCols pc;
    ValSrc vs{};
    vs.n = n_vals;
    if (!gfur) {
        pc.n = n_vals;
        for (int c = 0; c < n_vals; ++c) {
            pc.in[c] = vals[c];
            pc.width[c] = 4;
            pc.out[c] = ctx.scratch((size_t)n * 4);
            vs.col[c] = static_cast<const int32_t *>(pc.out[c]);
        }
        vs.rowid = nullptr;
    } else {
        pc.gen_rowid = true;
        pc.rowid_out = ctx.scratch((size_t)n * 4);
        for (int c = 0; c < n_vals; ++c) vs.col[c] = vals[c];
        vs.rowid = static_cast<const int32_t *>(pc.rowid_out);
    }
    const uint32_t np = nseg << 8;
    uint32_t *poff = ctx.scratch_n<uint32_t>(np + 1);
    partition_run_segments(ctx, key_bytes, key, pkey, pc, n, seg_off, nseg, seg_bits, poff, kDigitHash);

    PgbArgs a{};
    a.keys = pkey;
    a.poff = poff;
    a.np = np;
    a.tmp_keys = ctx.scratch((size_t)n * key_bytes);
    uint32_t *gcnt = ctx.scratch_n<uint32_t>(np + 1);
    uint32_t *stat = ctx.scratch_n<uint32_t>(4);
    fill_u32(st, stat, 0u, 4);
    a.gcnt = gcnt;
    a.stat = stat;
    uint32_t *du = ctx.scratch_n<uint32_t>(np + 1);
    GJ_LAUNCH("k_pgb_dunits", 12.0 * np, k_pgb_dunits, dim3(std::min<uint32_t>((np + 255) / 256, 1024)), dim3(256),
              0, st, poff, np, du);
    scan_exclusive_u32(ctx, du, du, np, du + np);
    a.dubase = du;
    const uint32_t max_du = 2 * ceil_div_u32(n, kDiscoverUnit) + 1;
    a.dcount = ctx.scratch_n<uint32_t>(max_du);
    // the two discovery kernels (partitions up to kDiscoverUnit rows, and slices of
    // larger ones) share one tag: together they read the keys twice
    if (key_bytes == 4) {
        GJ_LAUNCH("k_pgb_discover", 8.0 * n, k_pgb_discover<int32_t>, dim3(np), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_discover", 0.0, k_pgb_discover_unit<int32_t>, dim3(max_du), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_merge", 8.0 * np, k_pgb_merge<int32_t>, dim3(np), dim3(kBlock), 0, st, a);
    } else {
        GJ_LAUNCH("k_pgb_discover", 16.0 * n, k_pgb_discover<int64_t>, dim3(np), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_discover", 0.0, k_pgb_discover_unit<int64_t>, dim3(max_du), dim3(kBlock), 0, st, a);
        GJ_LAUNCH("k_pgb_merge", 16.0 * np, k_pgb_merge<int64_t>, dim3(np), dim3(kBlock), 0, st, a);
    }
    scan_exclusive_u32(ctx, gcnt, gcnt, np, gcnt + np);
    uint32_t *ucnt = ctx.scratch_n<uint32_t>(np + 1);
    GJ_LAUNCH("k_pgb_units", 16.0 * np, k_pgb_units, dim3(std::min<uint32_t>((np + 255) / 256, 1024)), dim3(256),
              0, st, poff, (const uint32_t *)gcnt, np, ucnt, stat + 2);
    scan_exclusive_u32(ctx, ucnt, ucnt, np, ucnt + np);

    a.spec = make_spec(aggs, n_aggs, pl.out_aggs);
    a.vals = vs;
    a.goff = gcnt;
    a.ubase = ucnt;
    a.out_key = pl.out_key;
    a.nunits = ucnt + np;
    a.cap_units = pl.cap_units;
    a.out_base = pl.out_base;
    a.lds_bytes = pl.lds_bytes;
    a.log2cap = 6;
    a.lds_records = 0;
    const uint32_t init_blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096));
    GJ_LAUNCH("k_out_init", 4.0 * a.spec.words * n, k_out_init_dev, dim3(init_blocks), dim3(256), 0, st, a.spec,
              pl.out_base, (const uint32_t *)(gcnt + np), pl.out_cap);
    GJ_LAUNCH("k_pgb_inst_offsets", 12.0 * (nseg + 1), k_pgb_inst_offsets,
              dim3(std::min<uint32_t>(ceil_div_u32(nseg + 1, 256), 1024)), dim3(256), 0, st, (const uint32_t *)gcnt,
              nseg, pl.out_base, pl.inst_goff);
    GJ_LAUNCH("k_pgb_status", 16.0, k_pgb_status, dim3(1), dim3(64), 0, st, pl.out_base,
              (const uint32_t *)(gcnt + np), pl.next_base, (const uint32_t *)stat, (const uint32_t *)(ucnt + np),
              pl.status);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(pl.cap_units, 4096));
    // Two launches over the same units: partitions of at most small_g groups run
    // with a small LDS (more workgroups per compute unit), the rest with the
    // plan's LDS, which holds the largest discoverable partition. The LDS of a
    // captured launch is fixed, and the group counts are only known on the device.
    const uint32_t small_lds = 24u * 1024u;
    uint32_t small_g = 0;
    for (uint32_t x = 16; x <= kDiscoverCap; x += 16) {
        const uint32_t tab = (1u << agg_table_log2(x)) * agg_slot_bytes(key_bytes) + 8u;
        const uint32_t rec = ((x + 1) * (uint32_t)a.spec.words + kSpareWords) * 4u;
        if (tab + rec + 8u > small_lds) break;
        small_g = x;
    }
    const double bytes = (double)n * (key_bytes + 4.0 * n_vals + (gfur ? 4.0 : 0.0));
    uint32_t lds = pl.lds_bytes;
#define GJ_PGB(K, NV) GJ_LAUNCH("k_pgb_aggregate", bytes, (k_pgb_aggregate<K, NV>), dim3(grid), dim3(kBlock), lds, st, a)
#define GJ_PGB_ALL                                                                                          \
    do {                                                                                                    \
        const int nvt = nv_tier(n_vals);                                                                    \
        if (key_bytes == 4) {                                                                               \
            if (nvt == 1) GJ_PGB(int32_t, 1); else if (nvt == 2) GJ_PGB(int32_t, 2);                        \
            else if (nvt == 4) GJ_PGB(int32_t, 4); else GJ_PGB(int32_t, 8);                                 \
        } else {                                                                                            \
            if (nvt == 1) GJ_PGB(int64_t, 1); else if (nvt == 2) GJ_PGB(int64_t, 2);                        \
            else if (nvt == 4) GJ_PGB(int64_t, 4); else GJ_PGB(int64_t, 8);                                 \
        }                                                                                                   \
    } while (0)
    if (small_g > 0) {
        a.lds_bytes = lds = small_lds;
        a.g_lo = 1;
        a.g_hi = small_g;
        GJ_PGB_ALL;
    }
    a.lds_bytes = lds = pl.lds_bytes;
    a.g_lo = small_g + 1;
    a.g_hi = 0xFFFFFFFFu;
    GJ_PGB_ALL;
#undef GJ_PGB_ALL
#undef GJ_PGB
}

// Stage 1 of Algorithm 1: dense group ids from a global table. Fills a.gid (for
// the inserting rows), a.gid_loc, a.tmp_keys (the key of each id) and returns
// the group count. One workgroup first inserts the first `prefix` rows a tile at
// a time, so that the keys seen there take the lowest ids (see groupby_hash).
// The table: 1.5 slots per row always holds every group; with a group-count
// estimate it is sized for that instead (load `occupancy`, default 0.45), and a
// row that finds no slot within 4096 probes sends the insert back to the
// row-sized table.
static uint32_t hgb_assign_ids(Ctx &ctx, HgbArgs &a, int key_bytes, const void *key, uint32_t n, uint32_t prefix,
                        double g_est, float occupancy) {
    hipStream_t st = ctx.stream;
    a.keys = key;
    a.n = n;
    const size_t slot = key_bytes == 4 ? 8 : 4;
    a.gid = ctx.scratch_n<uint32_t>(n);
    a.gid_loc = ctx.scratch_n<uint32_t>(n);
    a.ngroups = ctx.scratch_n<uint32_t>(2);
    a.tmp_keys = ctx.scratch((size_t)n * key_bytes);
    prefix = std::min(prefix, n);
    const uint32_t grid = std::min<uint32_t>(ceil_div_u32(n, kBlock), 256u * 16u);
    int log2rows = 4;
    while ((1ull << log2rows) < (uint64_t)n + n / 2) ++log2rows;
    const auto insert = [&](int log2cap, uint32_t max_probe) {
        a.log2cap = log2cap;
        a.max_probe = max_probe;
        a.table = ctx.scratch(((size_t)1 << log2cap) * slot);
        if (key_bytes == 4) fill_u64(st, static_cast<uint64_t *>(a.table), ~0ull, (uint64_t)1 << log2cap);
        else fill_u32(st, static_cast<uint32_t *>(a.table), 0xFFFFFFFFu, (uint64_t)1 << log2cap);
        fill_u32(st, a.ngroups, 0u, 2);
        HgbArgs ap = a;
        ap.n = prefix;
        if (key_bytes == 4) {
            GJ_LAUNCH("k_hgb_insert", 8.0 * prefix, k_hgb_insert<int32_t>, dim3(1), dim3(kBlock), 0, st, ap);
            if (n > prefix) {
                // up to a few thousand groups: every workgroup caches the keys it
                // resolved (an 8192-entry LDS table, at most three quarters full)
                if (g_est > 0.0 && g_est <= 6144.0 && ((uintptr_t)key & 15u) == 0 && ((uintptr_t)a.gid_loc & 15u) == 0)
                    GJ_LAUNCH("k_hgb_insert", 8.0 * n, k_hgb_insert_cached<13>,
                              dim3(std::min<uint32_t>(ceil_div_u32(n, kInsBlock * kInsRows), 512)), dim3(kInsBlock), 0, st,
                              a);
                else
                    GJ_LAUNCH("k_hgb_insert", 8.0 * n, k_hgb_insert<int32_t>, dim3(grid), dim3(kBlock), 0, st, a);
            }
        } else {
            GJ_LAUNCH("k_hgb_insert", 12.0 * prefix, k_hgb_insert<int64_t>, dim3(1), dim3(kBlock), 0, st, ap);
            if (n > prefix) {
                // up to a few thousand groups: a 4096-entry LDS cache per workgroup
                if (g_est > 0.0 && g_est <= 3072.0 && ((uintptr_t)key & 15u) == 0 && ((uintptr_t)a.gid_loc & 15u) == 0)
                    GJ_LAUNCH("k_hgb_insert", 12.0 * n, k_hgb_insert_cached8<12>,
                              dim3(std::min<uint32_t>(ceil_div_u32(n, kInsBlock * kInsRows8), 512)), dim3(kInsBlock),
                              0, st, a);
                else
                    GJ_LAUNCH("k_hgb_insert", 12.0 * n, k_hgb_insert<int64_t>, dim3(grid), dim3(kBlock), 0, st, a);
            }
        }
        uint32_t h[2];
        GJ_HIP(hipMemcpyAsync(h, a.ngroups, 8, hipMemcpyDeviceToHost, st));
        GJ_HIP(hipStreamSynchronize(st));
        return std::make_pair(h[0], h[1] != 0);
    };
    std::pair<uint32_t, bool> r{0, true};
    if (g_est > 0.0) {
        const double occ = occupancy > 0.0f ? (double)occupancy : 0.45;
        int log2est = 12;
        while (log2est < log2rows && (double)(1ull << log2est) * occ < g_est) ++log2est;
        if (log2est < log2rows) r = insert(log2est, 4096);
    }
    if (r.second) r = insert(log2rows, 0xFFFFFFFFu);
    require(!r.second, "hash group-by: no table slot for a key", GJ_EUNSUPPORTED);  // cannot happen: slots > rows
    return r.first;
}

int64_t groupby_hash(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                     const gj_agg *aggs, int n_aggs, int lds_budget, double g_est, float occupancy, void **out_key,
                     void **out_aggs) {
    hipStream_t st = ctx.stream;
    HgbArgs a{};
    const uint32_t grid = std::min<uint32_t>(ceil_div_u32(n, kBlock), 256u * 16u);
    // Group ids come from an atomic counter, so a full grid hands them out in the
    // order its first tiles happen to win, unrelated to key frequency. One
    // workgroup first inserts a prefix of the rows a tile at a time: the keys seen
    // there take the low ids, and under skew those are the frequent keys. Low ids
    // are the ones that keep LDS records when not every group fits. The full pass
    // then finds the prefix keys already present.
    const int n_vals = vc.n;
    std::vector<void *> no_outs(n_aggs, nullptr);
    const size_t rec_even = (size_t)make_spec(aggs, n_aggs, no_outs.data(), vc.width, false).words * 4;
    const size_t rec_odd = (size_t)make_spec(aggs, n_aggs, no_outs.data(), vc.width, true).words * 4;
    const size_t budget = std::min(lds_budget > 0 ? (size_t)lds_budget : (size_t)64 * 1024, (size_t)64 * 1024);
    const uint32_t prefix = (uint32_t)std::max<size_t>(2048, 2 * (budget / rec_even));
    const uint32_t g = hgb_assign_ids(ctx, a, key_bytes, key, n, prefix, g_est, occupancy);
    *out_key = ctx.output((size_t)std::max<uint32_t>(g, 1) * key_bytes);
    std::vector<void *> outs(n_aggs);
    for (int j = 0; j < n_aggs; ++j) {
        outs[j] = ctx.output((size_t)std::max<uint32_t>(g, 1) * agg_out_width(aggs[j], vc));
        out_aggs[j] = outs[j];
    }
    if (g == 0) return 0;
    a.vals = val_src(vc);
    a.g = g;
    const bool v64 = any_wide(vc);
    const int nvt = nv_tier(n_vals);
    // is_smem_enough, per slice: when the groups fit the LDS of a workgroup (at
    // most the 160 KB of a compute unit) in at most kHgbMaxSlices consecutive id
    // ranges, every record stays in LDS.
    const size_t max_lds = (size_t)160 * 1024;
    const size_t sbudget = std::min(lds_budget > 0 ? (size_t)lds_budget : max_lds, max_lds);
    const size_t fixed = kSpareWords * 4 + 16;  // spare words, alignment of the queues
    // several slices also need the row queues (for the workgroup size they will run)
    const bool q_wide = sbudget > max_lds / 4;
    const size_t qbytes = hgb_queue_bytes(nvt, v64 ? 8 : 4, q_wide ? 1024u : kBlock);
    const auto slices_for = [&](size_t rec) -> uint32_t {
        const auto groups_in = [&](size_t bytes) -> size_t {
            return bytes > fixed + rec ? (bytes - fixed) / rec - 1 : 0;
        };
        const size_t per_one = groups_in(sbudget);
        const size_t per_wg = g <= per_one ? per_one : groups_in(sbudget > qbytes ? sbudget - qbytes : 0);
        return per_wg >= 64 ? (uint32_t)((g + per_wg - 1) / per_wg) : 0u;
    };
    // Records without the padding word (odd sizes) hold about one group in nine more
    // but cost a parity test per field and row: taken only where they save a slice.
    const uint32_t s_even = slices_for(rec_even), s_odd = slices_for(rec_odd);
    const bool odd = s_odd >= 1 && s_odd <= kHgbMaxSlices && (s_even == 0 || s_even > kHgbMaxSlices || s_odd < s_even);
    const uint32_t slices = odd ? s_odd : s_even;
    const size_t rec = odd ? rec_odd : rec_even;
    a.spec = make_spec(aggs, n_aggs, outs.data(), vc.width, odd);
    init_outputs(st, a.spec, g);
    // stage 2 reads each row's values and its group id (gid_loc and gid[gid_loc], or
    // the resolved id once for several slices), and writes every group once
    double bytes = (double)n * (val_bytes(vc) + 8.0) + (double)g * (key_bytes + 4.0 * a.spec.words);
    // a handful of groups: register accumulators (four for up to two 4-byte value
    // columns, else two)
    const uint32_t few_max = (!v64 && nvt <= 2) ? 4u : 2u;
    if (g <= few_max) {
        a.lds_groups = g;
        const size_t alds = ((size_t)g + 1) * rec + kSpareWords * 4;
        const uint32_t fgrid = std::min<uint32_t>(grid, 2048);
#define GJ_HFEW(NV, V, G)     GJ_LAUNCH("k_hgb_aggregate", bytes, (k_hgb_aggregate_few<NV, V, G>), dim3(fgrid), dim3(kBlock), alds, st, a)
        if (v64) {
            if (nvt == 1) GJ_HFEW(1, long long, 2); else if (nvt == 2) GJ_HFEW(2, long long, 2);
            else if (nvt == 4) GJ_HFEW(4, long long, 2); else GJ_HFEW(8, long long, 2);
        } else {
            if (nvt == 1) GJ_HFEW(1, int, 4); else if (nvt == 2) GJ_HFEW(2, int, 4); else if (nvt == 4) GJ_HFEW(4, int, 2);
            else GJ_HFEW(8, int, 2);
        }
#undef GJ_HFEW
    } else if (slices >= 1 && slices <= kHgbMaxSlices) {
        a.slices = slices;
        a.slice_groups = ceil_div_u32(g, slices);
        const size_t rec_lds = ((((size_t)a.slice_groups + 1) * rec + kSpareWords * 4) + 15) & ~(size_t)15;
        const bool wide = slices > 1 ? q_wide : rec_lds > max_lds / 4;  // fewer than four 256-thread workgroups per CU
        const size_t alds = rec_lds + (slices > 1 ? hgb_queue_bytes(nvt, v64 ? 8 : 4, wide ? 1024u : kBlock) : 0);
        require(alds <= max_lds, "hash group-by: slice exceeds the LDS", GJ_EUNSUPPORTED);
        const uint32_t per_cu = (uint32_t)std::max<size_t>(1, std::min<size_t>(wide ? 2 : 8, max_lds / alds));
        // about two rounds of resident workgroups over all slices, chunks a multiple of the XCDs
        uint32_t chunks = ceil_div_u32(2u * 256u * per_cu, slices);
        chunks = std::max<uint32_t>(kXcds, (chunks + kXcds - 1) / kXcds * kXcds);
        a.chunks = chunks;
        a.chunk_rows = ceil_div_u32(n, chunks);
        a.gid_row = nullptr;
        if (slices > 1) {
            uint32_t *gr = ctx.scratch_n<uint32_t>(n);
            GJ_LAUNCH("k_hgb_resolve", 8.0 * n, k_hgb_resolve, dim3(std::min<uint32_t>(ceil_div_u32(n, kBlock * 16), 4096)),
                      dim3(kBlock), 0, st, a.gid_loc, a.gid, n, gr);
            a.gid_row = gr;
            bytes -= 4.0 * n;
        }
        const uint32_t sgrid = chunks * slices;
#define GJ_HAGG_S(NV, BT, V)                                                                                       \
    if (odd) GJ_LAUNCH("k_hgb_aggregate", bytes, (k_hgb_aggregate_sliced<NV, BT, V, true>), dim3(sgrid), dim3(BT),  \
                       alds, st, a);                                                                                  \
    else GJ_LAUNCH("k_hgb_aggregate", bytes, (k_hgb_aggregate_sliced<NV, BT, V, false>), dim3(sgrid), dim3(BT), alds, \
                   st, a)
#define GJ_HAGG_S_NV(BT, V) \
    if (nvt == 1) GJ_HAGG_S(1, BT, V); else if (nvt == 2) GJ_HAGG_S(2, BT, V); \
    else if (nvt == 4) GJ_HAGG_S(4, BT, V); else GJ_HAGG_S(8, BT, V)
        if (v64) {
            if (wide) { GJ_HAGG_S_NV(1024, long long); } else { GJ_HAGG_S_NV(256, long long); }
        } else {
            if (wide) { GJ_HAGG_S_NV(1024, int); } else { GJ_HAGG_S_NV(256, int); }
        }
#undef GJ_HAGG_S_NV
#undef GJ_HAGG_S
    } else {
        // Otherwise the lowest ids that fit (at most the budget, 64 KiB by default)
        // keep LDS records and the rest take global atomics; with the prefix insert
        // above, the frequent keys hold those ids under skew and most rows stay off
        // the contended global atomics.
        a.lds_groups = (uint32_t)std::min<size_t>(g, budget / rec);
        const size_t alds = a.lds_groups ? ((size_t)a.lds_groups + 1) * rec + kSpareWords * 4 : 0;
        // every workgroup folds its LDS records into the output with global atomics:
        // the grid keeps that near 2^19 record flushes, but never drops below one
        // round of resident workgroups (by LDS, and at most 7 per compute unit by
        // registers)
        const uint32_t per_cu = alds ? (uint32_t)std::max<size_t>(1, std::min<size_t>(7, (160u * 1024u) / alds)) : 0;
        const uint32_t agrid =
            alds ? std::min<uint32_t>(grid, std::max<uint32_t>(256u * per_cu, (1u << 19) / a.lds_groups)) : grid;
#define GJ_HAGG(NV, V) \
    GJ_LAUNCH("k_hgb_aggregate", bytes, (k_hgb_aggregate<NV, V>), dim3(agrid), dim3(kBlock), alds, st, a)
        if (v64) {
            if (nvt == 1) GJ_HAGG(1, long long); else if (nvt == 2) GJ_HAGG(2, long long);
            else if (nvt == 4) GJ_HAGG(4, long long); else GJ_HAGG(8, long long);
        } else {
            if (nvt == 1) GJ_HAGG(1, int); else if (nvt == 2) GJ_HAGG(2, int); else if (nvt == 4) GJ_HAGG(4, int);
            else GJ_HAGG(8, int);
        }
#undef GJ_HAGG
    }
    const uint32_t cb = std::min<uint32_t>(ceil_div_u32(g, 256), 4096);
    if (key_bytes == 4)
        GJ_LAUNCH("k_copy_keys", 8.0 * g, k_copy_keys<int32_t>, dim3(cb), dim3(256), 0, st,
                  static_cast<const int32_t *>(a.tmp_keys), static_cast<int32_t *>(*out_key), (uint64_t)g);
    else
        GJ_LAUNCH("k_copy_keys", 16.0 * g, k_copy_keys<int64_t>, dim3(cb), dim3(256), 0, st,
                  static_cast<const int64_t *>(a.tmp_keys), static_cast<int64_t *>(*out_key), (uint64_t)g);
    return g;
}

int64_t groupby_sort(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                     const gj_agg *aggs, int n_aggs, bool gfur, void **out_key, void **out_aggs) {
    hipStream_t st = ctx.stream;
    const int n_vals = vc.n;
    // transformation: LSD radix sort on the order-preserving key bits
    void *skey = ctx.scratch((size_t)n * key_bytes);
    PartCols pc;
    ValSrc vs{};
    if (!gfur) {
        val_transform(ctx, vc, n, pc, vs);
    } else {
        vs = val_src(vc);
        pc.gen_rowid = true;
        pc.rowid_out = ctx.scratch((size_t)n * 4);
        vs.rowid = static_cast<const int32_t *>(pc.rowid_out);
    }
    sort_run(ctx, key_bytes, key, skey, pc, n);

    SgbArgs a{};
    a.keys = skey;
    a.n = n;
    const uint32_t tiles = ceil_div_u32(n, kSgbTile);
    a.tile_heads = ctx.scratch_n<uint32_t>(tiles + 1);
    if (key_bytes == 4)
        GJ_LAUNCH("k_sgb_heads", 4.0 * n, k_sgb_heads<int32_t>, dim3(tiles), dim3(kBlock), 0, st, a);
    else
        GJ_LAUNCH("k_sgb_heads", 8.0 * n, k_sgb_heads<int64_t>, dim3(tiles), dim3(kBlock), 0, st, a);
    scan_exclusive_u32(ctx, a.tile_heads, a.tile_heads, tiles, a.tile_heads + tiles);
    const uint32_t g = read_back(a.tile_heads + tiles, st);
    *out_key = ctx.output((size_t)std::max<uint32_t>(g, 1) * key_bytes);
    std::vector<void *> outs(n_aggs);
    for (int j = 0; j < n_aggs; ++j) {
        outs[j] = ctx.output((size_t)std::max<uint32_t>(g, 1) * agg_out_width(aggs[j], vc));
        out_aggs[j] = outs[j];
    }
    if (g == 0) return 0;
    a.spec = make_spec(aggs, n_aggs, outs.data(), vc.width);
    a.vals = vs;
    a.out_key = *out_key;
    init_outputs(st, a.spec, g);
    const double bytes = (double)n * (key_bytes + val_bytes(vc) + (gfur ? 4.0 : 0.0)) +
                         (double)g * (key_bytes + 4.0 * a.spec.words);
    const int nvt = nv_tier(n_vals);
#define GJ_SGB(K, NV, V) \
    GJ_LAUNCH("k_sgb_reduce", bytes, (k_sgb_reduce<K, NV, V>), dim3(tiles), dim3(kBlock), 0, st, a)
#define GJ_SGB_NV(K, V) \
    if (nvt == 1) GJ_SGB(K, 1, V); else if (nvt == 2) GJ_SGB(K, 2, V); else if (nvt == 4) GJ_SGB(K, 4, V); \
    else GJ_SGB(K, 8, V)
    if (any_wide(vc)) {
        if (key_bytes == 4) { GJ_SGB_NV(int32_t, long long); } else { GJ_SGB_NV(int64_t, long long); }
    } else {
        if (key_bytes == 4) { GJ_SGB_NV(int32_t, int); } else { GJ_SGB_NV(int64_t, int); }
    }
#undef GJ_SGB_NV
#undef GJ_SGB
    return g;
}

int64_t groupby_sort_de(Ctx &ctx, int key_bytes, const void *key, const ValCols &vc, uint32_t n,
                        const gj_agg *aggs, int n_aggs, double g_est, float occupancy, void **out_key,
                        void **out_aggs) {
    hipStream_t st = ctx.stream;
    // the dictionary: Algorithm 1's dense ids over the distinct keys
    HgbArgs h{};
    const uint32_t g = hgb_assign_ids(ctx, h, key_bytes, key, n, 2048, g_est, occupancy);
    *out_key = ctx.output((size_t)std::max<uint32_t>(g, 1) * key_bytes);
    std::vector<void *> outs(n_aggs);
    for (int j = 0; j < n_aggs; ++j) {
        outs[j] = ctx.output((size_t)std::max<uint32_t>(g, 1) * agg_out_width(aggs[j], vc));
        out_aggs[j] = outs[j];
    }
    if (g == 0) return 0;
    // the distinct keys in order (they are the output keys) and each id's rank
    PartCols dc;
    dc.gen_rowid = true;
    int32_t *sorted_id = ctx.scratch_n<int32_t>(g);
    dc.rowid_out = sorted_id;
    sort_run(ctx, key_bytes, h.tmp_keys, *out_key, dc, g);
    uint32_t *rank = ctx.scratch_n<uint32_t>(g);
    GJ_LAUNCH("k_de_rank", 8.0 * g, k_de_rank, dim3(std::min<uint32_t>(ceil_div_u32(g, 256), 4096)), dim3(256), 0,
              st, sorted_id, g, rank);
    // encoding: one 4-byte code per row
    int32_t *code = ctx.scratch_n<int32_t>(n);
    GJ_LAUNCH("k_de_encode", 8.0 * n, k_de_encode, dim3(std::min<uint32_t>(ceil_div_u32(n, kBlock * 16), 4096)),
              dim3(kBlock), 0, st, h.gid_loc, h.gid, rank, n, code);
    // sort (code, values) on the code bytes that vary: ceil(log2 g / 8) passes
    int32_t *scode = ctx.scratch_n<int32_t>(n);
    PartCols pc;
    ValSrc vs{};
    val_transform(ctx, vc, n, pc, vs);
    sort_run(ctx, 4, code, scode, pc, n);
    // segmented reduction over the sorted codes: group j is code j
    SgbArgs a{};
    a.keys = scode;
    a.n = n;
    const uint32_t tiles = ceil_div_u32(n, kSgbTile);
    a.tile_heads = ctx.scratch_n<uint32_t>(tiles + 1);
    GJ_LAUNCH("k_sgb_heads", 4.0 * n, k_sgb_heads<int32_t>, dim3(tiles), dim3(kBlock), 0, st, a);
    scan_exclusive_u32(ctx, a.tile_heads, a.tile_heads, tiles, a.tile_heads + tiles);
    a.spec = make_spec(aggs, n_aggs, outs.data(), vc.width);
    a.vals = vs;
    a.out_key = nullptr;
    init_outputs(st, a.spec, g);
    const double bytes = (double)n * (4.0 + val_bytes(vc)) + (double)g * (key_bytes + 4.0 * a.spec.words);
    const int nvt = nv_tier(vc.n);
#define GJ_SGB(NV, V) \
    GJ_LAUNCH("k_sgb_reduce", bytes, (k_sgb_reduce<int32_t, NV, V>), dim3(tiles), dim3(kBlock), 0, st, a)
    if (any_wide(vc)) {
        if (nvt == 1) GJ_SGB(1, long long); else if (nvt == 2) GJ_SGB(2, long long);
        else if (nvt == 4) GJ_SGB(4, long long); else GJ_SGB(8, long long);
    } else {
        if (nvt == 1) GJ_SGB(1, int); else if (nvt == 2) GJ_SGB(2, int); else if (nvt == 4) GJ_SGB(4, int);
        else GJ_SGB(8, int);
    }
#undef GJ_SGB
    return g;
}

}  // namespace gj
