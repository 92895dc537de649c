// Match finding and materialization of the partitioned hash join
// (Section 4.1.4, steps 2 and 3).
//
// After partitioning, partition p of R and of S are contiguous ranges. Work
// units cut a partition pair into (R block of at most r_block rows) x (S piece
// of at most 2 x table rows), so that an oversized or skewed partition is spread
// over many workgroups (the load balancing of Sections 3.1.2 and 4.1.4). Per
// unit, a workgroup builds a bucketed hash table on the R block in LDS and
// streams the S piece through it. The table has 4096, 8192 or 16384 rows (the
// smallest that holds r_block) and the workgroup 16 table rows per thread.
//
// The output size is unknown (Section 2.2), so a count pass runs first: every
// wave counts its matches and records each S row's match; an exclusive scan
// over (unit, wave) gives every wave its output range. The write pass then
// writes (key, R payloads, S payloads) contiguously. In the common case (one R
// block per partition, at most one match per S row) it streams S with the
// recorded matches and needs no table; otherwise it rebuilds the table and
// enumerates the matches again. GFTR reads payloads from the partitioned
// copies at partition-local positions (clustered), staged in LDS when they
// fit; GFUR reads the original columns through the partitioned row ids
// (unclustered).
//
// In the write pass, chains of the LDS table list R rows in input order, so an
// S row with several matches emits them in R's input order, and the output is
// the same on every run.
#include "internal.hpp"

namespace gj {
namespace {

constexpr uint32_t kMaxChainSort = 32;
constexpr uint16_t kNoMatch = 0xFFFF;  // blocks hold at most 16384 rows
constexpr uint32_t kPersistentGrid = 4096;  // workgroups of a plan's count and write passes

// Shape of a work unit for a table of BUILD rows: threads, waves, S piece rows,
// bucket-count limit (as many buckets as keys in a table filled to half its
// rows: 2048 for 4096 rows, whose 32 KB of LDS then let four workgroups share a
// compute unit; 4096 for 8192 rows; 8192 for 16384) and probe rounds in flight
// per lane (the larger shapes have at most 128 registers per lane).
template <uint32_t BUILD>
struct Geo {
    static constexpr uint32_t kBuild = BUILD;
    static constexpr int kThreads = (int)(BUILD / 16);
    static constexpr int kWv = kThreads / kWave;
    static constexpr uint32_t kSPiece = 2 * BUILD;
    static constexpr int kMaxLog2nb = BUILD >= 16384 ? 13 : (BUILD == 4096 ? 11 : 12);
    static constexpr uint32_t kMaxNb = 1u << kMaxLog2nb;
    static constexpr int kPB = BUILD == 16384 ? 8 : 16;  // count pass
    static constexpr int kPBWrite = BUILD == 4096 ? 16 : 8;  // LDS write pass
    // waves per SIMD the register allocation must allow: the persistent
    // kernels and the one-unit-per-workgroup kernels (two 512-thread
    // workgroups per compute unit)
    static constexpr int kMinW = 4;
    static constexpr int kMinWWrite = BUILD == 4096 ? 3 : 4;
    static constexpr int kMinWEager = BUILD == 4096 ? 1 : 4;
    // the eager count pass: two 1024-thread workgroups per compute unit when their
    // LDS (sized by the largest R block) fits twice
    static constexpr int kMinWCount = BUILD == 16384 ? 8 : kMinWEager;
    static constexpr int kMinWStaged = BUILD == 4096 ? 2 : 4;
};

struct JoinArgs {
    const void *rkey;
    const void *skey;
    const uint32_t *rpo;
    const uint32_t *spo;
    uint32_t np;
    const uint32_t *ubase;  // exclusive prefix of units per partition
    uint32_t rc;            // R rows per build block (at most the table rows)
    int skip_bits;          // partition bits, excluded from the bucket hash
    uint64_t *wcnt;         // count pass: matches per (unit, wave)
    const uint64_t *woff;   // write pass: output offset per (unit, wave)
    uint64_t t_rows;        // write pass: output rows; every store is checked against it
    void *tkey;
    int nr, ns;
    const void *rp[8];
    int rw[8];
    void *tr[8];
    const void *sp[8];
    int sw[8];
    void *ts[8];
    const int32_t *rrow;  // GFUR: partitioned row ids of R
    const int32_t *srow;  // GFUR: partitioned row ids of S
    const uint8_t *seg_bits;  // batches: partition bits of instance p >> 8 (skip_bits unused)
    const uint8_t *seg_bshift;  // batches: extra LDS bucket bits of instance p >> 8 (else bshift)
    int bshift;                 // LDS buckets = 2^(ceil(log2 rows) + bshift), within the table's limit
    const uint32_t *nunits;     // device: work units (the kernels loop over them)
    const uint32_t *umap;       // partition of every unit (written by k_unit_map)
    uint32_t lds_rows;          // count and LDS write passes: rows of the largest R block
    uint32_t cap_units;         // units beyond this are not processed (a plan's capacity)
    const uint64_t *out_base;   // device: first output row of this call (nullptr = 0)
    // Streaming write path: the count pass records each S row's match (its row
    // in the R block, or kNoMatch), used when every partition has one R block
    // and no S row matches twice; flags[0] / flags[1] mark the contrary.
    uint16_t *midx;
    uint32_t *flags;            // [2]: most R rows in one partition (for LDS staging)
    int lds_if_complex;         // LDS write pass: do nothing unless a flag is set (plans)
    uint32_t rlds_off[8];       // staged streaming pass: byte offset of R column j in LDS
};

// Most work units one call may have: unit indices and their scanned offsets
// are 32-bit.
constexpr uint64_t kMaxUnits = 0x7FFFFFFFull;

// Units per partition pair. flags[0]: a partition spans several R blocks;
// flags[2]: most R rows in a partition that S rows probe; flags[3]: the units
// exceed kMaxUnits (their 64-bit total accumulates at flags + 4), and then no
// pass processes any unit, so a wrapped 32-bit scan is never read.
__global__ void k_unit_count(const uint32_t *__restrict__ rpo, const uint32_t *__restrict__ spo,
                             uint32_t np, uint32_t rc, uint32_t spiece, uint32_t *__restrict__ ucnt,
                             uint32_t *__restrict__ flags) {
    unsigned long long *total = reinterpret_cast<unsigned long long *>(flags + 4);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
        const uint32_t nr = rpo[p + 1] - rpo[p], ns = spo[p + 1] - spo[p];
        const uint64_t units = (nr && ns) ? (uint64_t)ceil_div_u32(nr, rc) * ceil_div_u32(ns, spiece) : 0ull;
        ucnt[p] = (uint32_t)min<uint64_t>(units, kMaxUnits);
        if (units) {
            const unsigned long long before = atomicAdd(total, (unsigned long long)units);
            if (before + units > kMaxUnits) atomicOr(&flags[3], 1u);
        }
        if (nr > rc && ns) atomicOr(&flags[0], 1u);  // a partition spans several R blocks
        if (ns) atomicMax(&flags[2], nr);
    }
}

// Units the passes process: none once the count overflowed, else at most the
// launch's (or plan's) capacity.
__device__ __forceinline__ uint32_t units_to_run(const uint32_t *nunits, const uint32_t *flags, uint32_t cap) {
    return flags[3] ? 0u : min(*nunits, cap);
}

// The partition of every unit to run, found once for all passes: each pass then
// reads it with one load, where a binary search over the unit offsets made a
// workgroup wait on 14 dependent loads per unit at 2^14 partitions.
__global__ void k_unit_map(const uint32_t *__restrict__ ubase, uint32_t np, const uint32_t *__restrict__ nunits,
                           const uint32_t *__restrict__ flags, uint32_t cap, uint32_t *__restrict__ umap) {
    const uint32_t n = units_to_run(nunits, flags, cap);
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = np;  // ubase[lo] <= u < ubase[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ubase[mid] <= u) lo = mid;
            else hi = mid;
        }
        umap[u] = lo;
    }
}

__device__ __forceinline__ void copy_val(void *dst, int dw, uint64_t di, const void *src, uint64_t si) {
    if (dw == 4) static_cast<uint32_t *>(dst)[di] = static_cast<const uint32_t *>(src)[si];
    else static_cast<uint64_t *>(dst)[di] = static_cast<const uint64_t *>(src)[si];
}

// Copies column values src[j][row[r]] to dst[j][pos[r]] for the PB rounds of a
// wave whose flag c[r] is set; all loads of one column are issued before its
// stores, so PB loads per lane are in flight.
template <int PB>
__device__ __forceinline__ void gather_cols(int ncols, const void *const *src, const int *width,
                                            void *const *dst, const uint32_t *row, const uint32_t *c,
                                            const uint64_t *pos, uint64_t t_rows) {
    for (int j = 0; j < ncols; ++j) {
        if (width[j] == 4) {
            const uint32_t *__restrict__ in = static_cast<const uint32_t *>(src[j]);
            uint32_t *__restrict__ out = static_cast<uint32_t *>(dst[j]);
            uint32_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = c[r] ? in[row[r]] : 0u;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (c[r] && pos[r] < t_rows) out[pos[r]] = v[r];
        } else {
            const uint64_t *__restrict__ in = static_cast<const uint64_t *>(src[j]);
            uint64_t *__restrict__ out = static_cast<uint64_t *>(dst[j]);
            uint64_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = c[r] ? in[row[r]] : 0ull;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (c[r] && pos[r] < t_rows) out[pos[r]] = v[r];
        }
    }
}

// Column moves of the streaming passes. Rows whose lrow[r] is ~0 have no match;
// output row = wbase + pos[r] (a 32-bit offset within the wave's range), dropped
// unless pos[r] < lim. gather_cols_wave reads src[j][rbase + row[r]];
// stream_cols_contig reads the contiguous rows row0 + r * 64 (one base address).
template <int PB>
__device__ __forceinline__ void gather_cols_wave(int ncols, const void *const *src, const int *width,
                                                 void *const *dst, uint32_t rbase,
                                                 const uint32_t *row, const uint32_t *lrow, const uint32_t *pos,
                                                 uint64_t wbase, uint32_t lim) {
    for (int j = 0; j < ncols; ++j) {
        if (width[j] == 4) {
            const uint32_t *__restrict__ in = static_cast<const uint32_t *>(src[j]) + rbase;
            uint32_t *__restrict__ out = static_cast<uint32_t *>(dst[j]) + wbase;
            uint32_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[row[r]] : 0u;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
        } else {
            const uint64_t *__restrict__ in = static_cast<const uint64_t *>(src[j]) + rbase;
            uint64_t *__restrict__ out = static_cast<uint64_t *>(dst[j]) + wbase;
            uint64_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[row[r]] : 0ull;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
        }
    }
}

template <int PB>
__device__ __forceinline__ void stream_cols_contig(int ncols, const void *const *src, const int *width,
                                                   void *const *dst, uint32_t row0, const uint32_t *lrow,
                                                   const uint32_t *pos, uint64_t wbase, uint32_t lim) {
    for (int j = 0; j < ncols; ++j) {
        if (width[j] == 4) {
            const uint32_t *__restrict__ in = static_cast<const uint32_t *>(src[j]) + row0;
            uint32_t *__restrict__ out = static_cast<uint32_t *>(dst[j]) + wbase;
            uint32_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[r * kWave] : 0u;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
        } else {
            const uint64_t *__restrict__ in = static_cast<const uint64_t *>(src[j]) + row0;
            uint64_t *__restrict__ out = static_cast<uint64_t *>(dst[j]) + wbase;
            uint64_t v[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[r * kWave] : 0ull;
#pragma unroll
            for (int r = 0; r < PB; ++r)
                if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
        }
    }
}

// LDS of a count or LDS-write unit, carved from dynamic shared memory for R
// blocks of at most `rows` rows (the largest block the call has, known after the
// unit count): the block's keys and rows, the bucket bounds (16-bit: a block
// holds at most 16384 rows) and a few words of workgroup state. Blocks of about
// 8192 rows then take 64-68 KB, and two 1024-thread workgroups share a compute
// unit, one building or loading while the other probes.
template <typename K>
struct JoinLds {
    K *rkey;         // R block keys: input order while building, bucket order after
    uint16_t *entry; // R block rows, grouped by bucket
    uint16_t *b;     // bucket boundaries
    uint32_t *tmp;   // kWv words
    uint32_t *unit;  // 6 words
    int *is_long;
};
constexpr size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }
template <typename K, uint32_t BUILD>
constexpr size_t join_lds_bytes(uint32_t rows) {
    return align8((size_t)rows * sizeof(K)) + align8((size_t)rows * 2) + align8(((size_t)Geo<BUILD>::kMaxNb + 1) * 2) +
           4 * ((size_t)Geo<BUILD>::kWv + 8);
}
template <typename K, uint32_t BUILD>
__device__ __forceinline__ JoinLds<K> join_lds(uint8_t *p, uint32_t rows) {
    JoinLds<K> L;
    L.rkey = reinterpret_cast<K *>(p);
    p += align8((size_t)rows * sizeof(K));
    L.entry = reinterpret_cast<uint16_t *>(p);
    p += align8((size_t)rows * 2);
    L.b = reinterpret_cast<uint16_t *>(p);
    p += align8(((size_t)Geo<BUILD>::kMaxNb + 1) * 2);
    L.tmp = reinterpret_cast<uint32_t *>(p);
    L.unit = L.tmp + Geo<BUILD>::kWv;
    L.is_long = reinterpret_cast<int *>(L.unit + 6);
    return L;
}
// 16-bit bucket counters updated through their 32-bit word (no carry or borrow
// crosses the halves: counts stay below 2^16 and never drop below zero).
__device__ __forceinline__ void b16_add1(uint16_t *b, uint32_t i) {
    atomicAdd(reinterpret_cast<uint32_t *>(b) + (i >> 1), 1u << ((i & 1u) * 16u));
}
__device__ __forceinline__ uint32_t b16_dec(uint16_t *b, uint32_t i) {  // the value before
    const uint32_t sh = (i & 1u) * 16u;
    return (atomicSub(reinterpret_cast<uint32_t *>(b) + (i >> 1), 1u << sh) >> sh) & 0xFFFFu;
}

// Build on the R block of unit u and probe it with the unit's S piece: count
// (WRITE = false) or write (WRITE = true) the matches.
// Probes of PB keys against the LDS table, shaped so that the PB lookups are
// independent: bucket bounds, then the first entry of every chain, read for all
// rows at once (clamped indices, so every read is in range); chains longer than
// one entry, rare with at least as many buckets as rows, are walked afterwards.
// c[r] = matches of key r, e1[r] = its first match's entry (bucket order).
template <typename K, int PB>
__device__ __forceinline__ void probe_rows(const K *s_rkey, const uint16_t *s_b, const K (&key)[PB],
                                           const bool (&valid)[PB], int skip_bits, int log2nb, uint32_t rn,
                                           uint32_t (&c)[PB], uint32_t (&e1)[PB]) {
    uint32_t lo[PB], hi[PB];
#pragma unroll
    for (int r = 0; r < PB; ++r) {
        const uint32_t b = bucket_of<K>(key[r], skip_bits, log2nb);
        lo[r] = s_b[b];
        hi[r] = valid[r] ? s_b[b + 1] : lo[r];
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {
        const K k0 = s_rkey[min(lo[r], rn - 1)];
        c[r] = (lo[r] < hi[r] && k0 == key[r]) ? 1u : 0u;
        e1[r] = lo[r];
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {
        for (uint32_t e = lo[r] + 1; e < hi[r]; ++e) {
            if (s_rkey[e] == key[r]) {
                if (c[r] == 0) e1[r] = e;
                ++c[r];
            }
        }
    }
}

// Unit u of the (R block) x (S piece) decomposition: s_unit[0..5] = first R
// row, R rows, first S row, S rows, partition bits, extra bucket bits.
template <uint32_t kSPiece>
__device__ __forceinline__ void decode_unit(const JoinArgs &a, uint32_t u, uint32_t *s_unit) {
    const uint32_t p = a.umap[u];
    const uint32_t nr = a.rpo[p + 1] - a.rpo[p], ns = a.spo[p + 1] - a.spo[p];
    const uint32_t nsb = ceil_div_u32(ns, kSPiece);
    const uint32_t local = u - a.ubase[p];
    const uint32_t ra = local / nsb, sb = local % nsb;
    s_unit[0] = a.rpo[p] + ra * a.rc;
    s_unit[1] = min(a.rc, nr - ra * a.rc);
    s_unit[2] = a.spo[p] + sb * kSPiece;
    s_unit[3] = min(kSPiece, ns - sb * kSPiece);
    s_unit[4] = a.seg_bits ? a.seg_bits[p >> 8] : (uint32_t)a.skip_bits;
    s_unit[5] = a.seg_bshift ? a.seg_bshift[p >> 8] : (uint32_t)a.bshift;
}

// Inclusive scan of the nb bucket counts in s_b (s_b[b] = end of bucket b), and
// s_b[nb] = rn.
template <uint32_t BUILD>
__device__ __forceinline__ void scan_buckets(uint16_t *s_b, uint32_t *s_tmp, uint32_t nb, uint32_t rn) {
    using G = Geo<BUILD>;
    constexpr int per = (int)((G::kMaxNb + G::kThreads - 1) / G::kThreads);
    const uint32_t first = threadIdx.x * per;
    uint32_t v[per];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = (first + k < nb) ? s_b[first + k] : 0u;
        sum += v[k];
    }
    uint32_t run = block_exclusive_sum<uint32_t, G::kWv>(sum, s_tmp, (uint32_t *)nullptr);
#pragma unroll
    for (int k = 0; k < per; ++k) {
        run += v[k];
        if (first + k < nb) s_b[first + k] = (uint16_t)run;
    }
    if (threadIdx.x == 0) s_b[nb] = (uint16_t)rn;
}

// Count pass of unit u: matches per (unit, wave), each S row's match recorded
// for the streaming write pass, and the flag for S rows with several matches.
// The table is built straight into bucket order from registers (the R keys of
// this thread: counts, scan, placement), since counts need no ordered chains;
// the wave's first round of S keys loads during the build.
template <typename K, uint32_t BUILD>
__device__ __forceinline__ void count_unit(const JoinArgs &a, uint32_t u, const JoinLds<K> &sh) {
    using G = Geo<BUILD>;
    constexpr int PB = G::kPB;
    constexpr int kT = G::kThreads;
    constexpr int kWv = G::kWv;
    constexpr int PER = (int)(BUILD / kT);
    K *s_rkey = sh.rkey;
    uint16_t *s_b = sh.b;
    uint16_t *s_entry = sh.entry;
    uint32_t *s_unit = sh.unit;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    if (tid == 0) decode_unit<G::kSPiece>(a, u, s_unit);
    __syncthreads();
    // the unit's shape is uniform: scalar registers (in vector ones they spilled)
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(s_unit[0]), rn = __builtin_amdgcn_readfirstlane(s_unit[1]);
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(s_unit[2]), sn = __builtin_amdgcn_readfirstlane(s_unit[3]);
    const int skip_bits = (int)__builtin_amdgcn_readfirstlane(s_unit[4]);
    int log2nb = 0;
    while ((1u << log2nb) < rn) ++log2nb;
    log2nb = min(log2nb + (int)__builtin_amdgcn_readfirstlane(s_unit[5]), G::kMaxLog2nb);
    const uint32_t nb = 1u << log2nb;

    // loads in flight during the build: this thread's R keys, its wave's first S keys
    const K *__restrict__ rk = static_cast<const K *>(a.rkey) + r0;
    K kr[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) kr[k] = (uint32_t)(tid + k * kT) < rn ? rk[tid + k * kT] : K(0);
    const uint32_t q = ceil_div_u32(sn, kWv);
    const uint32_t ws = __builtin_amdgcn_readfirstlane(min(sn, w * q)), we = __builtin_amdgcn_readfirstlane(min(sn, ws + q));
    const K *__restrict__ skey = static_cast<const K *>(a.skey) + s0;
    K key[PB];
#pragma unroll
    for (int r = 0; r < PB; ++r) key[r] = ws + r * kWave + lane < we ? skey[ws + r * kWave + lane] : K(0);

    for (uint32_t b = tid; b <= nb; b += kT) s_b[b] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if ((uint32_t)(tid + k * kT) < rn) b16_add1(s_b, bucket_of<K>(kr[k], skip_bits, log2nb));
    __syncthreads();
    scan_buckets<BUILD>(s_b, sh.tmp, nb, rn);
    __syncthreads();
    // placement from the end of each bucket; afterwards s_b[b] = start of bucket b
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if ((uint32_t)(tid + k * kT) < rn) {
            const uint32_t slot = b16_dec(s_b, bucket_of<K>(kr[k], skip_bits, log2nb)) - 1u;
            s_rkey[slot] = kr[k];
            s_entry[slot] = (uint16_t)(tid + k * kT);
        }
    }
    __syncthreads();

    uint32_t cnt = 0;
    bool multi = false;
    for (uint32_t base = ws; base < we; base += PB * kWave) {
        if (base != ws) {
#pragma unroll
            for (int r = 0; r < PB; ++r) key[r] = base + r * kWave + lane < we ? skey[base + r * kWave + lane] : K(0);
        }
        bool valid[PB];
#pragma unroll
        for (int r = 0; r < PB; ++r) valid[r] = base + r * kWave + lane < we;
        uint32_t c[PB], e1[PB];
        probe_rows<K, PB>(s_rkey, s_b, key, valid, skip_bits, log2nb, rn, c, e1);
#pragma unroll
        for (int r = 0; r < PB; ++r) {
            if (valid[r]) {
                cnt += c[r];
                multi |= c[r] > 1;
                if (a.midx) a.midx[s0 + base + r * kWave + lane] = c[r] ? s_entry[e1[r]] : kNoMatch;
            }
        }
    }
    const uint64_t tot = wave_sum<uint64_t>((uint64_t)cnt);
    if (lane == 0) a.wcnt[(uint64_t)u * kWv + w] = tot;
    if (a.flags && __ballot(multi) && lane == 0) atomicOr(&a.flags[1], 1u);
}

// Write pass of unit u on the LDS table (the general case: partitions spanning
// several R blocks, or S rows with several matches): build with chains in row
// order, probe, and write every match at the positions the count pass sized.
template <typename K, uint32_t BUILD>
__device__ __forceinline__ void write_unit(const JoinArgs &a, uint32_t u, uint64_t out_base, const JoinLds<K> &sh) {
    using G = Geo<BUILD>;
    constexpr int PB = G::kPBWrite;
    constexpr int kBlockT = G::kThreads;
    constexpr int kWv = G::kWv;
    constexpr uint32_t kSPiece = G::kSPiece;
    K *s_rkey = sh.rkey;
    uint16_t *s_b = sh.b;
    uint16_t *s_entry = sh.entry;
    uint32_t *s_unit = sh.unit;
    int &s_long = *sh.is_long;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    if (tid == 0) {
        decode_unit<kSPiece>(a, u, s_unit);
        s_long = 0;
    }
    __syncthreads();
    const uint32_t r0 = s_unit[0], rn = s_unit[1], s0 = s_unit[2], sn = s_unit[3];
    const int skip_bits = (int)s_unit[4];
    int log2nb = 0;
    while ((1u << log2nb) < rn) ++log2nb;
    log2nb = min(log2nb + (int)s_unit[5], G::kMaxLog2nb);
    const uint32_t nb = 1u << log2nb;

    // ---- build: bucket counts, scan, placement, per-bucket order by row ----
    const K *__restrict__ rkey = static_cast<const K *>(a.rkey);
    for (uint32_t i = tid; i < rn; i += kBlockT) s_rkey[i] = rkey[r0 + i];
    for (uint32_t b = tid; b <= nb; b += kBlockT) s_b[b] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < rn; i += kBlockT) b16_add1(s_b, bucket_of<K>(s_rkey[i], skip_bits, log2nb));
    __syncthreads();
    scan_buckets<BUILD>(s_b, sh.tmp, nb, rn);
    __syncthreads();
    // placement from the end of each bucket; afterwards s_b[b] = start of bucket b
    for (uint32_t i = tid; i < rn; i += kBlockT) {
        const uint32_t slot = b16_dec(s_b, bucket_of<K>(s_rkey[i], skip_bits, log2nb)) - 1u;
        s_entry[slot] = (uint16_t)i;
    }
    __syncthreads();
    // chains in row order, so that every S row emits its matches in R's input order
    for (uint32_t b = tid; b < nb; b += kBlockT) {
        const uint32_t lo = s_b[b], hi = s_b[b + 1];
        if (hi - lo > kMaxChainSort) {
            s_long = 1;
        } else {
            for (uint32_t x = lo + 1; x < hi; ++x) {
                const uint16_t e = s_entry[x];
                uint32_t y = x;
                while (y > lo && s_entry[y - 1] > e) {
                    s_entry[y] = s_entry[y - 1];
                    --y;
                }
                s_entry[y] = e;
            }
        }
    }
    __syncthreads();
    if (s_long) {
        // Rare (heavy duplicate keys): one wave places all rows again in row
        // order, ranking equal buckets within a round by ballot.
        if (w == 0) {
            for (uint32_t base = 0; base < rn; base += kWave) {
                const uint32_t i = base + lane;
                const bool valid = i < rn;
                const uint32_t b = valid ? bucket_of<K>(s_rkey[i], skip_bits, log2nb) : 0u;
                const uint64_t peers = match_peers(b, log2nb, valid);
                if (valid) {
                    const uint32_t rk = rank_below(peers);
                    const uint32_t st = s_b[b];
                    if (rk == 0) s_b[b] = (uint16_t)(st + (uint32_t)__popcll(peers));
                    s_entry[st + rk] = (uint16_t)i;
                }
            }
            // s_b[b] now holds the end of bucket b: shift right by one, top down
            for (int c = (int)((nb + kWave - 1) / kWave) - 1; c >= 0; --c) {
                const uint32_t b = (uint32_t)c * kWave + lane;
                const uint32_t v = b < nb ? s_b[b] : 0u;
                if (b < nb) s_b[b + 1] = (uint16_t)v;
            }
            if (lane == 0) s_b[0] = 0;
        }
        __syncthreads();
    }
    {
        // keys in bucket order (s_rkey[e] = key of entry e), so that a probe
        // compares keys without going through the row index
        constexpr int per = (int)(BUILD / kBlockT);
        K t[per];
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const uint32_t e = tid + k * kBlockT;
            t[k] = e < rn ? s_rkey[s_entry[e]] : K(0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const uint32_t e = tid + k * kBlockT;
            if (e < rn) s_rkey[e] = t[k];
        }
        __syncthreads();
    }

    // ---- probe: each wave streams a contiguous share of the S piece, PB
    // rounds of 64 rows at a time so that many loads are in flight ----
    const K *__restrict__ skey = static_cast<const K *>(a.skey);
    const uint32_t q = ceil_div_u32(sn, kWv);
    const uint32_t ws = min(sn, w * q), we = min(sn, ws + q);
    {
        uint64_t outpos = out_base + a.woff[(uint64_t)u * kWv + w];
        K *__restrict__ tkey = static_cast<K *>(a.tkey);
        for (uint32_t base = ws; base < we; base += PB * kWave) {
            K key[PB];
            uint32_t c[PB], e1[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) {
                const uint32_t i = base + r * kWave + lane;
                key[r] = i < we ? skey[s0 + i] : K(0);
            }
            bool valid[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) valid[r] = base + r * kWave + lane < we;
            probe_rows<K, PB>(s_rkey, s_b, key, valid, skip_bits, log2nb, rn, c, e1);
#pragma unroll
            for (int r = 0; r < PB; ++r) e1[r] = c[r] ? (uint32_t)s_entry[e1[r]] : 0u;
            uint64_t pos[PB];
            bool multi = false;
#pragma unroll
            for (int r = 0; r < PB; ++r) {
                const uint32_t incl = wave_inclusive_sum<uint32_t>(c[r]);
                pos[r] = outpos + incl - c[r];
                outpos += __shfl(incl, kWave - 1, kWave);
                multi |= __ballot(c[r] > 1) != 0ull;
            }
            if (!multi) {
                // at most one match per S row: every output row is (S row, its R row)
#pragma unroll
                for (int r = 0; r < PB; ++r)
                    if (c[r] && pos[r] < a.t_rows) tkey[pos[r]] = key[r];
                uint32_t srow[PB], rrow[PB];
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    const uint32_t i = base + r * kWave + lane;
                    srow[r] = s0 + i;
                    rrow[r] = r0 + e1[r];
                    if (a.srow && c[r]) srow[r] = (uint32_t)a.srow[srow[r]];
                    if (a.rrow && c[r]) rrow[r] = (uint32_t)a.rrow[rrow[r]];
                }
                gather_cols<PB>(a.ns, a.sp, a.sw, a.ts, srow, c, pos, a.t_rows);
                gather_cols<PB>(a.nr, a.rp, a.rw, a.tr, rrow, c, pos, a.t_rows);
            } else {
                // several matches for some row: enumerate the chain per lane
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    if (!c[r]) continue;
                    const uint32_t i = base + r * kWave + lane;
                    uint64_t p = pos[r];
                    const uint64_t sr = a.srow ? (uint64_t)a.srow[s0 + i] : (uint64_t)(s0 + i);
                    const uint32_t b = bucket_of<K>(key[r], skip_bits, log2nb);
                    for (uint32_t e = s_b[b], end = s_b[b + 1]; e < end; ++e) {
                        if (s_rkey[e] != key[r] || p >= a.t_rows) continue;
                        const uint32_t ri = s_entry[e];
                        const uint64_t rr = a.rrow ? (uint64_t)a.rrow[r0 + ri] : (uint64_t)(r0 + ri);
                        tkey[p] = key[r];
                        for (int j = 0; j < a.nr; ++j) copy_val(a.tr[j], a.rw[j], p, a.rp[j], rr);
                        for (int j = 0; j < a.ns; ++j) copy_val(a.ts[j], a.sw[j], p, a.sp[j], sr);
                        ++p;
                    }
                }
            }
        }
    }
}

template <typename K, uint32_t BUILD, bool WRITE>
__device__ __forceinline__ void join_unit(const JoinArgs &a, uint32_t u, uint64_t out_base, const JoinLds<K> &sh) {
    if constexpr (WRITE) write_unit<K, BUILD>(a, u, out_base, sh);
    else count_unit<K, BUILD>(a, u, sh);
}

// One work unit per workgroup (eager calls: the grid is the unit count).
template <typename K, uint32_t BUILD, bool WRITE>
__global__ __launch_bounds__(Geo<BUILD>::kThreads, WRITE ? Geo<BUILD>::kMinWEager : Geo<BUILD>::kMinWCount) void k_join(JoinArgs a) {
    extern __shared__ uint4 s_dyn4[];
    const JoinLds<K> sh = join_lds<K, BUILD>(reinterpret_cast<uint8_t *>(s_dyn4), a.lds_rows);
    if (blockIdx.x < units_to_run(a.nunits, a.flags, a.cap_units)) join_unit<K, BUILD, WRITE>(a, blockIdx.x, 0ull, sh);
}

// Write pass without a hash table, for the common case recorded by the count
// pass (one R block per partition, at most one match per S row): each wave
// streams its S rows with their recorded matches, takes output positions from
// the scanned counts plus a ballot prefix, and gathers the payloads (GFTR:
// partition-local R rows; GFUR: original rows through the row ids). It needs no
// LDS, so it always runs 256-thread workgroups whose waves take the count
// pass's (unit, wave) slots one by one, whatever the table shape.
template <typename K, uint32_t BUILD, bool GFUR>
__global__ __launch_bounds__(kBlock, GFUR ? 4 : 1) void k_join_stream(JoinArgs a) {
    using G = Geo<BUILD>;
    constexpr int PB = 16;
    constexpr int kWv = G::kWv;
    constexpr uint32_t kSPiece = G::kSPiece;
    if (a.flags[0] | a.flags[1]) return;  // the LDS write pass handles this input
    const int lane = lane_id();
    const uint32_t n_units = units_to_run(a.nunits, a.flags, a.cap_units);
    const uint64_t n_slots = (uint64_t)n_units * kWv;
    const uint64_t out_base = a.out_base ? *a.out_base : 0ull;
    const K *__restrict__ skey = static_cast<const K *>(a.skey);
    K *__restrict__ tkey = static_cast<K *>(a.tkey);
    for (uint64_t slot = (uint64_t)blockIdx.x * kWaves + threadIdx.x / kWave; slot < n_slots;
         slot += (uint64_t)gridDim.x * kWaves) {
        const uint32_t u = (uint32_t)(slot / kWv), w = (uint32_t)(slot % kWv);
        const uint32_t p = a.umap[u], sb = u - a.ubase[p];  // one R block: the unit is the S piece
        const uint32_t ns = a.spo[p + 1] - a.spo[p];
        const uint32_t s0 = a.spo[p] + sb * kSPiece, sn = min(kSPiece, ns - sb * kSPiece);
        const uint32_t r0 = a.rpo[p], rn = a.rpo[p + 1] - r0;
        const uint32_t q = ceil_div_u32(sn, kWv);
        const uint32_t ws = min(sn, w * q), we = min(sn, ws + q);
        // output rows of this wave: wbase + a 32-bit offset (a wave writes at most q rows)
        const uint64_t wbase = out_base + a.woff[slot];
        const uint32_t lim = a.t_rows > wbase ? (uint32_t)min<uint64_t>(a.t_rows - wbase, 0xFFFFFFFFull) : 0u;
        uint32_t off = 0;
        for (uint32_t base = ws; base < we; base += PB * kWave) {
            // lrow[r]: the match's row in the R block, or ~0 (none; a recorded row
            // past the block is impossible when the count pass ran on this input)
            uint32_t lrow[PB], pos[PB];
            {
                uint32_t m[PB];
                K key[PB];
                const uint16_t *__restrict__ mp = a.midx + (s0 + base + lane);
                const K *__restrict__ kp = skey + (s0 + base + lane);
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    const bool in = base + r * kWave + lane < we;
                    m[r] = in ? mp[r * kWave] : kNoMatch;
                    key[r] = in ? kp[r * kWave] : K(0);
                }
                K *__restrict__ tk = tkey + wbase;
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    lrow[r] = m[r] < rn ? m[r] : ~0u;
                    const uint64_t hit = __ballot(lrow[r] != ~0u);
                    pos[r] = off + rank_below(hit);
                    off += (uint32_t)__popcll(hit);
                    if (lrow[r] != ~0u && pos[r] < lim) tk[pos[r]] = key[r];
                }
            }
            if constexpr (!GFUR) {
                // GFTR: S rows are contiguous, R rows partition-local
                stream_cols_contig<PB>(a.ns, a.sp, a.sw, a.ts, s0 + base + lane, lrow, pos, wbase, lim);
                gather_cols_wave<PB>(a.nr, a.rp, a.rw, a.tr, r0, lrow, lrow, pos, wbase, lim);
            } else {
                // GFUR: original rows through the row ids
                uint32_t row[PB];
#pragma unroll
                for (int r = 0; r < PB; ++r) row[r] = lrow[r] != ~0u ? (uint32_t)a.srow[s0 + base + r * kWave + lane] : 0u;
                gather_cols_wave<PB>(a.ns, a.sp, a.sw, a.ts, 0u, row, lrow, pos, wbase, lim);
#pragma unroll
                for (int r = 0; r < PB; ++r) row[r] = lrow[r] != ~0u ? (uint32_t)a.rrow[r0 + lrow[r]] : 0u;
                gather_cols_wave<PB>(a.nr, a.rp, a.rw, a.tr, 0u, row, lrow, pos, wbase, lim);
            }
        }
    }
}

// Streaming write pass with the R side staged in LDS (GFTR, one R block per
// partition, at most one match per S row): a workgroup takes one unit (an S
// piece of one partition), copies the partition's R payload columns into LDS
// with coalesced reads, and streams the S piece as k_join_stream does, reading
// R values from LDS. Every R payload value then crosses HBM once per S piece,
// where the gathers of k_join_stream re-read lines that L2 has dropped when a
// compute unit's partitions outgrow its share of L2. A unit whose S piece has
// fewer rows than its R block (cold partitions under skew) gathers from HBM
// instead, since staging would move more bytes than it saves. Launched when
// the largest partition's R payload fits the dynamic LDS.
template <typename K, uint32_t BUILD>
__global__ __launch_bounds__(Geo<BUILD>::kThreads, Geo<BUILD>::kMinWStaged) void k_join_stream_staged(JoinArgs a) {
    using G = Geo<BUILD>;
    constexpr int PB = 16;
    constexpr int kWv = G::kWv;
    constexpr int kT = G::kThreads;
    constexpr uint32_t kSPiece = G::kSPiece;
    extern __shared__ uint4 s_dyn4[];
    uint8_t *s_dyn = reinterpret_cast<uint8_t *>(s_dyn4);
    __shared__ uint32_t s_unit[4];
    if (a.flags[0] | a.flags[1]) return;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    const uint32_t n_units = units_to_run(a.nunits, a.flags, a.cap_units);
    const uint64_t out_base = a.out_base ? *a.out_base : 0ull;
    const K *__restrict__ skey = static_cast<const K *>(a.skey);
    K *__restrict__ tkey = static_cast<K *>(a.tkey);
    for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        if (tid == 0) {
            const uint32_t p = a.umap[u], sb = u - a.ubase[p];  // one R block: the unit is the S piece
            const uint32_t ns = a.spo[p + 1] - a.spo[p];
            s_unit[0] = a.rpo[p];
            s_unit[1] = min(a.rpo[p + 1] - a.rpo[p], a.flags[2]);  // never past the staged rows
            s_unit[2] = a.spo[p] + sb * kSPiece;
            s_unit[3] = min(kSPiece, ns - sb * kSPiece);
        }
        __syncthreads();
        const uint32_t r0 = s_unit[0], rn = s_unit[1], s0 = s_unit[2], sn = s_unit[3];
        const bool staged = sn >= rn;  // uniform over the workgroup
        for (int j = 0; j < a.nr && staged; ++j) {
            if (a.rw[j] == 4) {
                const uint32_t *__restrict__ in = static_cast<const uint32_t *>(a.rp[j]) + r0;
                uint32_t *d = reinterpret_cast<uint32_t *>(s_dyn + a.rlds_off[j]);
                for (uint32_t i = tid; i < rn; i += kT) d[i] = in[i];
            } else {
                const uint64_t *__restrict__ in = static_cast<const uint64_t *>(a.rp[j]) + r0;
                uint64_t *d = reinterpret_cast<uint64_t *>(s_dyn + a.rlds_off[j]);
                for (uint32_t i = tid; i < rn; i += kT) d[i] = in[i];
            }
        }
        __syncthreads();
        const uint32_t q = ceil_div_u32(sn, kWv);
        const uint32_t ws = min(sn, w * q), we = min(sn, ws + q);
        // output rows of this wave: wbase + a 32-bit offset (a wave writes at most q rows)
        const uint64_t wbase = out_base + a.woff[(uint64_t)u * kWv + w];
        const uint32_t lim = a.t_rows > wbase ? (uint32_t)min<uint64_t>(a.t_rows - wbase, 0xFFFFFFFFull) : 0u;
        uint32_t off = 0;
        for (uint32_t base = ws; base < we; base += PB * kWave) {
            // lrow[r]: LDS row of the match, or ~0 (no match, or a row past the
            // staged block, impossible when the count pass ran on the same input)
            uint32_t lrow[PB], pos[PB];
            {
                uint32_t m[PB];
                K key[PB];
                const uint16_t *__restrict__ mp = a.midx + (s0 + base + lane);
                const K *__restrict__ kp = skey + (s0 + base + lane);
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    const bool in = base + r * kWave + lane < we;
                    m[r] = in ? mp[r * kWave] : kNoMatch;
                    key[r] = in ? kp[r * kWave] : K(0);
                }
                K *__restrict__ tk = tkey + wbase;
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    lrow[r] = m[r] < rn ? m[r] : ~0u;
                    const uint64_t hit = __ballot(lrow[r] != ~0u);
                    pos[r] = off + rank_below(hit);
                    off += (uint32_t)__popcll(hit);
                    if (lrow[r] != ~0u && pos[r] < lim) tk[pos[r]] = key[r];
                }
            }
            // S payloads: contiguous partitioned rows, one base address per column
            for (int j = 0; j < a.ns; ++j) {
                if (a.sw[j] == 4) {
                    const uint32_t *__restrict__ in = static_cast<const uint32_t *>(a.sp[j]) + (s0 + base + lane);
                    uint32_t *__restrict__ out = static_cast<uint32_t *>(a.ts[j]) + wbase;
                    uint32_t v[PB];
#pragma unroll
                    for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[r * kWave] : 0u;
#pragma unroll
                    for (int r = 0; r < PB; ++r)
                        if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
                } else {
                    const uint64_t *__restrict__ in = static_cast<const uint64_t *>(a.sp[j]) + (s0 + base + lane);
                    uint64_t *__restrict__ out = static_cast<uint64_t *>(a.ts[j]) + wbase;
                    uint64_t v[PB];
#pragma unroll
                    for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? in[r * kWave] : 0ull;
#pragma unroll
                    for (int r = 0; r < PB; ++r)
                        if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
                }
            }
            // R payloads from LDS, or from the partitioned column in HBM
            for (int j = 0; j < a.nr; ++j) {
                if (!staged) {
                    if (a.rw[j] == 4) {
                        const uint32_t *__restrict__ col = static_cast<const uint32_t *>(a.rp[j]) + r0;
                        uint32_t *__restrict__ out = static_cast<uint32_t *>(a.tr[j]) + wbase;
                        uint32_t v[PB];
#pragma unroll
                        for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? col[lrow[r]] : 0u;
#pragma unroll
                        for (int r = 0; r < PB; ++r)
                            if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
                    } else {
                        const uint64_t *__restrict__ col = static_cast<const uint64_t *>(a.rp[j]) + r0;
                        uint64_t *__restrict__ out = static_cast<uint64_t *>(a.tr[j]) + wbase;
                        uint64_t v[PB];
#pragma unroll
                        for (int r = 0; r < PB; ++r) v[r] = lrow[r] != ~0u ? col[lrow[r]] : 0ull;
#pragma unroll
                        for (int r = 0; r < PB; ++r)
                            if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = v[r];
                    }
                } else if (a.rw[j] == 4) {
                    const uint32_t *col = reinterpret_cast<const uint32_t *>(s_dyn + a.rlds_off[j]);
                    uint32_t *__restrict__ out = static_cast<uint32_t *>(a.tr[j]) + wbase;
#pragma unroll
                    for (int r = 0; r < PB; ++r)
                        if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = col[lrow[r]];
                } else {
                    const uint64_t *col = reinterpret_cast<const uint64_t *>(s_dyn + a.rlds_off[j]);
                    uint64_t *__restrict__ out = static_cast<uint64_t *>(a.tr[j]) + wbase;
#pragma unroll
                    for (int r = 0; r < PB; ++r)
                        if (lrow[r] != ~0u && pos[r] < lim) out[pos[r]] = col[lrow[r]];
                }
            }
        }
        __syncthreads();  // the next unit restages the LDS
    }
}

// Persistent workgroups over the unit count held in device memory (plans).
template <typename K, uint32_t BUILD, bool WRITE>
__global__ __launch_bounds__(Geo<BUILD>::kThreads, WRITE ? Geo<BUILD>::kMinWWrite : Geo<BUILD>::kMinW) void k_join_persist(JoinArgs a) {
    extern __shared__ uint4 s_dyn4[];
    const JoinLds<K> sh = join_lds<K, BUILD>(reinterpret_cast<uint8_t *>(s_dyn4), a.lds_rows);
    if (WRITE && a.lds_if_complex && !(a.flags[0] | a.flags[1])) return;  // the streaming pass writes
    const uint32_t n_units = units_to_run(a.nunits, a.flags, a.cap_units);
    const uint64_t out_base = a.out_base ? *a.out_base : 0ull;
    for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        join_unit<K, BUILD, WRITE>(a, u, out_base, sh);
        __syncthreads();  // the unit's LDS state is rebuilt by the next one
    }
}

// Output offset of each instance of a batch: the write offset of its first unit.
// Units past the processed count (a plan's capacity) contribute nothing.
__global__ void k_instance_offsets(const uint32_t *__restrict__ ubase, const uint64_t *__restrict__ woff,
                                   uint32_t waves_per_unit, uint32_t n_inst, const uint32_t *__restrict__ nunits,
                                   const uint32_t *__restrict__ flags, uint32_t cap_units,
                                   const uint64_t *__restrict__ total, const uint64_t *__restrict__ base,
                                   uint64_t *__restrict__ out) {
    const uint32_t nu = units_to_run(nunits, flags, cap_units);
    const uint64_t b = base ? *base : 0ull;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n_inst; i += gridDim.x * blockDim.x) {
        const uint32_t u = (i == n_inst) ? nu : min(ubase[i << 8], nu);
        out[i] = b + (u == nu ? *total : woff[(uint64_t)u * waves_per_unit]);
    }
}

// next = base + total (the first output row of a plan's next group), and the
// group's unit count for the plan's capacity check.
// An overflowed unit count reports the largest count, so that the plan's result
// flags the group as beyond its capacity.
__global__ void k_advance_base(const uint64_t *__restrict__ base, const uint64_t *__restrict__ total,
                               uint64_t *__restrict__ next, const uint32_t *__restrict__ nunits,
                               const uint32_t *__restrict__ flags, uint32_t *__restrict__ units_out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (next) *next = (base ? *base : 0ull) + *total;
        if (units_out) *units_out = flags[3] ? 0xFFFFFFFFu : *nunits;
    }
}

// The count and write kernels of one table shape.
template <typename K, uint32_t BUILD>
struct JoinKernels {
    using G = Geo<BUILD>;
    static void count(hipStream_t s, bool planned, uint32_t grid, const JoinArgs &a, double bytes) {
        const size_t shm = join_lds_bytes<K, BUILD>(a.lds_rows);
        if (planned) GJ_LAUNCH("k_join_count", bytes, (k_join_persist<K, BUILD, false>), dim3(grid), dim3(G::kThreads), shm, s, a);
        else GJ_LAUNCH("k_join_count", bytes, (k_join<K, BUILD, false>), dim3(grid), dim3(G::kThreads), shm, s, a);
    }
    // grid: workgroups of the unit passes; the streaming pass has kWaves-wave workgroups
    static void stream(hipStream_t s, uint32_t grid, const JoinArgs &a, double bytes) {
        grid = (uint32_t)std::min<uint64_t>((uint64_t)grid * G::kWv / kWaves, 1u << 30);
        if (a.srow) GJ_LAUNCH("k_join_write", bytes, (k_join_stream<K, BUILD, true>), dim3(grid), dim3(kBlock), 0, s, a);
        else GJ_LAUNCH("k_join_write", bytes, (k_join_stream<K, BUILD, false>), dim3(grid), dim3(kBlock), 0, s, a);
    }
    static void staged(hipStream_t s, uint32_t grid, size_t shm, const JoinArgs &a, double bytes) {
        GJ_LAUNCH("k_join_write", bytes, (k_join_stream_staged<K, BUILD>), dim3(grid), dim3(G::kThreads), shm, s, a);
    }
    static void write_lds(hipStream_t s, bool planned, uint32_t grid, const JoinArgs &a, double bytes) {
        const size_t shm = join_lds_bytes<K, BUILD>(a.lds_rows);
        if (planned) GJ_LAUNCH("k_join_write_lds", bytes, (k_join_persist<K, BUILD, true>), dim3(grid), dim3(G::kThreads), shm, s, a);
        else GJ_LAUNCH("k_join_write_lds", bytes, (k_join<K, BUILD, true>), dim3(grid), dim3(G::kThreads), shm, s, a);
    }
};

// Pass 0 = count, 1 = streaming write, 2 = LDS write, 3 = streaming write with
// the R side staged in shm bytes of LDS; the table shape holds r_block rows.
void launch_join_pass(int pass, int key_bytes, uint32_t table_rows, hipStream_t s, bool planned, uint32_t grid,
                      const JoinArgs &a, double bytes, size_t shm = 0) {
#define GJ_JP(K, B)                                                 \
    do {                                                            \
        if (pass == 0) JoinKernels<K, B>::count(s, planned, grid, a, bytes);     \
        else if (pass == 1) JoinKernels<K, B>::stream(s, grid, a, bytes);        \
        else if (pass == 3) JoinKernels<K, B>::staged(s, grid, shm, a, bytes);   \
        else JoinKernels<K, B>::write_lds(s, planned, grid, a, bytes);           \
    } while (0)
    if (key_bytes == 4) {
        if (table_rows == 4096) GJ_JP(int32_t, 4096);
        else if (table_rows == 8192) GJ_JP(int32_t, 8192);
        else GJ_JP(int32_t, 16384);
    } else {
        if (table_rows == 4096) GJ_JP(int64_t, 4096);
        else GJ_JP(int64_t, 8192);
    }
#undef GJ_JP
}

uint32_t waves_per_unit(uint32_t table_rows) { return table_rows / 16 / kWave; }

// Largest LDS the staged streaming pass may take (GJ_JOIN_STAGED_LDS overrides;
// 0 turns the staged pass off).
size_t staged_lds_limit() {
    static const size_t lim = [] {
        if (const char *e = getenv("GJ_JOIN_STAGED_LDS")) return (size_t)strtoull(e, nullptr, 10);
        return kJoinStagedLds;
    }();
    return lim;
}

}  // namespace

int64_t join_partitioned(Ctx &ctx, int key_bytes, const JoinSide &R, const JoinSide &S, int bits,
                         int r_block, bool gfur, JoinOut *out, const uint8_t *seg_bits, uint32_t n_inst,
                         uint64_t *inst_off, const JoinPlanned *pl, JoinStats *stats) {
    hipStream_t s = ctx.stream;
    require(r_block >= 64 && r_block <= join_max_r_block(key_bytes),
            key_bytes == 4 ? "R build block must be 64..16384 rows" : "R build block must be 64..8192 rows for 8-byte keys");
    const uint32_t table_rows = join_table_rows(r_block);
    const uint32_t wpu = waves_per_unit(table_rows);
    const uint32_t np = seg_bits ? (n_inst << 8) : (1u << bits);
    uint32_t *ucnt = ctx.scratch_n<uint32_t>(np + 1);
    uint32_t *flags = ctx.scratch_n<uint32_t>(6);  // [0..3] flags, [4..5] 64-bit unit total
    fill_u32(s, flags, 0u, 6);
    GJ_LAUNCH("k_unit_count", 20.0 * np, k_unit_count, dim3(std::min<uint32_t>((np + 255) / 256, 1024)),
              dim3(256), 0, s, R.poff, S.poff, np, (uint32_t)r_block, join_s_piece(r_block), ucnt, flags);
    scan_exclusive_u32(ctx, ucnt, ucnt, np, ucnt + np);
    // Eager calls read the unit count and size every launch exactly; a plan sizes
    // for its capacity and the kernels read the count from device memory.
    uint32_t cap_units, grid;
    uint32_t lds_rows = (uint32_t)r_block;  // rows of the largest R block a unit builds on
    if (pl) {
        cap_units = pl->cap_units;
        grid = std::max<uint32_t>(1, std::min<uint32_t>(cap_units, kPersistentGrid));
    } else {
        uint32_t hf[6];
        GJ_HIP(hipMemcpyAsync(&cap_units, ucnt + np, 4, hipMemcpyDeviceToHost, s));
        GJ_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
        GJ_HIP(hipStreamSynchronize(s));
        // hf[2]: most R rows in a partition that S probes (a block holds at most r_block)
        lds_rows = std::max<uint32_t>(64, (std::min<uint32_t>(hf[2], (uint32_t)r_block) + 63) & ~63u);
        if (hf[3]) throw Error(GJ_EOVERFLOW, "more than 2^31-1 join work units (R partitions far larger than the "
                                             "build block)");
        if (stats) {
            stats->max_r_rows = hf[2];
            stats->multi_block = hf[0] != 0;
            if (stats->check_spread && hf[2] > stats->spread_limit) return -1;
        }
        grid = cap_units;
        if (cap_units == 0) {
            if (inst_off) fill_u64(s, inst_off, 0ull, (uint64_t)n_inst + 1);
            return 0;
        }
    }

    JoinArgs a{};
    a.rkey = R.key;
    a.skey = S.key;
    a.rpo = R.poff;
    a.spo = S.poff;
    a.np = np;
    a.ubase = ucnt;
    a.rc = (uint32_t)r_block;
    a.lds_rows = lds_rows;
    a.skip_bits = (stats && stats->hashed_digits) ? 0 : bits;
    a.seg_bits = seg_bits;
    a.seg_bshift = pl ? pl->seg_bshift : nullptr;
    a.bshift = 0;
    a.nunits = ucnt + np;
    a.cap_units = cap_units;
    a.out_base = pl ? pl->out_base : nullptr;
    a.midx = ctx.scratch_n<uint16_t>(std::max<uint32_t>(S.rows, 1));
    a.flags = flags;
    a.lds_if_complex = pl ? 1 : 0;
    uint32_t *umap = ctx.scratch_n<uint32_t>(cap_units);
    GJ_LAUNCH("k_unit_map", 4.0 * cap_units, k_unit_map,
              dim3(std::max<uint32_t>(1, std::min<uint32_t>(ceil_div_u32(cap_units, 256), 1024))),
              dim3(256), 0, s, ucnt, np, ucnt + np, (const uint32_t *)flags, cap_units, umap);
    a.umap = umap;
    const uint64_t nw = (uint64_t)cap_units * wpu;
    uint64_t *wcnt = ctx.scratch_n<uint64_t>(nw + 1);
    uint64_t *total = pl ? pl->total : wcnt + nw;
    a.wcnt = wcnt;
    const double nrows_r = R.rows, nrows_s = S.rows;
    const double key_reads = (nrows_r + nrows_s) * key_bytes;
    launch_join_pass(0, key_bytes, table_rows, s, pl != nullptr, grid, a, key_reads);
    if (pl) scan_exclusive_u64_dev(ctx, wcnt, wcnt, nw, ucnt + np, wpu, total);
    else scan_exclusive_u64(ctx, wcnt, wcnt, nw, total);
    uint64_t T;
    bool complex = true;  // plans launch both write passes; each decides on the device
    uint32_t max_r_rows = 0;
    if (pl) {
        T = pl->out_cap;  // stores are checked against the capacity; the true count stays on the device
        *out = pl->out;
    } else {
        uint32_t hf[3];
        GJ_HIP(hipMemcpyAsync(&T, total, 8, hipMemcpyDeviceToHost, s));
        GJ_HIP(hipMemcpyAsync(hf, flags, 12, hipMemcpyDeviceToHost, s));
        GJ_HIP(hipStreamSynchronize(s));
        complex = (hf[0] | hf[1]) != 0;
        max_r_rows = hf[2];
    }
    if (inst_off)
        GJ_LAUNCH("k_instance_offsets", 16.0 * n_inst, k_instance_offsets,
                  dim3(std::min<uint32_t>(ceil_div_u32(n_inst + 1, 256), 1024)), dim3(256), 0, s, ucnt, wcnt, wpu,
                  n_inst, ucnt + np, (const uint32_t *)flags, cap_units, total, a.out_base, inst_off);
    if (pl && (pl->next_base || pl->units_out))
        GJ_LAUNCH("k_advance_base", 16.0, k_advance_base, dim3(1), dim3(64), 0, s, a.out_base, total, pl->next_base,
                  (const uint32_t *)(ucnt + np), (const uint32_t *)flags, pl->units_out);
    if (T == 0) return 0;

    if (!pl) {
        out->key = ctx.output(T * (uint64_t)key_bytes);
        for (int j = 0; j < R.n_pay; ++j) out->r[j] = ctx.output(T * (uint64_t)R.width[j]);
        for (int j = 0; j < S.n_pay; ++j) out->s[j] = ctx.output(T * (uint64_t)S.width[j]);
    }
    a.woff = wcnt;
    a.t_rows = T;
    a.tkey = out->key;
    a.nr = R.n_pay;
    a.ns = S.n_pay;
    for (int j = 0; j < R.n_pay; ++j) {
        a.rp[j] = R.pay[j];
        a.rw[j] = R.width[j];
        a.tr[j] = out->r[j];
    }
    for (int j = 0; j < S.n_pay; ++j) {
        a.sp[j] = S.pay[j];
        a.sw[j] = S.width[j];
        a.ts[j] = out->s[j];
    }
    a.rrow = gfur ? R.rowid : nullptr;
    a.srow = gfur ? S.rowid : nullptr;
    // algorithmic bytes: keys of both sides, payload reads (GFTR: each partitioned
    // row once; GFUR: one gathered value per output row and column, plus row ids),
    // and the output rows (a plan counts its expected rows, given by the caller)
    double rw_sum = 0, sw_sum = 0;
    for (int j = 0; j < R.n_pay; ++j) rw_sum += R.width[j];
    for (int j = 0; j < S.n_pay; ++j) sw_sum += S.width[j];
    const double t_rows = pl ? (double)pl->expect_rows : (double)T;
    double wbytes = key_reads + t_rows * (key_bytes + rw_sum + sw_sum);
    if (gfur) wbytes += t_rows * (rw_sum + sw_sum) + 4.0 * (nrows_r + nrows_s);
    else wbytes += nrows_r * rw_sum + nrows_s * sw_sum;
    // the streaming pass reads no R keys
    const double sbytes = wbytes - nrows_r * key_bytes;
    // Eager GFTR calls stage the R side in LDS when the largest partition's R
    // payload fits (staged_lds_limit() bytes).
    size_t shm = 0;
    if (!pl && !complex && !gfur && R.n_pay > 0) {
        for (int j = 0; j < R.n_pay; ++j) {
            a.rlds_off[j] = (uint32_t)shm;
            shm += ((size_t)max_r_rows * R.width[j] + 15) & ~(size_t)15;
        }
        if (shm > staged_lds_limit()) shm = 0;
    }
    // Eager calls launch the one write pass the count pass chose; plans launch
    // both, and the one that does not apply returns at once.
    if (shm) launch_join_pass(3, key_bytes, table_rows, s, false, grid, a, sbytes, shm);
    else if (pl || !complex) launch_join_pass(1, key_bytes, table_rows, s, pl != nullptr, grid, a, sbytes);
    if (pl || complex) {
        const double lbytes = pl ? 0.0 : wbytes;  // a plan counts its bytes once, on the streaming pass
        launch_join_pass(2, key_bytes, table_rows, s, pl != nullptr, grid, a, lbytes);
    }
    return pl ? 0 : (int64_t)T;
}

}  // namespace gj
