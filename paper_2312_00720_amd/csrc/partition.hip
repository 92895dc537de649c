// Stable radix partitioning (the radix-partition primitive of Section 2.3, used
// as the transformation of the partitioned hash join in Section 4.1.4 and of the
// partition-based group-by in Section 4.3).
//
// One pass reorders rows stably by a digit of at most 8 bits. A pass works on
// segments (pass 1: the whole input; pass 2: every partition of pass 1), which
// are cut into chunks of whole tiles:
//   k_chunk_table  chunks per segment and their exclusive prefix
//   k_hist         per chunk, rows per digit -> hist[seg][digit][chunk]
//   scan           flat exclusive scan of hist = absolute output offset of each
//                  (segment, digit, chunk) run, because that order is the
//                  output order
//   k_scatter      per chunk, tile by tile: wave-level ranking by ballot (no
//                  atomics, so equal digits keep input order), LDS staging in
//                  digit order, then runs written contiguously; the key and
//                  every payload column reuse the same positions
//   k_poff         partition boundaries (segment, digit) for the next pass
// Two passes with the top bits first give rows sorted stably by the full digit,
// i.e. every partition contiguous and in input order.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "internal.hpp"

namespace gj {
namespace {

// Default scatter shape: the wide kernel (1024 threads x 16 rows, one column at
// a time with a rolling prefetch); group 0 names it among the shapes.
constexpr int kScatterBlock = 1024;
constexpr int kItems = 16;
constexpr int kGroup = 0;
constexpr uint32_t kTile = kBlock * kItems;

struct PassArgs {
    const void *key_in;
    void *key_out;
    int ncols;
    int n4;         // columns 0..n4-1 are 4 bytes wide, the rest 8 bytes
    int rowid_col;  // index of the generated row-id column, or -1
    const void *col_in[kMaxCols];
    void *col_out[kMaxCols];
    int col_w[kMaxCols];
    DigitFn dig;
    int bits;
    const uint32_t *seg_off;  // nseg + 1 row offsets
    uint32_t nseg;
    const uint32_t *chunk_base;  // nseg + 1 chunk offsets
    uint32_t chunk_rows;
    uint32_t *hist;  // [chunks][2^bits], laid out as (segment, digit, chunk)
    uint32_t n_rows; // rows of the output columns; every store is checked against it
    const uint8_t *seg_bits;  // optional: digit bits per segment (<= bits; batches of instances)
};

// The digit function of the segment a chunk belongs to.
__device__ __forceinline__ DigitFn seg_digit(const PassArgs &a, uint32_t seg) {
    DigitFn d = a.dig;
    if (a.seg_bits) d.mask = (1u << a.seg_bits[seg]) - 1u;
    return d;
}

struct ChunkLoc {
    uint32_t seg, j, m, row0, row1, hbase;
    int ok;
};

__device__ ChunkLoc locate_chunk(const PassArgs &a, uint32_t c) {
    ChunkLoc L{};
    const uint32_t total = a.chunk_base[a.nseg];
    if (c >= total) {
        L.ok = 0;
        return L;
    }
    uint32_t lo = 0, hi = a.nseg;  // chunk_base[lo] <= c < chunk_base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.chunk_base[mid] <= c) lo = mid;
        else hi = mid;
    }
    const uint32_t cb = a.chunk_base[lo];
    L.seg = lo;
    L.j = c - cb;
    L.m = a.chunk_base[lo + 1] - cb;
    const uint32_t s0 = a.seg_off[lo], s1 = a.seg_off[lo + 1];
    L.row0 = s0 + L.j * a.chunk_rows;
    L.row1 = min(L.row0 + a.chunk_rows, s1);
    L.hbase = cb << a.bits;
    L.ok = 1;
    return L;
}

__global__ __launch_bounds__(kBlock) void k_chunk_table(const uint32_t *__restrict__ seg_off,
                                                        uint32_t nseg, uint32_t chunk_rows,
                                                        uint32_t *__restrict__ chunk_base) {
    __shared__ uint32_t s_tmp[kWaves];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nseg; base += kBlock) {
        const uint32_t s = base + threadIdx.x;
        const uint32_t cnt = s < nseg ? ceil_div_u32(seg_off[s + 1] - seg_off[s], chunk_rows) : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum<uint32_t>(cnt, s_tmp, &tot);
        if (s < nseg) chunk_base[s] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) chunk_base[nseg] = carry;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_hist(PassArgs a) {
    constexpr int U = 16;  // loads in flight per thread
    __shared__ uint32_t s_cnt[kWaves][kRadix];
    __shared__ ChunkLoc s_loc;
    if (threadIdx.x == 0) s_loc = locate_chunk(a, blockIdx.x);
    for (int i = threadIdx.x; i < kWaves * kRadix; i += kBlock) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const ChunkLoc L = s_loc;
    if (!L.ok) return;
    const K *__restrict__ keys = static_cast<const K *>(a.key_in);
    const int tid = threadIdx.x, w = tid / kWave;
    const DigitFn dig = seg_digit(a, L.seg);
    for (uint32_t base = L.row0; base < L.row1; base += kBlock * U) {
        K k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t row = base + u * kBlock + tid;
            k[u] = row < L.row1 ? keys[row] : K(0);
        }
        // counting needs no order, so plain LDS atomics into the wave's own histogram
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kBlock + tid < L.row1) atomicAdd(&s_cnt[w][digit_of<K>(k[u], dig)], 1u);
        }
    }
    __syncthreads();
    const uint32_t R = 1u << a.bits;
    for (uint32_t d = threadIdx.x; d < R; d += kBlock) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) t += s_cnt[q][d];
        a.hist[L.hbase + d * L.m + L.j] = t;
    }
}

// Histogram of a single-segment pass from per-chunk counts of the low 8 bits
// of the digit source (made while the keys were read for another purpose):
// digit d of `bits` bits gathers the 8-bit values congruent to d.
__global__ void k_fold_hist(const uint32_t *__restrict__ hist8, uint32_t m, int bits, uint32_t *__restrict__ hist) {
    const uint32_t R = 1u << bits;
    const uint32_t per = 256u >> bits;  // 8-bit values per digit
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < R * m; idx += gridDim.x * blockDim.x) {
        const uint32_t d = idx / m, j = idx % m;
        const uint32_t *h = hist8 + (size_t)j * 256u;
        uint32_t t = 0;
        for (uint32_t q = 0; q < per; ++q) t += h[d + (q << bits)];
        hist[idx] = t;  // (segment 0, digit d, chunk j)
    }
}

// Loads of one tile: ITEMS keys per thread and the first group of up to G 4-byte
// columns (a generated row id is its row index). Rows past nt read as zero.
template <typename K, int BLOCK, int ITEMS, int G>
__device__ __forceinline__ void scatter_load_keys(const PassArgs &a, uint32_t tile0, uint32_t nt, K (&key)[ITEMS]) {
    const K *__restrict__ keys = static_cast<const K *>(a.key_in);
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t lbase = (uint32_t)(w * kWave * ITEMS + lane);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) key[r] = lbase + r * kWave < nt ? keys[tile0 + lbase + r * kWave] : K(0);
}

template <int BLOCK, int ITEMS>
__device__ __forceinline__ void scatter_load_col(const PassArgs &a, int c, uint32_t tile0, uint32_t nt,
                                                 uint32_t (&v)[ITEMS]) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t lbase = (uint32_t)(w * kWave * ITEMS + lane);
    const bool gen = (c == a.rowid_col);
    const uint32_t *__restrict__ in = static_cast<const uint32_t *>(a.col_in[c]);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t row = tile0 + lbase + r * kWave;
        v[r] = gen ? row : (lbase + r * kWave < nt ? in[row] : 0u);
    }
}

// One tile of the stable scatter: nt rows from tile0, whose keys are already in
// `key`. Once the keys are in LDS, their registers receive the next tile's keys
// (next0, next_nt rows; next_nt = 0: none), so that those loads are in flight
// during this tile's column work and the next tile ranks without waiting.
// Columns 0..n4-1 are 4-byte (the generated row id among them), columns
// n4..ncols-1 are 8-byte.
template <int BLOCK>
struct ScatterShared {
    static constexpr int W = BLOCK / kWave;
    uint32_t wcnt[W][kRadix];
    uint32_t start[kRadix];
    uint32_t tot[kRadix];
    uint32_t cur[kRadix];
    uint32_t tmp[kWaves];
};

template <typename K, int BLOCK, int ITEMS, int G>
__device__ __forceinline__ void scatter_tile(const PassArgs &a, const DigitFn &dig, ScatterShared<BLOCK> &S,
                                             uint32_t (*s_buf)[BLOCK * ITEMS], uint32_t tile0, uint32_t nt,
                                             K (&key)[ITEMS], uint32_t next0, uint32_t next_nt) {
    constexpr int W = BLOCK / kWave;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    K *__restrict__ kout = static_cast<K *>(a.key_out);
    K *sk = reinterpret_cast<K *>(&s_buf[0][0]);
    uint64_t *s8 = reinterpret_cast<uint64_t *>(&s_buf[0][0]);
    const int n4 = a.n4;
    const bool full = (nt == BLOCK * ITEMS);
    const uint32_t lbase = (uint32_t)(w * kWave * ITEMS + lane);
#define GJ_VALID(r) (full || lbase + (r) * kWave < nt)

    for (int i = tid; i < W * kRadix; i += BLOCK) (&S.wcnt[0][0])[i] = 0;
    // the first column group is loaded now and consumed after the ranking
    uint32_t v[G][ITEMS];
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (g < n4) scatter_load_col<BLOCK, ITEMS>(a, g, tile0, nt, v[g]);
    __syncthreads();

    // stable rank within the wave: ballot peers, the leader bumps the wave counter
    uint32_t pos[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = GJ_VALID(r);
        const uint32_t d = digit_of<K>(key[r], dig);
        const uint64_t peers = match_peers(d, a.bits, valid);
        uint32_t p = 0;
        if (valid) {
            const uint32_t rk = rank_below(peers);
            const uint32_t b = S.wcnt[w][d];
            if (rk == 0) S.wcnt[w][d] = b + (uint32_t)__popcll(peers);
            p = b + rk;
        }
        pos[r] = p;
    }
    __syncthreads();
    if (tid < kRadix) {
        // threads 0..255 (one per digit): tile totals and cross-wave exclusive prefix
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint32_t c = S.wcnt[q][tid];
            S.wcnt[q][tid] = t;
            t += c;
        }
        S.tot[tid] = t;
        // exclusive scan over the 256 digits by the first four waves
        const uint32_t inc = wave_inclusive_sum<uint32_t>(t);
        if (lane == kWave - 1) S.tmp[w] = inc;
        S.start[tid] = inc - t;
    }
    __syncthreads();
    if (tid < kRadix) {
        uint32_t before = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) before += (q < w) ? S.tmp[q] : 0u;
        S.start[tid] += before;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (GJ_VALID(r)) {
            const uint32_t d = digit_of<K>(key[r], dig);
            pos[r] += S.start[d] + S.wcnt[w][d];
            sk[pos[r]] = key[r];
        }
    }
    // the key registers are free: next tile's keys
    if (next_nt) scatter_load_keys<K, BLOCK, ITEMS, G>(a, next0, next_nt, key);
    __syncthreads();

    uint32_t dst[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = (uint32_t)(k * BLOCK + tid);
        dst[k] = 0xFFFFFFFFu;
        if (full || i < nt) {
            const K kk = sk[i];
            const uint32_t d = digit_of<K>(kk, dig);
            const uint32_t t = S.cur[d] + i - S.start[d];
            if (t < a.n_rows) {  // always true when the offsets are right
                dst[k] = t;
                kout[t] = kk;
            }
        }
    }
    // 4-byte keys sit in buffer 0, so the first column goes to buffer 1; 8-byte
    // keys use both buffers and need a barrier before reuse.
    int par = 1;
    if constexpr (sizeof(K) == 8) {
        __syncthreads();
        par = 0;
    }
    for (int c0 = 0; c0 < n4; c0 += G) {
        if (c0 > 0) {
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (c0 + g < n4) scatter_load_col<BLOCK, ITEMS>(a, c0 + g, tile0, nt, v[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (c0 + g < n4) {
                uint32_t *sb = s_buf[par];
#pragma unroll
                for (int r = 0; r < ITEMS; ++r)
                    if (GJ_VALID(r)) sb[pos[r]] = v[g][r];
                __syncthreads();
                uint32_t *__restrict__ out = static_cast<uint32_t *>(a.col_out[c0 + g]);
#pragma unroll
                for (int k = 0; k < ITEMS; ++k)
                    if (dst[k] != 0xFFFFFFFFu) out[dst[k]] = sb[k * BLOCK + tid];
                par ^= 1;
            }
        }
    }
    for (int c = n4; c < a.ncols; ++c) {
        uint64_t x[ITEMS];
        const uint64_t *__restrict__ in = static_cast<const uint64_t *>(a.col_in[c]);
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) x[r] = GJ_VALID(r) ? in[tile0 + lbase + r * kWave] : 0ull;
        __syncthreads();  // both buffers free
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (GJ_VALID(r)) s8[pos[r]] = x[r];
        __syncthreads();
        uint64_t *__restrict__ out = static_cast<uint64_t *>(a.col_out[c]);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (dst[k] != 0xFFFFFFFFu) out[dst[k]] = s8[k * BLOCK + tid];
    }
#undef GJ_VALID
    __syncthreads();
    if (tid < kRadix) S.cur[tid] += S.tot[tid];
    __syncthreads();
}

// Loads of the wide kernel: one 64-bit base address per thread, every row at a
// constant offset from it (r * 64 rows), so that the 16 loads of a column need
// no per-row address registers. A full tile loads without row checks; in a
// partial one, rows past nt read as zero. A generated row id is its row index.
template <typename K, int ITEMS>
__device__ __forceinline__ void wide_load_keys(const PassArgs &a, uint32_t tile0, uint32_t nt, K (&key)[ITEMS]) {
    constexpr uint32_t TILE = 1024u * ITEMS;
    const uint32_t lbase = (uint32_t)((threadIdx.x / kWave) * kWave * ITEMS + lane_id());
    const K *__restrict__ p = static_cast<const K *>(a.key_in) + (tile0 + lbase);
    if (nt == TILE) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) key[r] = p[r * kWave];
    } else {
        const uint32_t rem = nt > lbase ? nt - lbase : 0u;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) key[r] = (uint32_t)(r * kWave) < rem ? p[r * kWave] : K(0);
    }
}

template <int ITEMS>
__device__ __forceinline__ void wide_load_col(const PassArgs &a, int c, uint32_t tile0, uint32_t nt,
                                              uint32_t (&v)[ITEMS]) {
    constexpr uint32_t TILE = 1024u * ITEMS;
    const uint32_t lbase = (uint32_t)((threadIdx.x / kWave) * kWave * ITEMS + lane_id());
    if (c == a.rowid_col) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) v[r] = tile0 + lbase + r * kWave;
        return;
    }
    const uint32_t *__restrict__ p = static_cast<const uint32_t *>(a.col_in[c]) + (tile0 + lbase);
    if (nt == TILE) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) v[r] = p[r * kWave];
    } else {
        const uint32_t rem = nt > lbase ? nt - lbase : 0u;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) v[r] = (uint32_t)(r * kWave) < rem ? p[r * kWave] : 0u;
    }
}

// Wide tiles: 1024 threads x 16 rows = 16384-row tiles, twice the rows of the
// default shape, so that every digit's run per tile (the burst each column
// writes to HBM) is twice as long. The shorter the bursts, the slower the
// scatter: at equal work, 8-bit digits over 8192-row tiles write at about 55%
// of the rate of one-digit tiles. The larger tile fits the registers because
// columns move one at a time: while column c is staged and stored, column
// c + 1 (or the next tile's first column) is already loading into the one
// column register array, and 8-byte columns move in two halves of 8 rows.
// FULL tiles (all but a chunk's last) carry no per-row checks.
template <typename K, int BLOCK, int ITEMS, bool FULL>
__device__ __forceinline__ void scatter_tile_wide(const PassArgs &a, const DigitFn &dig, ScatterShared<BLOCK> &S,
                                                  uint32_t (*s_buf)[BLOCK * ITEMS], uint32_t tile0, uint32_t nt,
                                                  K (&key)[ITEMS], uint32_t (&v)[ITEMS], uint32_t next0,
                                                  uint32_t next_nt) {
    constexpr int W = BLOCK / kWave;
    // the thread index passes through an empty asm statement, so that nothing
    // derived from it is hoisted out of a caller's tile loop (it would hold
    // registers across the whole loop)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int w = tid / kWave, lane = tid % kWave;
    K *__restrict__ kout = static_cast<K *>(a.key_out);
    K *sk = reinterpret_cast<K *>(&s_buf[0][0]);
    uint64_t *s8 = reinterpret_cast<uint64_t *>(&s_buf[0][0]);
    const int n4 = a.n4;
    const uint32_t lbase = (uint32_t)(w * kWave * ITEMS + lane);
    // rows of this thread (r * 64 < lrem) and staged slots of this thread (k * BLOCK < srem)
    const uint32_t lrem = FULL ? 0xFFFFFFFFu : (nt > lbase ? nt - lbase : 0u);
    const uint32_t srem = FULL ? 0xFFFFFFFFu : (nt > (uint32_t)tid ? nt - (uint32_t)tid : 0u);
#define GJ_VALID(r) (FULL || (uint32_t)((r) * kWave) < lrem)

    for (int i = tid; i < W * kRadix; i += BLOCK) (&S.wcnt[0][0])[i] = 0;
    __syncthreads();

    // stable rank within the wave: ballot peers, the leader bumps the wave counter
    uint32_t pos[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = GJ_VALID(r);
        const uint32_t d = digit_of<K>(key[r], dig);
        const uint64_t peers = match_peers(d, a.bits, valid);
        uint32_t p = 0;
        if (valid) {
            const uint32_t rk = rank_below(peers);
            const uint32_t b = S.wcnt[w][d];
            if (rk == 0) S.wcnt[w][d] = b + (uint32_t)__popcll(peers);
            p = b + rk;
        }
        pos[r] = p;
    }
    __syncthreads();
    if (tid < kRadix) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint32_t c = S.wcnt[q][tid];
            S.wcnt[q][tid] = t;
            t += c;
        }
        S.tot[tid] = t;
        const uint32_t inc = wave_inclusive_sum<uint32_t>(t);
        if (lane == kWave - 1) S.tmp[w] = inc;
        S.start[tid] = inc - t;
    }
    __syncthreads();
    if (tid < kRadix) {
        uint32_t before = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) before += (q < w) ? S.tmp[q] : 0u;
        S.start[tid] += before;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (GJ_VALID(r)) {
            const uint32_t d = digit_of<K>(key[r], dig);
            pos[r] += S.start[d] + S.wcnt[w][d];
            sk[pos[r]] = key[r];
        }
    }
    // the key registers are free: next tile's keys
    if (next_nt) wide_load_keys<K, ITEMS>(a, next0, next_nt, key);
    // LDS slots (< 16384) two to a register from here on
    uint32_t pp[ITEMS / 2];
#pragma unroll
    for (int r = 0; r < ITEMS / 2; ++r) pp[r] = (pos[2 * r] & 0xFFFFu) | (pos[2 * r + 1] << 16);
#define GJ_POS(r) ((pp[(r) >> 1] >> (16 * ((r) & 1))) & 0xFFFFu)
    __syncthreads();

    uint32_t dst[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = (uint32_t)(k * BLOCK + tid);
        dst[k] = 0xFFFFFFFFu;
        if (FULL || (uint32_t)(k * BLOCK) < srem) {
            const K kk = sk[i];
            const uint32_t d = digit_of<K>(kk, dig);
            const uint32_t t = S.cur[d] + i - S.start[d];
            if (t < a.n_rows) {  // always true when the offsets are right
                dst[k] = t;
                kout[t] = kk;
            }
        }
    }

    // 4-byte keys sit in buffer 0, so the first column goes to buffer 1; 8-byte
    // keys use both buffers and need a barrier before reuse.
    int par = 1;
    if constexpr (sizeof(K) == 8) {
        __syncthreads();
        par = 0;
    }
#pragma unroll 1
    for (int c = 0; c < n4; ++c) {
        uint32_t *sb = s_buf[par];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (GJ_VALID(r)) sb[GJ_POS(r)] = v[r];
        // v is free: the next column of this tile, or the next tile's first one
        // (one load sequence for both cases keeps the register count down)
        const bool more = c + 1 < n4;
        if (more || next_nt)
            wide_load_col<ITEMS>(a, more ? c + 1 : 0, more ? tile0 : next0, more ? nt : next_nt, v);
        __syncthreads();
        uint32_t *__restrict__ out = static_cast<uint32_t *>(a.col_out[c]);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (dst[k] != 0xFFFFFFFFu) out[dst[k]] = sb[k * BLOCK + tid];
        par ^= 1;
    }
#pragma unroll 1
    for (int c = n4; c < a.ncols; ++c) {
        constexpr int HI = ITEMS / 2;
        const uint64_t *__restrict__ in = static_cast<const uint64_t *>(a.col_in[c]) + (tile0 + lbase);
        uint64_t x[HI];
#pragma unroll
        for (int r = 0; r < HI; ++r) x[r] = GJ_VALID(r) ? in[r * kWave] : 0ull;
        __syncthreads();  // both buffers free
#pragma unroll
        for (int r = 0; r < HI; ++r)
            if (GJ_VALID(r)) s8[GJ_POS(r)] = x[r];
#pragma unroll
        for (int r = 0; r < HI; ++r) x[r] = GJ_VALID(HI + r) ? in[(HI + r) * kWave] : 0ull;
#pragma unroll
        for (int r = 0; r < HI; ++r)
            if (GJ_VALID(HI + r)) s8[GJ_POS(HI + r)] = x[r];
        __syncthreads();
        uint64_t *__restrict__ out = static_cast<uint64_t *>(a.col_out[c]);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (dst[k] != 0xFFFFFFFFu) out[dst[k]] = s8[k * BLOCK + tid];
    }
#undef GJ_POS
#undef GJ_VALID
    __syncthreads();
    if (tid < kRadix) S.cur[tid] += S.tot[tid];
    __syncthreads();
}

template <typename K, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_scatter_wide(PassArgs a) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    static_assert(BLOCK == 1024, "the wide loads assume 1024 threads");
    __shared__ ScatterShared<BLOCK> S;
    __shared__ uint32_t s_buf[2][TILE];  // double buffer for 4-byte columns; 8-byte data spans both
    __shared__ ChunkLoc s_loc;

    if (threadIdx.x == 0) s_loc = locate_chunk(a, blockIdx.x);
    __syncthreads();
    const ChunkLoc L = s_loc;
    if (!L.ok) return;

    const uint32_t R = 1u << a.bits;
    const uint32_t base_off = a.seg_off[0];
    for (uint32_t d = threadIdx.x; d < kRadix; d += BLOCK)
        S.cur[d] = d < R ? base_off + a.hist[L.hbase + d * L.m + L.j] : 0u;

    const DigitFn dig = seg_digit(a, L.seg);
    K key[ITEMS];
    uint32_t v[ITEMS];
    uint32_t tile0 = L.row0;
    uint32_t nt = min(TILE, L.row1 - tile0);
    if (nt) {
        wide_load_keys<K, ITEMS>(a, tile0, nt, key);
        if (a.n4 > 0) wide_load_col<ITEMS>(a, 0, tile0, nt, v);
    }
    // full tiles, then at most one partial tile (a chunk's last)
    while (nt == TILE) {
        const uint32_t next0 = tile0 + nt;
        const uint32_t next_nt = next0 < L.row1 ? min(TILE, L.row1 - next0) : 0u;
        scatter_tile_wide<K, BLOCK, ITEMS, true>(a, dig, S, s_buf, tile0, nt, key, v, next0, next_nt);
        tile0 = next0;
        nt = next_nt;
    }
    if (nt) scatter_tile_wide<K, BLOCK, ITEMS, false>(a, dig, S, s_buf, tile0, nt, key, v, 0u, 0u);
}

// MINW: minimum waves per SIMD the register allocation must allow (4 lets two
// 512-thread workgroups share a compute unit).
template <typename K, int BLOCK, int ITEMS, int G, int MINW>
__global__ __launch_bounds__(BLOCK, MINW) void k_scatter(PassArgs a) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ ScatterShared<BLOCK> S;
    __shared__ uint32_t s_buf[2][TILE];  // double buffer for 4-byte columns; 8-byte data spans both
    __shared__ ChunkLoc s_loc;

    if (threadIdx.x == 0) s_loc = locate_chunk(a, blockIdx.x);
    __syncthreads();
    const ChunkLoc L = s_loc;
    if (!L.ok) return;

    const uint32_t R = 1u << a.bits;
    const uint32_t base_off = a.seg_off[0];
    for (uint32_t d = threadIdx.x; d < kRadix; d += BLOCK)
        S.cur[d] = d < R ? base_off + a.hist[L.hbase + d * L.m + L.j] : 0u;

    const DigitFn dig = seg_digit(a, L.seg);
    K key[ITEMS];
    uint32_t tile0 = L.row0;
    uint32_t nt = min(TILE, L.row1 - tile0);
    if (nt) scatter_load_keys<K, BLOCK, ITEMS, G>(a, tile0, nt, key);
    while (nt) {
        const uint32_t next0 = tile0 + nt;
        const uint32_t next_nt = next0 < L.row1 ? min(TILE, L.row1 - next0) : 0u;
        scatter_tile<K, BLOCK, ITEMS, G>(a, dig, S, s_buf, tile0, nt, key, next0, next_nt);
        tile0 = next0;
        nt = next_nt;
    }
}

__global__ void k_poff(const uint32_t *__restrict__ seg_off, uint32_t nseg,
                       const uint32_t *__restrict__ chunk_base, const uint32_t *__restrict__ hist,
                       int bits, uint32_t *__restrict__ poff) {
    const uint32_t R = 1u << bits;
    const uint64_t total = (uint64_t)nseg * R;
    const uint32_t base_off = seg_off[0];
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = (uint32_t)(idx >> bits), d = (uint32_t)(idx & (R - 1));
        const uint32_t cb = chunk_base[s], m = chunk_base[s + 1] - cb;
        poff[idx] = m ? base_off + hist[((uint64_t)cb << bits) + (uint64_t)d * m] : seg_off[s];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) poff[total] = seg_off[nseg];
}

__global__ void k_set_range(uint32_t *p, uint32_t a, uint32_t b) {
    if (threadIdx.x == 0) {
        p[0] = a;
        p[1] = b;
    }
}

// Scatter tile shapes (rows per thread x 4-byte columns loaded together). The
// shape changes speed only; GJ_SCATTER_SHAPE=<items>x<group> picks one.
struct Shape {
    int block, items, group;
};
// Group 0 is the wide-tile kernel (one column at a time, rolling prefetch).
constexpr Shape kVariants[kScatterVariants] = {{256, 8, 4},  {512, 8, 4},  {1024, 8, 4}, {512, 4, 4},
                                               {1024, 4, 4}, {256, 16, 2}, {512, 8, 2},  {512, 16, 2},
                                               {512, 16, 4}, {1024, 8, 2},  {1024, 16, 2}, {1024, 16, 1},
                                               {512, 16, 1}, {1024, 16, 0}};
thread_local int g_variant = 0;

Shape scatter_shape() {
    if (g_variant >= 1 && g_variant <= kScatterVariants) return kVariants[g_variant - 1];
    static Shape sh = [] {
        Shape x{kScatterBlock, kItems, kGroup};
        if (const char *e = getenv("GJ_SCATTER_SHAPE")) {
            int b = 0, i = 0, g = 0;
            if (sscanf(e, "%dx%dx%d", &b, &i, &g) == 3) x = Shape{b, i, g};
        }
        return x;
    }();
    return sh;
}

template <typename K>
void launch_scatter(const Shape &sh, dim3 grid, hipStream_t s, const PassArgs &a, double bytes) {
#define GJ_SC(B, I, G_)                                                                    \
    if (sh.block == B && sh.items == I && sh.group == G_) {                                \
        GJ_LAUNCH("k_scatter", bytes, (k_scatter<K, B, I, G_, (B == 512 && I == 16 && G_ == 1) ? 4 : 1>), grid, \
                  dim3(B), 0, s, a);                                                       \
        return;                                                                            \
    }
    GJ_SC(256, 8, 4) GJ_SC(512, 8, 4) GJ_SC(1024, 8, 4) GJ_SC(512, 4, 4) GJ_SC(1024, 4, 4)
    GJ_SC(256, 16, 2) GJ_SC(512, 8, 2) GJ_SC(512, 16, 2) GJ_SC(512, 16, 4) GJ_SC(1024, 8, 2)
    GJ_SC(1024, 16, 2) GJ_SC(1024, 16, 1) GJ_SC(512, 16, 1)
#undef GJ_SC
    if (sh.block == 1024 && sh.items == 16 && sh.group == 0) {
        GJ_LAUNCH("k_scatter", bytes, (k_scatter_wide<K, 1024, 16>), grid, dim3(1024), 0, s, a);
        return;
    }
    throw Error(GJ_EINVAL, "unknown scatter shape");
}

// Fills the column part of PassArgs: 4-byte columns first (the scatter loads them in
// groups), then 8-byte ones. cin/cout are indexed by logical column (the row id, if
// generated, is column cols.n); map[c] receives the slot of logical column c.
void assign_cols(PassArgs &a, const PartCols &cols, const void *const *cin, void *const *cout, bool first_pass,
                 int *map) {
    const int ncols = cols.n + (cols.gen_rowid ? 1 : 0);
    a.ncols = ncols;
    a.rowid_col = -1;
    a.n4 = 0;
    int slot = 0;
    for (int pass4 = 1; pass4 >= 0; --pass4) {
        for (int c = 0; c < ncols; ++c) {
            const bool is_rowid = cols.gen_rowid && c == cols.n;
            const int w = is_rowid ? 4 : cols.width[c];
            if ((w == 4) != (pass4 == 1)) continue;
            a.col_w[slot] = w;
            a.col_in[slot] = cin[c];
            a.col_out[slot] = cout[c];
            // the row id is generated in the first pass and moved like a payload afterwards
            if (is_rowid && first_pass) a.rowid_col = slot;
            map[c] = slot;
            if (w == 4) a.n4++;
            ++slot;
        }
    }
}

template <typename K>
__global__ void k_key_bits(const K *__restrict__ keys, uint32_t n, unsigned long long *__restrict__ acc) {
    // OR and AND of the order-preserving key bits over all keys, 16 loads in
    // flight per thread
    constexpr int U = 16;
    unsigned long long o = 0, x = ~0ull;
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x * U + threadIdx.x; base < n; base += step * U) {
        K k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = base + u * blockDim.x;
            k[u] = i < n ? keys[i] : keys[base];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned long long v = digit_source<K>(k[u], kDigitOrdered);
            o |= v;
            x &= v;
        }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        o |= __shfl_xor(o, d, kWave);
        x &= __shfl_xor(x, d, kWave);
    }
    if (lane_id() == 0) {
        atomicOr(&acc[0], o);
        atomicAnd(&acc[1], x);
    }
}

// Aim for ~4096 chunks: a few per resident workgroup, each a whole number of tiles.
uint32_t chunk_rows_for(uint32_t n) {
    const Shape sh = scatter_shape();
    const uint32_t tile = (uint32_t)(sh.block * sh.items);
    const uint32_t tiles = ceil_div_u32(n, tile);
    const uint32_t per = tiles > 4096 ? ceil_div_u32(tiles, 4096) : 1;
    return per * tile;
}

template <typename K>
void run_pass(Ctx &ctx, PassArgs &a, uint32_t n, const uint32_t *hist8 = nullptr) {
    hipStream_t s = ctx.stream;
    const uint32_t R = 1u << a.bits;
    const Shape sh = scatter_shape();
    a.chunk_rows = chunk_rows_for(n);
    const uint64_t max_chunks = (uint64_t)ceil_div_u32(n, a.chunk_rows) + a.nseg;
    uint32_t *chunk_base = ctx.scratch_n<uint32_t>(a.nseg + 1);
    a.chunk_base = chunk_base;
    const uint64_t hn = max_chunks * R;
    uint32_t *hist = ctx.scratch_n<uint32_t>(hn);
    a.hist = hist;
    // algorithmic bytes of one scatter: read and write the key and every column
    // once (a generated row id is only written)
    double row_bytes = 2.0 * sizeof(K);
    for (int c = 0; c < a.ncols; ++c) row_bytes += (c == a.rowid_col ? 0 : a.col_w[c]) + a.col_w[c];
    GJ_LAUNCH("k_chunk_table", 8.0 * (a.nseg + 1), k_chunk_table, dim3(1), dim3(kBlock), 0, s, a.seg_off,
              a.nseg, a.chunk_rows, chunk_base);
    fill_u32(s, hist, 0u, hn);
    if (hist8) {
        // one segment: chunks 0..m-1, the digit the low bits of the same source
        const uint32_t m = ceil_div_u32(n, a.chunk_rows);
        GJ_LAUNCH("k_fold_hist", 4.0 * m * 256 + 4.0 * m * R, k_fold_hist,
                  dim3(std::min<uint32_t>(ceil_div_u32(R * m, kBlock), 4096)), dim3(kBlock), 0, s, hist8, m, a.bits,
                  hist);
    } else {
        GJ_LAUNCH("k_hist", (double)n * sizeof(K), k_hist<K>, dim3((uint32_t)max_chunks), dim3(kBlock), 0, s, a);
    }
    scan_exclusive_u32(ctx, hist, hist, hn, nullptr);
    launch_scatter<K>(sh, dim3((uint32_t)max_chunks), s, a, (double)n * row_bytes);
}

}  // namespace

void set_scatter_variant(int v) { g_variant = v; }

uint32_t pass_chunk_rows(uint32_t n) { return chunk_rows_for(n); }

void partition_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                   uint32_t n, int bit_lo, int bits, int passes, int mode, uint32_t *poff, const uint32_t *hist8) {
    require(!hist8 || (passes == 1 && bit_lo == 0), "a precomputed histogram serves one pass from bit 0");
    require(key_bytes == 4 || key_bytes == 8, "key width must be 4 or 8 bytes");
    require(bits >= 1 && bits <= 16, "partition bits must be 1..16");
    require(passes >= 1 && passes <= 2, "partition passes must be 1 or 2");
    require(bits <= 8 * passes, "at most 8 bits per pass");
    require(passes == 1 || bits >= 2, "two passes need at least 2 bits");
    const int ncols = cols.n + (cols.gen_rowid ? 1 : 0);
    require(ncols <= kMaxCols, "too many columns");
    hipStream_t s = ctx.stream;

    int b[2];
    b[0] = passes == 1 ? bits : (bits + 1) / 2;  // pass 1 takes the top bits
    b[1] = bits - b[0];

    // Per-pass output buffers: the last pass writes the caller's buffers.
    const void *kin = key_in;
    const void *cin[kMaxCols];
    for (int c = 0; c < cols.n; ++c) cin[c] = cols.in[c];
    if (cols.gen_rowid) cin[cols.n] = nullptr;

    int map[kMaxCols];
    uint32_t *seg = ctx.scratch_n<uint32_t>(2);
    GJ_LAUNCH("k_set_range", 8.0, k_set_range, dim3(1), dim3(64), 0, s, seg, 0u, n);
    uint32_t nseg = 1;

    for (int p = 0; p < passes; ++p) {
        const bool last = (p == passes - 1);
        PassArgs a{};
        a.key_in = kin;
        a.key_out = last ? key_out : ctx.scratch((size_t)n * key_bytes);
        void *cout[kMaxCols];
        for (int c = 0; c < ncols; ++c) {
            const bool is_rowid = cols.gen_rowid && c == cols.n;
            const int w = is_rowid ? 4 : cols.width[c];
            cout[c] = last ? (is_rowid ? cols.rowid_out : cols.out[c]) : ctx.scratch((size_t)n * w);
        }
        assign_cols(a, cols, cin, cout, p == 0, map);
        const int shift = bit_lo + (p == 0 ? b[1] : 0);
        a.bits = b[p];
        a.dig = DigitFn{mode, shift, (1u << b[p]) - 1u};
        a.seg_off = seg;
        a.nseg = nseg;
        a.n_rows = n;
        if (n > 0) {
            if (key_bytes == 4) run_pass<int32_t>(ctx, a, n, hist8);
            else run_pass<int64_t>(ctx, a, n, hist8);
        } else {
            uint32_t *cb = ctx.scratch_n<uint32_t>(nseg + 1);
            fill_u32(s, cb, 0u, nseg + 1);
            a.chunk_base = cb;
            a.hist = ctx.scratch_n<uint32_t>(1);
        }
        const uint64_t np = (uint64_t)nseg << b[p];
        uint32_t *next = last ? poff : ctx.scratch_n<uint32_t>(np + 1);
        GJ_LAUNCH("k_poff", 8.0 * (np + 1), k_poff, dim3((uint32_t)std::min<uint64_t>((np + 255) / 256, 4096)),
                  dim3(256), 0, s, seg, nseg, a.chunk_base, a.hist, b[p], next);
        seg = next;
        nseg = (uint32_t)np;
        kin = a.key_out;
        for (int c = 0; c < ncols; ++c) cin[c] = a.col_out[map[c]];
    }
}


void sort_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols, uint32_t n) {
    require(key_bytes == 4 || key_bytes == 8, "key width must be 4 or 8 bytes");
    hipStream_t s = ctx.stream;
    const int ncols = cols.n + (cols.gen_rowid ? 1 : 0);
    // bytes of the order-preserving key that differ between keys; equal bytes need no pass
    std::vector<int> passes;
    if (n > 0) {
        unsigned long long *acc = reinterpret_cast<unsigned long long *>(ctx.scratch_n<uint64_t>(2));
        fill_u64(s, reinterpret_cast<uint64_t *>(acc), 0ull, 1);
        fill_u64(s, reinterpret_cast<uint64_t *>(acc) + 1, ~0ull, 1);
        const uint32_t grid = std::min<uint32_t>(ceil_div_u32(n, 256 * 16), 2048);
        if (key_bytes == 4)
            GJ_LAUNCH("k_key_bits", 4.0 * n, k_key_bits<int32_t>, dim3(grid), dim3(256), 0, s,
                      static_cast<const int32_t *>(key_in), n, acc);
        else
            GJ_LAUNCH("k_key_bits", 8.0 * n, k_key_bits<int64_t>, dim3(grid), dim3(256), 0, s,
                      static_cast<const int64_t *>(key_in), n, acc);
        uint64_t h[2];
        GJ_HIP(hipMemcpyAsync(h, acc, 16, hipMemcpyDeviceToHost, s));
        GJ_HIP(hipStreamSynchronize(s));
        const uint64_t diff = h[0] ^ h[1];
        for (int b = 0; b < key_bytes; ++b)
            if ((diff >> (8 * b)) & 0xFF) passes.push_back(b);
    }
    if (passes.empty()) passes.push_back(0);  // a pass on an equal digit is a stable copy
    uint32_t *seg = ctx.scratch_n<uint32_t>(2);
    GJ_LAUNCH("k_set_range", 8.0, k_set_range, dim3(1), dim3(64), 0, s, seg, 0u, n);
    const void *kin = key_in;
    const void *cin[kMaxCols];
    for (int c = 0; c < cols.n; ++c) cin[c] = cols.in[c];
    if (cols.gen_rowid) cin[cols.n] = nullptr;
    void *bufk[2] = {nullptr, nullptr};
    void *bufc[2][kMaxCols];
    const int P = (int)passes.size();
    for (int p = 0; p < P; ++p) {
        const bool last = (p == P - 1);
        PassArgs a{};
        void *cout[kMaxCols];
        void *kout;
        if (last) {
            kout = key_out;
            for (int c = 0; c < ncols; ++c) cout[c] = (cols.gen_rowid && c == cols.n) ? cols.rowid_out : cols.out[c];
        } else {
            const int b = p & 1;
            if (!bufk[b]) {
                bufk[b] = ctx.scratch((size_t)n * key_bytes);
                for (int c = 0; c < ncols; ++c)
                    bufc[b][c] = ctx.scratch((size_t)n * ((cols.gen_rowid && c == cols.n) ? 4 : cols.width[c]));
            }
            kout = bufk[b];
            for (int c = 0; c < ncols; ++c) cout[c] = bufc[b][c];
        }
        a.key_in = kin;
        a.key_out = kout;
        int map[kMaxCols];
        assign_cols(a, cols, cin, cout, p == 0, map);
        a.bits = 8;
        a.dig = DigitFn{kDigitOrdered, 8 * passes[p], 0xFFu};
        a.seg_off = seg;
        a.nseg = 1;
        a.n_rows = n;
        if (n > 0) {
            if (key_bytes == 4) run_pass<int32_t>(ctx, a, n);
            else run_pass<int64_t>(ctx, a, n);
        }
        kin = kout;
        for (int c = 0; c < ncols; ++c) cin[c] = cout[c];
    }
}


void partition_run_segments(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                            uint32_t n, const uint32_t *seg_off, uint32_t nseg, const uint8_t *seg_bits,
                            uint32_t *poff, int mode) {
    require(key_bytes == 4 || key_bytes == 8, "key width must be 4 or 8 bytes");
    hipStream_t s = ctx.stream;
    const int ncols = cols.n + (cols.gen_rowid ? 1 : 0);
    require(ncols <= kMaxCols, "too many columns");
    const void *cin[kMaxCols];
    void *cout[kMaxCols];
    for (int c = 0; c < ncols; ++c) {
        const bool is_rowid = cols.gen_rowid && c == cols.n;
        cin[c] = is_rowid ? nullptr : cols.in[c];
        cout[c] = is_rowid ? cols.rowid_out : cols.out[c];
    }
    PassArgs a{};
    a.key_in = key_in;
    a.key_out = key_out;
    int map[kMaxCols];
    assign_cols(a, cols, cin, cout, true, map);
    a.bits = 8;
    a.dig = DigitFn{mode, 0, 0xFFu};
    a.seg_off = seg_off;
    a.nseg = nseg;
    a.n_rows = n;
    a.seg_bits = seg_bits;
    if (n > 0) {
        if (key_bytes == 4) run_pass<int32_t>(ctx, a, n);
        else run_pass<int64_t>(ctx, a, n);
    } else {
        uint32_t *cb = ctx.scratch_n<uint32_t>(nseg + 1);
        fill_u32(s, cb, 0u, nseg + 1);
        a.chunk_base = cb;
        a.hist = ctx.scratch_n<uint32_t>(1);
    }
    const uint64_t np = (uint64_t)nseg << 8;
    GJ_LAUNCH("k_poff", 8.0 * (np + 1), k_poff, dim3((uint32_t)std::min<uint64_t>((np + 255) / 256, 4096)),
              dim3(256), 0, s, seg_off, nseg, a.chunk_base, a.hist, 8, poff);
}

}  // namespace gj
