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
#include "internal.hpp"

namespace gj {
namespace {

constexpr int kItems = 16;
constexpr uint32_t kTile = kBlock * kItems;

struct PassArgs {
    const void *key_in;
    void *key_out;
    int ncols;
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
};

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
    __shared__ uint32_t s_cnt[kWaves][kRadix];
    __shared__ ChunkLoc s_loc;
    if (threadIdx.x == 0) s_loc = locate_chunk(a, blockIdx.x);
    for (int i = threadIdx.x; i < kWaves * kRadix; i += kBlock) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const ChunkLoc L = s_loc;
    if (!L.ok) return;
    const K *__restrict__ keys = static_cast<const K *>(a.key_in);
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (uint32_t base = L.row0 + w * kWave; base < L.row1; base += kBlock) {
        const uint32_t row = base + lane;
        const bool valid = row < L.row1;
        const uint32_t d = valid ? digit_of<K>(keys[row], a.dig) : 0u;
        const uint64_t peers = match_peers(d, a.bits, valid);
        if (valid && rank_below(peers) == 0) s_cnt[w][d] += (uint32_t)__popcll(peers);
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

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scatter(PassArgs a) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    __shared__ uint32_t s_wcnt[kWaves][kRadix];
    __shared__ uint32_t s_start[kRadix];
    __shared__ uint32_t s_tot[kRadix];
    __shared__ uint32_t s_cur[kRadix];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint64_t s_buf[TILE];
    __shared__ ChunkLoc s_loc;

    if (threadIdx.x == 0) s_loc = locate_chunk(a, blockIdx.x);
    __syncthreads();
    const ChunkLoc L = s_loc;
    if (!L.ok) return;

    const uint32_t R = 1u << a.bits;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    const uint32_t base_off = a.seg_off[0];
    for (uint32_t d = tid; d < kRadix; d += kBlock)
        s_cur[d] = d < R ? base_off + a.hist[L.hbase + d * L.m + L.j] : 0u;

    const K *__restrict__ keys = static_cast<const K *>(a.key_in);
    K *__restrict__ kout = static_cast<K *>(a.key_out);
    K *sk = reinterpret_cast<K *>(s_buf);

    for (uint32_t tile0 = L.row0; tile0 < L.row1; tile0 += TILE) {
        const uint32_t nt = min(TILE, L.row1 - tile0);
        for (int i = tid; i < kWaves * kRadix; i += kBlock) (&s_wcnt[0][0])[i] = 0;
        __syncthreads();

        K key[ITEMS];
        uint32_t dg[ITEMS], pos[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint32_t local = (uint32_t)(w * kWave * ITEMS + r * kWave + lane);
            const bool valid = local < nt;
            key[r] = valid ? keys[tile0 + local] : K(0);
            const uint32_t d = digit_of<K>(key[r], a.dig);
            const uint64_t peers = match_peers(d, a.bits, valid);
            uint32_t p = 0;
            if (valid) {
                const uint32_t rk = rank_below(peers);
                const uint32_t b = s_wcnt[w][d];
                if (rk == 0) s_wcnt[w][d] = b + (uint32_t)__popcll(peers);
                p = b + rk;
            }
            pos[r] = p;
            dg[r] = valid ? d : 0xFFFFFFFFu;
        }
        __syncthreads();
        {
            // tid == digit: per-digit tile totals and cross-wave exclusive prefix
            uint32_t t = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                const uint32_t c = s_wcnt[q][tid];
                s_wcnt[q][tid] = t;
                t += c;
            }
            s_tot[tid] = t;
            s_start[tid] = block_exclusive_sum<uint32_t>(t, s_tmp, (uint32_t *)nullptr);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            if (dg[r] != 0xFFFFFFFFu) {
                pos[r] += s_start[dg[r]] + s_wcnt[w][dg[r]];
                sk[pos[r]] = key[r];
            }
        }
        __syncthreads();

        uint32_t dst[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = (uint32_t)(k * kBlock + tid);
            dst[k] = 0;
            if (i < nt) {
                const K kk = sk[i];
                const uint32_t d = digit_of<K>(kk, a.dig);
                dst[k] = s_cur[d] + i - s_start[d];
                if (dst[k] >= a.n_rows) dst[k] = 0xFFFFFFFFu;  // never taken when offsets are right
                else kout[dst[k]] = kk;
            }
        }

        for (int c = 0; c < a.ncols; ++c) {
            __syncthreads();
            if (a.col_w[c] == 4) {
                uint32_t *sb = reinterpret_cast<uint32_t *>(s_buf);
                if (c == a.rowid_col) {
#pragma unroll
                    for (int r = 0; r < ITEMS; ++r) {
                        if (dg[r] != 0xFFFFFFFFu)
                            sb[pos[r]] = tile0 + (uint32_t)(w * kWave * ITEMS + r * kWave + lane);
                    }
                } else {
                    const uint32_t *__restrict__ in = static_cast<const uint32_t *>(a.col_in[c]);
#pragma unroll
                    for (int r = 0; r < ITEMS; ++r) {
                        if (dg[r] != 0xFFFFFFFFu)
                            sb[pos[r]] = in[tile0 + (uint32_t)(w * kWave * ITEMS + r * kWave + lane)];
                    }
                }
                __syncthreads();
                uint32_t *__restrict__ out = static_cast<uint32_t *>(a.col_out[c]);
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const uint32_t i = (uint32_t)(k * kBlock + tid);
                    if (i < nt && dst[k] != 0xFFFFFFFFu) out[dst[k]] = sb[i];
                }
            } else {
                const uint64_t *__restrict__ in = static_cast<const uint64_t *>(a.col_in[c]);
#pragma unroll
                for (int r = 0; r < ITEMS; ++r) {
                    if (dg[r] != 0xFFFFFFFFu) {
                        const uint32_t row = tile0 + (uint32_t)(w * kWave * ITEMS + r * kWave + lane);
                        s_buf[pos[r]] = in[row];
                    }
                }
                __syncthreads();
                uint64_t *__restrict__ out = static_cast<uint64_t *>(a.col_out[c]);
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const uint32_t i = (uint32_t)(k * kBlock + tid);
                    if (i < nt && dst[k] != 0xFFFFFFFFu) out[dst[k]] = s_buf[i];
                }
            }
        }
        __syncthreads();
        s_cur[tid] += s_tot[tid];
        __syncthreads();
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

template <typename K>
void run_pass(Ctx &ctx, PassArgs &a, uint32_t n) {
    hipStream_t s = ctx.stream;
    const uint32_t R = 1u << a.bits;
    // Aim for ~4096 chunks: a few per resident workgroup, each a whole number of tiles.
    uint32_t tiles = ceil_div_u32(n, kTile);
    uint32_t per = tiles > 4096 ? ceil_div_u32(tiles, 4096) : 1;
    a.chunk_rows = per * kTile;
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
    GJ_LAUNCH("k_hist", (double)n * sizeof(K), k_hist<K>, dim3((uint32_t)max_chunks), dim3(kBlock), 0, s, a);
    scan_exclusive_u32(ctx, hist, hist, hn, nullptr);
    GJ_LAUNCH("k_scatter", (double)n * row_bytes, (k_scatter<K, kItems>), dim3((uint32_t)max_chunks),
              dim3(kBlock), 0, s, a);
}

}  // namespace

void partition_run(Ctx &ctx, int key_bytes, const void *key_in, void *key_out, const PartCols &cols,
                   uint32_t n, int bit_lo, int bits, int passes, int mode, uint32_t *poff) {
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

    uint32_t *seg = ctx.scratch_n<uint32_t>(2);
    GJ_LAUNCH("k_set_range", 8.0, k_set_range, dim3(1), dim3(64), 0, s, seg, 0u, n);
    uint32_t nseg = 1;

    for (int p = 0; p < passes; ++p) {
        const bool last = (p == passes - 1);
        PassArgs a{};
        a.key_in = kin;
        a.key_out = last ? key_out : ctx.scratch((size_t)n * key_bytes);
        a.ncols = ncols;
        a.rowid_col = -1;
        for (int c = 0; c < ncols; ++c) {
            const bool is_rowid = cols.gen_rowid && c == cols.n;
            const int w = is_rowid ? 4 : cols.width[c];
            a.col_w[c] = w;
            a.col_in[c] = cin[c];
            a.col_out[c] = last ? (is_rowid ? cols.rowid_out : cols.out[c]) : ctx.scratch((size_t)n * w);
            // the row id is generated in pass 1 and moved like a payload afterwards
            if (is_rowid && p == 0) a.rowid_col = c;
        }
        const int shift = bit_lo + (p == 0 ? b[1] : 0);
        a.bits = b[p];
        a.dig = DigitFn{mode, shift, (1u << b[p]) - 1u};
        a.seg_off = seg;
        a.nseg = nseg;
        a.n_rows = n;
        if (n > 0) {
            if (key_bytes == 4) run_pass<int32_t>(ctx, a, n);
            else run_pass<int64_t>(ctx, a, n);
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
        for (int c = 0; c < ncols; ++c) cin[c] = a.col_out[c];
    }
}

}  // namespace gj
