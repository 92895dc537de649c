// Sort-merge join (Section 3.1.1): transformation by full-key radix sort of both
// relations, match finding with the Merge Path split of the two sorted key
// sequences, and materialization under GFTR (payloads sorted with the keys and
// gathered from the sorted copies, at positions that only grow) or GFUR (keys
// sorted with row ids; payloads gathered from the original columns).
//
// Match finding. Merging R' and S' with S rows placed before R rows of an equal
// key, the R rows that precede S'[j] are exactly those with smaller keys, so
// the merged position of S'[j] minus j is its lower bound in R'. The merged
// sequence is cut into tiles of kMergeTile elements along its diagonals (one
// binary search per diagonal: the Merge Path of Green, McColl and Bader); each
// workgroup loads its tile's two ranges into LDS and every thread merges
// kMergeItems consecutive elements after its own diagonal search, so the work
// per thread is the same whatever the key distribution. The matches of S'[j]
// are R'[lb, ub); ub comes from a galloping search from lb (one probe for a
// unique key). Counts, an exclusive scan and a write pass produce T in key
// order, ties in S' order then R' order.
#include "internal.hpp"

namespace gj {
namespace {

constexpr int kMergeItems = 16;
constexpr uint32_t kMergeTile = kBlock * kMergeItems;

// Ordered view of a key: the sign bit flipped, so unsigned order = signed order.
template <typename K>
__device__ __forceinline__ uint64_t ord(K k) {
    return digit_source<K>(k, kDigitOrdered);
}

// Number of S elements among the first d of the merged sequence (S before R
// on equal keys), for sorted r[0..m) and s[0..n).
template <typename K>
__device__ __forceinline__ uint32_t merge_split(const K *r, uint32_t m, const K *s, uint32_t n, uint32_t d) {
    uint32_t lo = d > m ? d - m : 0u, hi = d < n ? d : n;
    while (lo < hi) {
        const uint32_t a = (lo + hi) >> 1, b = d - a;
        // S[a] goes before R[b - 1] when its key is not greater: then a is too small
        if (ord<K>(s[a]) <= ord<K>(r[b - 1])) lo = a + 1;
        else hi = a;
    }
    return lo;
}

template <typename K>
__global__ void k_merge_diag(const K *__restrict__ r, uint32_t m, const K *__restrict__ s, uint32_t n,
                             uint32_t tiles, uint32_t *__restrict__ split) {
    const uint64_t total = (uint64_t)m + n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= tiles; t += gridDim.x * blockDim.x) {
        const uint64_t d = min<uint64_t>((uint64_t)t * kMergeTile, total);
        split[t] = merge_split<K>(r, m, s, n, (uint32_t)d);
    }
}

// lb[j] = lower bound of S'[j] in R', for the S rows of one merge tile.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_merge_lb(const K *__restrict__ r, uint32_t m, const K *__restrict__ s,
                                                     uint32_t n, const uint32_t *__restrict__ split,
                                                     uint32_t *__restrict__ lb) {
    __shared__ K s_r[kMergeTile];
    __shared__ K s_s[kMergeTile];
    const uint32_t t = blockIdx.x;
    const uint64_t total = (uint64_t)m + n;
    const uint32_t d0 = (uint32_t)min<uint64_t>((uint64_t)t * kMergeTile, total);
    const uint32_t d1 = (uint32_t)min<uint64_t>((uint64_t)d0 + kMergeTile, total);
    const uint32_t a0 = split[t], a1 = split[t + 1];
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t na = a1 - a0, nb = b1 - b0;  // na + nb = d1 - d0 <= kMergeTile
    for (uint32_t i = threadIdx.x; i < na; i += kBlock) s_s[i] = s[a0 + i];
    for (uint32_t i = threadIdx.x; i < nb; i += kBlock) s_r[i] = r[b0 + i];
    __syncthreads();
    const uint32_t dl = min(threadIdx.x * (uint32_t)kMergeItems, na + nb);
    const uint32_t dh = min(dl + (uint32_t)kMergeItems, na + nb);
    uint32_t a = merge_split<K>(s_r, nb, s_s, na, dl), b = dl - a;
    for (uint32_t d = dl; d < dh; ++d) {
        if (a < na && (b >= nb || ord<K>(s_s[a]) <= ord<K>(s_r[b]))) {
            lb[a0 + a] = b0 + b;
            ++a;
        } else {
            ++b;
        }
    }
}

// Matches of S'[j]: R'[lb, ub) with equal keys; ub by galloping from lb.
template <typename K>
__device__ __forceinline__ uint32_t match_end(const K *__restrict__ r, uint32_t m, uint32_t lb, K key) {
    if (lb >= m || r[lb] != key) return lb;
    uint32_t lo = lb + 1, step = 1;  // r[lo - 1] == key
    while (lo < m && r[lo] == key) {
        const uint32_t next = lo + step;
        if (next >= m || r[next] != key) {
            // the end lies in (lo, min(next, m)]: binary search
            uint32_t hi = next < m ? next : m;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (r[mid] == key) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        }
        lo = next + 1;
        step <<= 1;
    }
    return lo;
}

template <typename K>
__global__ void k_smj_count(const K *__restrict__ r, uint32_t m, const K *__restrict__ s, uint32_t n,
                            const uint32_t *__restrict__ lb, uint64_t *__restrict__ cnt) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        cnt[j] = match_end<K>(r, m, lb[j], s[j]) - lb[j];
}

struct SmjCols {
    int nr, ns;
    const void *rp[8];
    int rw[8];
    const void *sp[8];
    int sw[8];
    void *tr[8];
    void *ts[8];
    const int32_t *rrow;  // GFUR: R' row ids (payloads read from the original columns)
    const int32_t *srow;  // GFUR: S' row ids
};

__device__ __forceinline__ void smj_copy(void *dst, int w, uint64_t di, const void *src, uint64_t si) {
    if (w == 4) static_cast<uint32_t *>(dst)[di] = static_cast<const uint32_t *>(src)[si];
    else static_cast<uint64_t *>(dst)[di] = static_cast<const uint64_t *>(src)[si];
}

// One thread per S' row: its matches R'[lb, lb + c) go to output rows off[j] + k.
template <typename K>
__global__ void k_smj_write(const K *__restrict__ s, uint32_t n, const uint32_t *__restrict__ lb,
                            const uint64_t *__restrict__ off, const uint64_t *__restrict__ cnt, uint64_t t_rows,
                            K *__restrict__ tkey, SmjCols c) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const uint64_t o = off[j], k = cnt[j];
        if (k == 0) continue;
        const K key = s[j];
        const uint64_t sr = c.srow ? (uint64_t)c.srow[j] : (uint64_t)j;
        for (uint64_t q = 0; q < k; ++q) {
            const uint64_t p = o + q;
            if (p >= t_rows) break;  // never when the counts are right
            const uint64_t ri = (uint64_t)lb[j] + q;
            const uint64_t rr = c.rrow ? (uint64_t)c.rrow[ri] : ri;
            tkey[p] = key;
            for (int i = 0; i < c.nr; ++i) smj_copy(c.tr[i], c.rw[i], p, c.rp[i], rr);
            for (int i = 0; i < c.ns; ++i) smj_copy(c.ts[i], c.sw[i], p, c.sp[i], sr);
        }
    }
}

template <typename K>
int64_t smj_typed(Ctx &ctx, const JoinSide &R, const JoinSide &S, bool gfur, JoinOut *out) {
    hipStream_t st = ctx.stream;
    const K *rk = static_cast<const K *>(R.key);
    const K *sk = static_cast<const K *>(S.key);
    const uint32_t m = R.rows, n = S.rows;
    const uint64_t total = (uint64_t)m + n;
    const uint32_t tiles = (uint32_t)((total + kMergeTile - 1) / kMergeTile);
    uint32_t *split = ctx.scratch_n<uint32_t>((size_t)tiles + 1);
    uint32_t *lb = ctx.scratch_n<uint32_t>(n);
    GJ_LAUNCH("k_merge_diag", 16.0 * tiles, k_merge_diag<K>, dim3(std::min<uint32_t>(ceil_div_u32(tiles + 1, 256), 4096)),
              dim3(256), 0, st, rk, m, sk, n, tiles, split);
    GJ_LAUNCH("k_merge_lb", (double)total * sizeof(K) + 4.0 * n, k_merge_lb<K>, dim3(tiles), dim3(kBlock), 0, st, rk,
              m, sk, n, split, lb);
    uint64_t *cnt = ctx.scratch_n<uint64_t>((size_t)n + 1);
    const uint32_t grid = std::min<uint32_t>(ceil_div_u32(n, 256), 8192);
    GJ_LAUNCH("k_smj_count", (double)n * (sizeof(K) + 12.0), k_smj_count<K>, dim3(grid), dim3(256), 0, st, rk, m, sk,
              n, lb, cnt);
    uint64_t *total_rows = cnt + n;
    uint64_t *off = ctx.scratch_n<uint64_t>(n);
    scan_exclusive_u64(ctx, cnt, off, n, total_rows);
    const uint64_t T = read_back(total_rows, st);
    if (T == 0) return 0;
    out->key = ctx.output(T * sizeof(K));
    SmjCols c{};
    c.nr = R.n_pay;
    c.ns = S.n_pay;
    double pay = 0;
    for (int i = 0; i < R.n_pay; ++i) {
        c.rp[i] = R.pay[i];
        c.rw[i] = R.width[i];
        out->r[i] = ctx.output(T * (uint64_t)R.width[i]);
        c.tr[i] = out->r[i];
        pay += R.width[i];
    }
    for (int i = 0; i < S.n_pay; ++i) {
        c.sp[i] = S.pay[i];
        c.sw[i] = S.width[i];
        out->s[i] = ctx.output(T * (uint64_t)S.width[i]);
        c.ts[i] = out->s[i];
        pay += S.width[i];
    }
    c.rrow = gfur ? R.rowid : nullptr;
    c.srow = gfur ? S.rowid : nullptr;
    // algorithmic bytes: S keys, bounds, offsets, counts, payload reads, output rows
    const double bytes = (double)n * (sizeof(K) + 20.0) + (double)T * (2.0 * pay + sizeof(K)) +
                         (gfur ? 4.0 * ((double)n + (double)T) : 0.0);
    GJ_LAUNCH("k_smj_write", bytes, k_smj_write<K>, dim3(grid), dim3(256), 0, st, sk, n, lb, off, cnt, T,
              static_cast<K *>(out->key), c);
    return (int64_t)T;
}

}  // namespace

int64_t join_sort_merge(Ctx &ctx, int key_bytes, const JoinSide &R, const JoinSide &S, bool gfur, JoinOut *out) {
    return key_bytes == 4 ? smj_typed<int32_t>(ctx, R, S, gfur, out) : smj_typed<int64_t>(ctx, R, S, gfur, out);
}

}  // namespace gj
