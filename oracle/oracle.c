/*
 * Plain CPU oracle for the join and group-by hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. The GPU library never links,
 * calls or includes anything from here, and this file includes nothing from it.
 *
 * Every function computes the plain relational definition, using a library
 * sort (qsort) and binary search as its only building blocks. Nothing here is
 * blocked, partitioned or fused the way the GPU method is.
 *
 * Keys are 4-byte or 8-byte signed integers (key_bytes = 4 or 8). They are
 * widened to int64, which keeps equality and the signed order.
 *
 * Parity status of each function (pins live in tests/):
 *   oracle_join_pairs        pinned: brute-force nested loop, closed form for
 *                            PK-FK inputs, the sum over keys of |R_k|*|S_k|
 *   oracle_groupby           pinned: brute force per distinct key, bincount
 *                            closed form, sum invariants
 *   oracle_groupby64         pinned: brute force per distinct key over int64
 *                            values, np.add.at / minimum.at closed forms
 *   oracle_partition         pinned: Python's stable sort on tiny inputs,
 *                            permutation and order invariants
 *   oracle_hgb_ids           pinned: dictionary brute force, bijection invariant
 *   oracle_rows_fingerprint  pinned: equals the sum computed in Python
 *   oracle_join_fingerprint  pinned: equals the fingerprint of oracle_join_pairs
 *   oracle_hll_registers     pinned: union is the register-wise max, duplicates
 *                            change nothing, and the estimate built on it stays
 *                            within the sketch's published error bound
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t key;
    int64_t idx;
} kv_t;

static int64_t load_key(const void *keys, int key_bytes, int64_t i) {
    if (key_bytes == 4) return (int64_t)((const int32_t *)keys)[i];
    return ((const int64_t *)keys)[i];
}

static int cmp_kv(const void *a, const void *b) {
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/* R rows sorted by (key, row index): a sorted copy used as an index. */
static kv_t *sorted_index(const void *keys, int key_bytes, int64_t n) {
    kv_t *a = (kv_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(kv_t));
    if (!a) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = load_key(keys, key_bytes, i);
        a[i].idx = i;
    }
    qsort(a, (size_t)n, sizeof(kv_t), cmp_kv);
    return a;
}

/* First position p in a[0..n) with a[p].key >= k. */
static int64_t lower_bound(const kv_t *a, int64_t n, int64_t k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid].key < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/*
 * Inner equi-join R |><| S on key (Section 2.2): every pair (r, s) with
 * r.key == s.key, enumerated for s in S's input order and, for each s, r in
 * R's input order. Writes the matching row indices into out_r / out_s when
 * they are not NULL (capacity `cap` pairs). Returns the number of pairs, or -1
 * when memory runs out or the capacity is too small.
 */
int64_t oracle_join_pairs(int key_bytes, const void *r_key, int64_t n_r,
                          const void *s_key, int64_t n_s,
                          int64_t *out_r, int64_t *out_s, int64_t cap) {
    kv_t *idx = sorted_index(r_key, key_bytes, n_r);
    if (!idx) return -1;
    int64_t t = 0;
    for (int64_t j = 0; j < n_s; ++j) {
        int64_t k = load_key(s_key, key_bytes, j);
        for (int64_t p = lower_bound(idx, n_r, k); p < n_r && idx[p].key == k; ++p) {
            if (out_r) {
                if (t >= cap) { free(idx); return -1; }
                out_r[t] = idx[p].idx;
                out_s[t] = j;
            }
            ++t;
        }
    }
    free(idx);
    return t;
}

static inline uint64_t mix64(uint64_t z) {
    /* splitmix64 output function (Steele, Lea, Flood 2014). */
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Hash of one row: the row's column values (as 64-bit words) chained through mix64. */
static inline uint64_t row_hash_step(uint64_t h, uint64_t v) { return mix64(h ^ v); }

static uint64_t col_word(const void *col, int width, int64_t i) {
    if (width == 4) return (uint64_t)(int64_t)((const int32_t *)col)[i];
    return (uint64_t)((const int64_t *)col)[i];
}

/*
 * Order-independent fingerprint of a table: out[0] = number of rows,
 * out[1] = sum of H(row), out[2] = sum of H(row)^2, both modulo 2^64, where H
 * chains every column value of the row through mix64.
 */
void oracle_rows_fingerprint(const void *const *cols, const int32_t *widths, int32_t n_cols,
                             int64_t n, uint64_t out[3]) {
    uint64_t s1 = 0, s2 = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t h = 0x243F6A8885A308D3ull;
        for (int32_t c = 0; c < n_cols; ++c) h = row_hash_step(h, col_word(cols[c], widths[c], i));
        s1 += h;
        s2 += h * h;
    }
    out[0] = (uint64_t)n;
    out[1] = s1;
    out[2] = s2;
}

/*
 * Fingerprint of the join output T(key, r_1..r_cR, s_1..s_cS) without
 * materializing it: the same enumeration as oracle_join_pairs, with each
 * output row hashed as oracle_rows_fingerprint does. Payload widths are 4 or 8.
 */
int oracle_join_fingerprint(int key_bytes, const void *r_key, int64_t n_r,
                            const void *const *r_pay, const int32_t *r_w, int32_t c_r,
                            const void *s_key, int64_t n_s,
                            const void *const *s_pay, const int32_t *s_w, int32_t c_s,
                            uint64_t out[3]) {
    kv_t *idx = sorted_index(r_key, key_bytes, n_r);
    if (!idx) return -1;
    uint64_t t = 0, s1 = 0, s2 = 0;
    for (int64_t j = 0; j < n_s; ++j) {
        int64_t k = load_key(s_key, key_bytes, j);
        for (int64_t p = lower_bound(idx, n_r, k); p < n_r && idx[p].key == k; ++p) {
            uint64_t h = 0x243F6A8885A308D3ull;
            h = row_hash_step(h, (uint64_t)k);
            for (int32_t c = 0; c < c_r; ++c) h = row_hash_step(h, col_word(r_pay[c], r_w[c], idx[p].idx));
            for (int32_t c = 0; c < c_s; ++c) h = row_hash_step(h, col_word(s_pay[c], s_w[c], j));
            s1 += h;
            s2 += h * h;
            ++t;
        }
    }
    free(idx);
    out[0] = t;
    out[1] = s1;
    out[2] = s2;
    return 0;
}

/*
 * Grouped aggregation with one group key (Section 2.2): for every distinct key
 * k, in ascending signed order, COUNT(*) and, per value column, SUM (int64,
 * exact), MIN and MAX (int32). Output arrays have room for n groups;
 * out_sum/out_min/out_max are laid out column-major [n_vals][n].
 * Returns the number of groups, or -1 when memory runs out.
 */
int64_t oracle_groupby(int key_bytes, const void *keys, int64_t n,
                       const int32_t *const *vals, int32_t n_vals,
                       int64_t *out_key, int64_t *out_count,
                       int64_t *out_sum, int32_t *out_min, int32_t *out_max) {
    kv_t *a = sorted_index(keys, key_bytes, n);
    if (!a) return -1;
    int64_t g = 0;
    for (int64_t p = 0; p < n;) {
        int64_t q = p;
        while (q < n && a[q].key == a[p].key) ++q;
        out_key[g] = a[p].key;
        out_count[g] = q - p;
        for (int32_t v = 0; v < n_vals; ++v) {
            int64_t s = 0;
            int32_t mn = INT32_MAX, mx = INT32_MIN;
            for (int64_t r = p; r < q; ++r) {
                int32_t x = vals[v][a[r].idx];
                s += x;
                if (x < mn) mn = x;
                if (x > mx) mx = x;
            }
            out_sum[(int64_t)v * n + g] = s;
            out_min[(int64_t)v * n + g] = mn;
            out_max[(int64_t)v * n + g] = mx;
        }
        ++g;
        p = q;
    }
    free(a);
    return g;
}

/*
 * The same group-by over 8-byte value columns (Section 5.2 evaluates 8-byte
 * payloads): per distinct key, COUNT, SUM, MIN and MAX of int64 values. SUM is
 * taken modulo 2^64 (two's complement), which is exact whenever the true sum
 * fits in int64. Same output layout as oracle_groupby, with int64 minima and
 * maxima.
 */
int64_t oracle_groupby64(int key_bytes, const void *keys, int64_t n,
                         const int64_t *const *vals, int32_t n_vals,
                         int64_t *out_key, int64_t *out_count,
                         int64_t *out_sum, int64_t *out_min, int64_t *out_max) {
    kv_t *a = sorted_index(keys, key_bytes, n);
    if (!a) return -1;
    int64_t g = 0;
    for (int64_t p = 0; p < n;) {
        int64_t q = p;
        while (q < n && a[q].key == a[p].key) ++q;
        out_key[g] = a[p].key;
        out_count[g] = q - p;
        for (int32_t v = 0; v < n_vals; ++v) {
            uint64_t s = 0;
            int64_t mn = INT64_MAX, mx = INT64_MIN;
            for (int64_t r = p; r < q; ++r) {
                int64_t x = vals[v][a[r].idx];
                s += (uint64_t)x;
                if (x < mn) mn = x;
                if (x > mx) mx = x;
            }
            out_sum[(int64_t)v * n + g] = (int64_t)s;
            out_min[(int64_t)v * n + g] = mn;
            out_max[(int64_t)v * n + g] = mx;
        }
        ++g;
        p = q;
    }
    free(a);
    return g;
}

/* MurmurHash3 32-bit finalizer (Appleby), applied to the key's low word
 * (4-byte keys) or to the xor of its two words (8-byte keys). */
static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

static uint64_t digit_source(int64_t key, int key_bytes, int mode) {
    uint64_t u = (uint64_t)key;
    if (key_bytes == 4) u &= 0xFFFFFFFFull;
    if (mode == 1) {
        uint32_t w = key_bytes == 4 ? (uint32_t)u : (uint32_t)u ^ (uint32_t)(u >> 32);
        return (uint64_t)fmix32(w);
    }
    if (mode == 2) {
        /* order-preserving bits: flip the sign bit of the two's-complement word */
        return key_bytes == 4 ? (u ^ 0x80000000ull) : (u ^ 0x8000000000000000ull);
    }
    return u;
}

/* The digit source of one key (exposed so tests can pin the hash to its
 * published test vectors). */
uint64_t oracle_digit_source(int key_bytes, int64_t key, int mode) {
    return digit_source(key, key_bytes, mode);
}

/* HyperLogLog registers (Flajolet, Fusy, Gandouet and Meunier, 2007) over the
 * 32-bit MurmurHash3 finalizer of the keys (digit source mode 1): the top
 * `bits` bits of a key's hash name its register, and the register keeps the
 * largest position, counted from 1, of the first 1 bit among the remaining
 * 32 - bits bits (33 - bits when they are all zero). regs has 2^bits entries. */
void oracle_hll_registers(int key_bytes, const void *keys, int64_t n, int bits, uint32_t *regs) {
    const uint32_t m = 1u << bits;
    for (uint32_t j = 0; j < m; ++j) regs[j] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t h = (uint32_t)digit_source(load_key(keys, key_bytes, i), key_bytes, 1);
        const uint32_t j = h >> (32 - bits);
        uint32_t rho = 1;
        for (int b = 31 - bits; b >= 0 && !((h >> b) & 1u); --b) ++rho;
        if (rho > regs[j]) regs[j] = rho;
    }
}

typedef struct {
    uint64_t digit;
    int64_t idx;
} di_t;

static int cmp_di(const void *a, const void *b) {
    const di_t *x = (const di_t *)a, *y = (const di_t *)b;
    if (x->digit < y->digit) return -1;
    if (x->digit > y->digit) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/*
 * The radix-partition primitive of Section 2.3 as a definition: the digit of a
 * row is bits [lo, lo+bits) of its digit source (mode 0: the key's unsigned
 * bit pattern; mode 1: the 32-bit MurmurHash3 finalizer of the key; mode 2:
 * the key with its sign bit flipped, which orders signed keys). The output
 * order is the rows sorted by digit, rows with equal digits kept in input
 * order. perm[i] = input row placed at output position i; hist[d] = rows with
 * digit d (2^bits entries).
 */
int oracle_partition(int key_bytes, const void *keys, int64_t n, int lo, int bits, int mode,
                     int64_t *perm, int64_t *hist) {
    di_t *a = (di_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(di_t));
    if (!a) return -1;
    uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    int64_t nb = (int64_t)1 << bits;
    for (int64_t d = 0; d < nb; ++d) hist[d] = 0;
    for (int64_t i = 0; i < n; ++i) {
        a[i].digit = (digit_source(load_key(keys, key_bytes, i), key_bytes, mode) >> lo) & mask;
        a[i].idx = i;
        hist[a[i].digit] += 1;
    }
    qsort(a, (size_t)n, sizeof(di_t), cmp_di);
    for (int64_t i = 0; i < n; ++i) perm[i] = a[i].idx;
    free(a);
    return 0;
}

/*
 * Group-ID assignment of the optimized hash group-by (Algorithm 1, stage 1),
 * run sequentially over i = 0..n-1: the first row with a given key inserts it
 * and takes the next group ID; every row records in gid_loc the row index
 * with which its key was inserted. gid[i] is set only for inserting rows and
 * is -1 elsewhere. Returns the number of groups, or -1 when memory runs out.
 * A sorted index stands in for the hash table; it answers the same question
 * (the first row holding a key).
 */
int64_t oracle_hgb_ids(int key_bytes, const void *keys, int64_t n, int64_t *gid, int64_t *gid_loc) {
    kv_t *a = sorted_index(keys, key_bytes, n);
    if (!a) return -1;
    int64_t g = 0;
    for (int64_t i = 0; i < n; ++i) gid[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = load_key(keys, key_bytes, i);
        int64_t first = a[lower_bound(a, n, k)].idx; /* smallest row index holding k */
        gid_loc[i] = first;
        if (first == i) gid[i] = g++;
    }
    free(a);
    return g;
}
