// C ABI of libgj: argument checks, planning (bits, passes, materialization),
// scratch management and dispatch to the kernel drivers.
#include <string.h>

#include <algorithm>

#include <string>
#include <vector>

#include "internal.hpp"

namespace {

thread_local std::string g_last_error;

using gj::fail;

constexpr int64_t kMaxRows = 2147483647LL;

int dtype_bytes(int32_t dt) { return dt == GJ_I32 ? 4 : (dt == GJ_I64 ? 8 : 0); }

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

void check_col(const gj_col &c, int64_t n, const char *what) {
    gj::require(dtype_bytes(c.dtype) != 0, std::string(what) + ": dtype must be GJ_I32 or GJ_I64");
    gj::require(n == 0 || c.data != nullptr, std::string(what) + ": null data");
}

void check_rel(const gj_rel *r, const char *what) {
    gj::require(r != nullptr, std::string(what) + ": null relation");
    gj::require(r->n_rows >= 0, std::string(what) + ": negative row count");
    gj::require(r->n_rows <= kMaxRows, std::string(what) + ": more than 2^31-1 rows", GJ_EOVERFLOW);
    gj::require(r->n_payloads >= 0 && r->n_payloads <= 8, std::string(what) + ": 0..8 payload columns");
    gj::require(r->n_payloads == 0 || r->payloads != nullptr, std::string(what) + ": null payload array");
    check_col(r->key, r->n_rows, what);
    for (int i = 0; i < r->n_payloads; ++i) check_col(r->payloads[i], r->n_rows, what);
}

}  // namespace

namespace gj {
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }
}  // namespace gj

extern "C" {

const char *gj_last_error(void) { return g_last_error.c_str(); }

const char *gj_version(void) { return "gj 0.1 (gfx950)"; }

int gj_partition(gj_col key, const gj_col *cols, int32_t n_cols, int64_t n_rows, int32_t bit_lo,
                 int32_t bits, int32_t passes, int32_t mode, void *out_key, void *const *out_cols,
                 void *out_rowid, int32_t *out_offsets, const gj_allocator *alloc, void *stream) {
    try {
        g_last_error.clear();
        gj::require(n_rows >= 0, "negative row count");
        gj::require(n_rows <= kMaxRows, "more than 2^31-1 rows", GJ_EOVERFLOW);
        gj::require(n_cols >= 0 && n_cols <= 8, "0..8 columns");
        gj::require(n_cols == 0 || (cols && out_cols), "null column arrays");
        gj::require(bits >= 1 && bits <= 16, "bits must be 1..16");
        gj::require(mode >= 0 && mode <= 2, "bad digit mode");
        const int kb = dtype_bytes(key.dtype);
        check_col(key, n_rows, "key");
        gj::require(bit_lo >= 0 && bit_lo + bits <= 8 * kb, "digit bits outside the key");
        gj::require(n_rows == 0 || out_key, "null output key");
        if (passes == 0) passes = bits > 8 ? 2 : 1;
        gj::require(passes == 1 || passes == 2, "passes must be 0, 1 or 2");
        gj::require(bits <= 8 * passes, "at most 8 bits per pass");
        gj::Ctx ctx(alloc, (hipStream_t)stream);
        gj::PartCols pc;
        pc.n = n_cols;
        for (int i = 0; i < n_cols; ++i) {
            check_col(cols[i], n_rows, "column");
            gj::require(n_rows == 0 || out_cols[i], "null output column");
            pc.in[i] = cols[i].data;
            pc.out[i] = out_cols[i];
            pc.width[i] = dtype_bytes(cols[i].dtype);
        }
        pc.gen_rowid = out_rowid != nullptr;
        pc.rowid_out = out_rowid;
        uint32_t *poff = out_offsets ? reinterpret_cast<uint32_t *>(out_offsets)
                                     : ctx.scratch_n<uint32_t>(((size_t)1 << bits) + 1);
        gj::partition_run(ctx, kb, key.data, out_key, pc, (uint32_t)n_rows, bit_lo, bits, passes, mode, poff);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

int gj_join(const gj_rel *R, const gj_rel *S, const gj_join_opts *opts, const gj_allocator *alloc,
            void *stream, gj_join_out *out) {
    try {
        g_last_error.clear();
        gj::require(out != nullptr, "null output");
        check_rel(R, "R");
        check_rel(S, "S");
        gj::require(R->key.dtype == S->key.dtype, "R.key and S.key dtypes differ");
        gj::require(R->n_payloads == 0 || out->r_payloads, "null r_payloads array");
        gj::require(S->n_payloads == 0 || out->s_payloads, "null s_payloads array");
        gj_join_opts o{};
        if (opts) o = *opts;
        gj::require(o.mat >= 0 && o.mat <= 2, "bad materialization");
        gj::require(o.passes >= 0 && o.passes <= 2, "passes must be 0, 1 or 2");
        gj::require(o.radix_bits >= 0 && o.radix_bits <= 16, "radix_bits must be 0..16");
        gj::require(o.block_size == 0 || o.block_size == gj::kBlock, "block_size must be 0 or 256");
        gj::check_join_lds_budget(o.lds_budget, dtype_bytes(R->key.dtype));
        gj::require(o.flags == 0, "flags must be 0");
        gj::require(o.algo >= GJ_JOIN_AUTO && o.algo <= GJ_JOIN_SMJ, "bad join algorithm");

        out->n_rows = 0;
        out->key = nullptr;
        for (int i = 0; i < R->n_payloads; ++i) out->r_payloads[i] = nullptr;
        for (int i = 0; i < S->n_payloads; ++i) out->s_payloads[i] = nullptr;
        if (R->n_rows == 0 || S->n_rows == 0) return GJ_OK;

        const int kb = dtype_bytes(R->key.dtype);
        int mat = o.mat;
        if (mat == GJ_MAT_AUTO) {
            // the selector picks among partitioned GFTR / GFUR and sort-merge GFTR;
            // an algorithm the caller fixed keeps its own materialization choice
            float f[12];
            gj::features_join(f, (double)R->n_rows, (double)S->n_rows, kb, R->n_payloads, S->n_payloads,
                              o.match_ratio_hint, o.skew_hint);
            const int c = gj::select_algorithm(f, 0, nullptr);
            mat = c == 1 && o.algo != GJ_JOIN_SMJ ? GJ_MAT_GFUR : GJ_MAT_GFTR;
            if (o.algo == GJ_JOIN_AUTO) o.algo = c == 6 ? GJ_JOIN_SMJ : GJ_JOIN_PHJ;
        }
        const bool gfur = (mat == GJ_MAT_GFUR);
        int r_pay_bytes = 0;
        for (int i = 0; i < R->n_payloads; ++i) r_pay_bytes += dtype_bytes(R->payloads[i].dtype);
        const int r_block = o.lds_budget ? o.lds_budget
                                         : gj::join_default_r_block((uint64_t)R->n_rows, kb, gfur, r_pay_bytes);
        const int bits = o.radix_bits ? o.radix_bits : gj::join_default_bits((uint64_t)R->n_rows, r_block);
        int passes = o.passes ? o.passes : (bits > 8 ? 2 : 1);
        gj::require(bits <= 8 * passes, "at most 8 bits per pass");
        if (passes == 2 && bits < 2) passes = 1;

        gj::Ctx ctx(alloc, (hipStream_t)stream);
        gj::JoinSide side[2];
        const gj_rel *rel[2] = {R, S};
        if (o.algo == GJ_JOIN_SMJ) {
            // transformation: full-key LSD radix sort of (key, payloads) or (key, row id)
            for (int t = 0; t < 2; ++t) {
                const gj_rel *X = rel[t];
                const uint32_t n = (uint32_t)X->n_rows;
                gj::JoinSide &js = side[t];
                js.key = ctx.scratch((size_t)n * kb);
                js.rows = n;
                js.n_pay = X->n_payloads;
                js.poff = nullptr;
                gj::PartCols pc;
                for (int i = 0; i < X->n_payloads; ++i) js.width[i] = dtype_bytes(X->payloads[i].dtype);
                if (!gfur) {
                    pc.n = X->n_payloads;
                    for (int i = 0; i < X->n_payloads; ++i) {
                        pc.in[i] = X->payloads[i].data;
                        pc.width[i] = js.width[i];
                        pc.out[i] = ctx.scratch((size_t)n * js.width[i]);
                        js.pay[i] = pc.out[i];
                    }
                    js.rowid = nullptr;
                } else {
                    for (int i = 0; i < X->n_payloads; ++i) js.pay[i] = X->payloads[i].data;
                    pc.gen_rowid = true;
                    pc.rowid_out = ctx.scratch_n<int32_t>(n);
                    js.rowid = static_cast<const int32_t *>(pc.rowid_out);
                }
                gj::sort_run(ctx, kb, X->key.data, const_cast<void *>(js.key), pc, n);
            }
            gj::JoinOut jo{};
            const int64_t T = gj::join_sort_merge(ctx, kb, side[0], side[1], gfur, &jo);
            out->n_rows = T;
            if (T > 0) {
                out->key = jo.key;
                for (int i = 0; i < R->n_payloads; ++i) out->r_payloads[i] = jo.r[i];
                for (int i = 0; i < S->n_payloads; ++i) out->s_payloads[i] = jo.s[i];
            }
            ctx.commit();
            return GJ_OK;
        }
        // Join digits are the low key bits (dense keys spread evenly over them).
        // Keys whose low bits barely vary (multiples of a power of two, say) pile
        // into a few partitions: when the largest R partition holds more than four
        // times the mean plus a build block, both sides are partitioned again on
        // hashed keys, into the same buffers. The result is the same either way.
        gj::JoinStats st;
        st.check_spread = true;
        const uint64_t mean_r = ((uint64_t)R->n_rows + (1ull << bits) - 1) >> bits;
        st.spread_limit = (uint32_t)std::min<uint64_t>(4 * mean_r + (uint64_t)r_block, 0xFFFFFFFFull);
        for (int t = 0; t < 2; ++t) {
            const gj_rel *X = rel[t];
            const uint32_t n = (uint32_t)X->n_rows;
            gj::JoinSide &js = side[t];
            js.key = ctx.scratch((size_t)n * kb);
            js.rows = n;
            js.n_pay = X->n_payloads;
            for (int i = 0; i < X->n_payloads; ++i) js.width[i] = dtype_bytes(X->payloads[i].dtype);
            if (!gfur) {
                for (int i = 0; i < X->n_payloads; ++i) js.pay[i] = ctx.scratch((size_t)n * js.width[i]);
                js.rowid = nullptr;
            } else {
                for (int i = 0; i < X->n_payloads; ++i) js.pay[i] = X->payloads[i].data;
                js.rowid = ctx.scratch_n<int32_t>(n);
            }
            js.poff = ctx.scratch_n<uint32_t>(((size_t)1 << bits) + 1);
        }
        gj::JoinOut jo{};
        int64_t T = -1;
        for (int digit_mode = gj::kDigitBits; T < 0; digit_mode = gj::kDigitHash) {
            for (int t = 0; t < 2; ++t) {
                const gj_rel *X = rel[t];
                gj::JoinSide &js = side[t];
                gj::PartCols pc;
                if (!gfur) {
                    pc.n = X->n_payloads;
                    for (int i = 0; i < X->n_payloads; ++i) {
                        pc.in[i] = X->payloads[i].data;
                        pc.width[i] = js.width[i];
                        pc.out[i] = const_cast<void *>(js.pay[i]);
                    }
                } else {
                    pc.gen_rowid = true;
                    pc.rowid_out = const_cast<int32_t *>(js.rowid);
                }
                gj::partition_run(ctx, kb, X->key.data, const_cast<void *>(js.key), pc, js.rows, 0, bits, passes,
                                  digit_mode, const_cast<uint32_t *>(js.poff));
            }
            st.hashed_digits = digit_mode == gj::kDigitHash;
            st.check_spread = !st.hashed_digits;
            T = gj::join_partitioned(ctx, kb, side[0], side[1], bits, r_block, gfur, &jo, nullptr, 0, nullptr,
                                     nullptr, &st);
        }
        out->n_rows = T;
        if (T > 0) {
            out->key = jo.key;
            for (int i = 0; i < R->n_payloads; ++i) out->r_payloads[i] = jo.r[i];
            for (int i = 0; i < S->n_payloads; ++i) out->s_payloads[i] = jo.s[i];
        }
        ctx.commit();
        return GJ_OK;
    } catch (const gj::Error &e) {
        if (out) {
            out->n_rows = 0;
            out->key = nullptr;
        }
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

int gj_join_batch(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts,
                  const gj_allocator *alloc, void *stream, gj_join_out *out, int64_t *out_offsets) {
    try {
        g_last_error.clear();
        gj::require(R && S && out && out_offsets, "null argument");
        const int32_t n = R->n_instances;
        gj::require(n >= 1 && S->n_instances == n, "R and S need the same positive instance count");
        gj::require(R->offsets && S->offsets, "null offsets");
        gj::require(R->key.dtype == S->key.dtype, "R.key and S.key dtypes differ");
        const gj_rel_batch *rel[2] = {R, S};
        for (int t = 0; t < 2; ++t) {
            const gj_rel_batch *X = rel[t];
            gj::require(X->offsets[0] == 0, "offsets[0] must be 0");
            for (int i = 0; i < n; ++i) gj::require(X->offsets[i + 1] >= X->offsets[i], "offsets must not decrease");
            gj::require(X->offsets[n] <= kMaxRows, "a side of the batch has more than 2^31-1 rows", GJ_EOVERFLOW);
            gj::require(X->n_payloads >= 0 && X->n_payloads <= 8, "0..8 payload columns");
            gj::require(X->n_payloads == 0 || X->payloads, "null payload array");
            check_col(X->key, X->offsets[n], "key");
            for (int i = 0; i < X->n_payloads; ++i) check_col(X->payloads[i], X->offsets[n], "payload");
        }
        gj::require(R->n_payloads == 0 || out->r_payloads, "null r_payloads array");
        gj::require(S->n_payloads == 0 || out->s_payloads, "null s_payloads array");
        gj_join_opts o{};
        if (opts) o = *opts;
        gj::require(o.mat >= 0 && o.mat <= 2, "bad materialization");
        gj::check_join_lds_budget(o.lds_budget, dtype_bytes(R->key.dtype));
        gj::require(o.flags == 0, "flags must be 0");
        gj::require(o.algo == GJ_JOIN_AUTO || o.algo == GJ_JOIN_PHJ, "batches run the partitioned hash join only",
                    GJ_EUNSUPPORTED);
        out->n_rows = 0;
        out->key = nullptr;
        for (int i = 0; i < R->n_payloads; ++i) out->r_payloads[i] = nullptr;
        for (int i = 0; i < S->n_payloads; ++i) out->s_payloads[i] = nullptr;
        for (int i = 0; i <= n; ++i) out_offsets[i] = 0;
        const uint32_t nr = (uint32_t)R->offsets[n], ns = (uint32_t)S->offsets[n];
        if (nr == 0 || ns == 0) return GJ_OK;

        const int kb = dtype_bytes(R->key.dtype);
        const bool gfur = (o.mat == GJ_MAT_GFUR);
        const int r_block = o.lds_budget ? o.lds_budget : 4096;
        const uint64_t target = (uint64_t)std::max(1, r_block / 2);
        std::vector<uint8_t> bits(n);
        std::vector<uint32_t> roff(n + 1), soff(n + 1);
        for (int i = 0; i < n; ++i) {
            const uint64_t rows = (uint64_t)(R->offsets[i + 1] - R->offsets[i]);
            bits[i] = (uint8_t)std::min(8, ceil_log2((rows + target - 1) / target));
        }
        for (int i = 0; i <= n; ++i) {
            roff[i] = (uint32_t)R->offsets[i];
            soff[i] = (uint32_t)S->offsets[i];
        }
        gj::Ctx ctx(alloc, (hipStream_t)stream);
        hipStream_t st = (hipStream_t)stream;
        uint8_t *d_bits = static_cast<uint8_t *>(ctx.scratch(n));
        uint32_t *d_off[2] = {ctx.scratch_n<uint32_t>(n + 1), ctx.scratch_n<uint32_t>(n + 1)};
        GJ_HIP(hipMemcpyAsync(d_bits, bits.data(), n, hipMemcpyHostToDevice, st));
        GJ_HIP(hipMemcpyAsync(d_off[0], roff.data(), 4ull * (n + 1), hipMemcpyHostToDevice, st));
        GJ_HIP(hipMemcpyAsync(d_off[1], soff.data(), 4ull * (n + 1), hipMemcpyHostToDevice, st));

        gj::JoinSide side[2];
        for (int t = 0; t < 2; ++t) {
            const gj_rel_batch *X = rel[t];
            const uint32_t rows = (uint32_t)X->offsets[n];
            gj::PartCols pc;
            void *kout = ctx.scratch((size_t)rows * kb);
            gj::JoinSide &js = side[t];
            js.key = kout;
            js.rows = rows;
            js.n_pay = X->n_payloads;
            for (int i = 0; i < X->n_payloads; ++i) js.width[i] = dtype_bytes(X->payloads[i].dtype);
            if (!gfur) {
                pc.n = X->n_payloads;
                for (int i = 0; i < X->n_payloads; ++i) {
                    pc.in[i] = X->payloads[i].data;
                    pc.width[i] = js.width[i];
                    pc.out[i] = ctx.scratch((size_t)rows * js.width[i]);
                    js.pay[i] = pc.out[i];
                }
                js.rowid = nullptr;
            } else {
                pc.gen_rowid = true;
                pc.rowid_out = ctx.scratch((size_t)rows * 4);
                for (int i = 0; i < X->n_payloads; ++i) js.pay[i] = X->payloads[i].data;
                js.rowid = static_cast<const int32_t *>(pc.rowid_out);
            }
            uint32_t *poff = ctx.scratch_n<uint32_t>(((size_t)n << 8) + 1);
            js.poff = poff;
            gj::partition_run_segments(ctx, kb, X->key.data, kout, pc, rows, d_off[t], (uint32_t)n, d_bits, poff);
        }
        uint64_t *inst_off = ctx.scratch_n<uint64_t>(n + 1);
        gj::JoinOut jo{};
        const int64_t T = gj::join_partitioned(ctx, kb, side[0], side[1], 0, r_block, gfur, &jo, d_bits, (uint32_t)n,
                                               inst_off);
        std::vector<uint64_t> h(n + 1);
        GJ_HIP(hipMemcpyAsync(h.data(), inst_off, 8ull * (n + 1), hipMemcpyDeviceToHost, st));
        GJ_HIP(hipStreamSynchronize(st));
        for (int i = 0; i <= n; ++i) out_offsets[i] = (int64_t)h[i];
        out->n_rows = T;
        if (T > 0) {
            out->key = jo.key;
            for (int i = 0; i < R->n_payloads; ++i) out->r_payloads[i] = jo.r[i];
            for (int i = 0; i < S->n_payloads; ++i) out->s_payloads[i] = jo.s[i];
        }
        ctx.commit();
        return GJ_OK;
    } catch (const gj::Error &e) {
        if (out) {
            out->n_rows = 0;
            out->key = nullptr;
        }
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

int gj_groupby(gj_col key, const gj_col *vals, int32_t n_vals, int64_t n_rows, const gj_agg *aggs,
               int32_t n_aggs, const gj_groupby_opts *opts, const gj_allocator *alloc, void *stream,
               gj_groupby_out *out) {
    try {
        g_last_error.clear();
        gj::require(out != nullptr, "null output");
        gj::require(n_rows >= 0, "negative row count");
        gj::require(n_rows <= kMaxRows, "more than 2^31-1 rows", GJ_EOVERFLOW);
        check_col(key, n_rows, "key");
        gj::require(n_vals >= 0 && n_vals <= 8, "0..8 value columns");
        gj::require(n_vals == 0 || vals != nullptr, "null value array");
        for (int i = 0; i < n_vals; ++i) check_col(vals[i], n_rows, "value");
        gj::require(n_aggs >= 1 && n_aggs <= 16, "1..16 aggregates");
        gj::require(aggs != nullptr && out->aggs != nullptr, "null aggregate arrays");
        for (int j = 0; j < n_aggs; ++j) {
            gj::require(aggs[j].op >= GJ_SUM && aggs[j].op <= GJ_MAX, "unknown aggregate");
            gj::require(aggs[j].op == GJ_COUNT || (aggs[j].col >= 0 && aggs[j].col < n_vals),
                        "aggregate column out of range");
        }
        gj_groupby_opts o{};
        if (opts) o = *opts;
        gj::require(o.algo >= GJ_GB_AUTO && o.algo <= GJ_GB_SORT_DE, "bad group-by algorithm");
        gj::require(o.mat >= 0 && o.mat <= 2, "bad materialization");
        gj::require(o.radix_bits >= 0 && o.radix_bits <= 16, "radix_bits must be 0..16");
        gj::require(o.block_size == 0 || o.block_size == gj::kBlock, "block_size must be 0 or 256");
        gj::require(o.lds_budget >= 0, "negative lds_budget");
        gj::require(o.ht_occupancy >= 0.0f && o.ht_occupancy <= 64.0f, "ht_occupancy must be 0..64");

        out->n_groups = 0;
        out->key = nullptr;
        for (int j = 0; j < n_aggs; ++j) out->aggs[j] = nullptr;
        if (n_rows == 0) return GJ_OK;

        const int kb = dtype_bytes(key.dtype);
        const uint32_t n = (uint32_t)n_rows;
        const bool gfur = (o.mat == GJ_MAT_GFUR);
        int algo = o.algo;
        gj::ValCols vcols;
        vcols.n = n_vals;
        for (int i = 0; i < n_vals; ++i) {
            vcols.col[i] = vals[i].data;
            vcols.width[i] = dtype_bytes(vals[i].dtype);
        }

        gj::Ctx ctx(alloc, (hipStream_t)stream);
        // the group count decides the algorithm and the partition passes: estimate it
        double g_est = 0.0;
        int varying = 0;
        // a partition group-by (chosen, or possibly chosen) takes its first pass's
        // histogram from the same read of the keys
        const uint32_t *hist8 = nullptr;
        const bool want_hist = algo == GJ_GB_AUTO || (algo == GJ_GB_PARTITION && o.radix_bits == 0);
        if (algo == GJ_GB_AUTO || algo == GJ_GB_HASH || algo == GJ_GB_SORT_DE ||
            (algo == GJ_GB_PARTITION && o.radix_bits == 0))
            g_est = gj::estimate_groups(ctx, kb, key.data, n, &varying, want_hist ? &hist8 : nullptr);
        if (algo == GJ_GB_AUTO) {
            float f[12];
            gj::features_groupby(f, (double)n, kb, n_vals, g_est, varying, o.skew_hint,
                                 (double)gj::hgb_record_bytes(aggs, n_aggs, vcols.width));
            const int c = gj::select_algorithm(f, 1, nullptr);
            algo = c == 2 ? GJ_GB_HASH : c == 3 ? GJ_GB_SORT : c == 5 ? GJ_GB_SORT_DE : GJ_GB_PARTITION;
        }
        void *okey = nullptr;
        void *oaggs[16] = {nullptr};
        int64_t g = -1;
        if (algo == GJ_GB_PARTITION) {
            int bits = o.radix_bits;
            if (bits == 0) {
                // One pass (at most 8 bits, partitions of at least 2048 rows) whenever
                // the estimated groups leave about 1000 or fewer keys per partition.
                // Up to ~128 groups, 8 bits leave about one group per partition, which
                // aggregates in registers. Beyond that, about sqrt(g) partitions of
                // sqrt(g) groups: a handful of groups per partition would make the
                // LDS record updates collide within a wave, and fewer bits also make
                // the scatter's digits longer. Past 2^18 groups, about 512 groups per
                // partition (fewer bits than partitions of 2048 rows would take),
                // within the 4096 keys a partition's discovery table holds.
                const int row_bits = std::min(16, std::max(1, ceil_log2((n + 2047) / 2048)));
                if (g_est <= 128.0) {
                    bits = std::min(row_bits, 8);
                } else if (g_est <= (double)(1u << 18)) {
                    const int half = (ceil_log2((uint64_t)g_est) + 1) / 2;
                    bits = std::min(row_bits, std::max(1, std::min(8, half)));
                } else {
                    const int g_bits = ceil_log2((uint64_t)(g_est / 512.0));
                    bits = std::max(1, std::min({16, row_bits, std::max(9, g_bits)}));
                }
            }
            int fell_back = 0;
            g = gj::groupby_partition(ctx, kb, key.data, vcols, n, aggs, n_aggs, gfur, bits, &okey, oaggs,
                                      &fell_back, hist8);
            if (fell_back) algo = GJ_GB_HASH;  // too many distinct keys per partition
        }
        if (algo == GJ_GB_HASH)
            g = gj::groupby_hash(ctx, kb, key.data, vcols, n, aggs, n_aggs, o.lds_budget, g_est,
                                 o.ht_occupancy, &okey, oaggs);
        else if (algo == GJ_GB_SORT)
            g = gj::groupby_sort(ctx, kb, key.data, vcols, n, aggs, n_aggs, gfur, &okey, oaggs);
        else if (algo == GJ_GB_SORT_DE)
            g = gj::groupby_sort_de(ctx, kb, key.data, vcols, n, aggs, n_aggs, g_est, o.ht_occupancy, &okey,
                                    oaggs);
        out->n_groups = g;
        out->key = okey;
        for (int j = 0; j < n_aggs; ++j) out->aggs[j] = oaggs[j];
        ctx.commit();
        return GJ_OK;
    } catch (const gj::Error &e) {
        if (out) {
            out->n_groups = 0;
            out->key = nullptr;
        }
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

int gj_join_features(const gj_rel *R, const gj_rel *S, const gj_join_opts *opts, float features[12]) {
    try {
        g_last_error.clear();
        gj::require(features != nullptr, "null features");
        check_rel(R, "R");
        check_rel(S, "S");
        gj_join_opts o{};
        if (opts) o = *opts;
        gj::features_join(features, (double)R->n_rows, (double)S->n_rows, dtype_bytes(R->key.dtype), R->n_payloads,
                          S->n_payloads, o.match_ratio_hint, o.skew_hint);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

int gj_groupby_features(gj_col key, const gj_col *vals, int32_t n_vals, const gj_agg *aggs, int32_t n_aggs,
                        int64_t n_rows, const gj_groupby_opts *opts, const gj_allocator *alloc, void *stream,
                        float features[12]) {
    try {
        g_last_error.clear();
        gj::require(features != nullptr, "null features");
        gj::require(n_rows >= 0, "negative row count");
        gj::require(n_rows <= kMaxRows, "more than 2^31-1 rows", GJ_EOVERFLOW);
        gj::require(n_vals >= 0 && n_vals <= 8, "0..8 value columns");
        gj::require(n_vals == 0 || vals != nullptr, "null value array");
        check_col(key, n_rows, "key");
        int vw[8] = {0};
        for (int i = 0; i < n_vals; ++i) {
            check_col(vals[i], n_rows, "value");
            vw[i] = dtype_bytes(vals[i].dtype);
        }
        gj::require(n_aggs >= 1 && n_aggs <= 16 && aggs != nullptr, "1..16 aggregates");
        for (int j = 0; j < n_aggs; ++j) {
            gj::require(aggs[j].op >= GJ_SUM && aggs[j].op <= GJ_MAX, "unknown aggregate");
            gj::require(aggs[j].op == GJ_COUNT || (aggs[j].col >= 0 && aggs[j].col < n_vals),
                        "aggregate column out of range");
        }
        gj_groupby_opts o{};
        if (opts) o = *opts;
        const int kb = dtype_bytes(key.dtype);
        gj::Ctx ctx(alloc, (hipStream_t)stream);
        int varying = 0;
        // the same sketch kernel gj_groupby runs for these options (with the
        // per-chunk hash histogram for a partition pass, which is dropped here)
        const bool want_hist = o.algo == GJ_GB_AUTO || (o.algo == GJ_GB_PARTITION && o.radix_bits == 0);
        const uint32_t *hist8 = nullptr;
        const double g_est =
            gj::estimate_groups(ctx, kb, key.data, (uint32_t)n_rows, &varying, want_hist ? &hist8 : nullptr);
        gj::features_groupby(features, (double)n_rows, kb, n_vals, g_est, varying, o.skew_hint,
                             (double)gj::hgb_record_bytes(aggs, n_aggs, vw));
        return GJ_OK;
    } catch (const gj::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::exception &e) {
        return fail(GJ_EHIP, e.what());
    }
}

}  // extern "C"
