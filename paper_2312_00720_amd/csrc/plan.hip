// Batch plans: a batch of independent join instances whose whole execution is
// fixed in advance, so that it can be captured once into a HIP graph and replayed
// with a single launch.
//
// Creating a plan validates the batch, picks each instance's parameters (partition
// bits, LDS bucket count: the built-in rule or an autotuned table per size class),
// cuts the instances into consecutive groups of at most 2^30 rows per side, and
// then runs the enqueue code once with launches switched off and scratch served by
// a measuring arena. That dry run yields the exact scratch size and the number of
// launches; the plan allocates the arena, the per-group device parameters and the
// output columns, and uploads the parameters. A run enqueues, per group: the
// segmented partition of R and S (one pass, instance = segment), the work-unit
// count and scan, the count pass, the scan of the per-wave counts, the per-instance
// output offsets and the write pass. No step reads device memory on the host; the
// count and write passes are persistent workgroups that loop over the unit count
// held in device memory, and output rows land at (group base + scanned position),
// where each group's base is the previous one's base plus its row count, again in
// device memory.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace gj {
thread_local bool g_dry_run = false;
thread_local int64_t g_dry_launches = 0;
}  // namespace gj

namespace {

using gj::Error;
using gj::require;

constexpr int64_t kMaxRows = 2147483647LL;
constexpr int64_t kGroupRows = 1LL << 30;
constexpr int kDefaultPartLog2 = 11;
constexpr uint32_t kUnitFactor = 2;  // room for R partitions of up to twice the build block

int dtype_bytes(int32_t dt) { return dt == GJ_I32 ? 4 : (dt == GJ_I64 ? 8 : 0); }

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

int floor_log2(uint64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

struct Group {
    uint32_t i0, i1;           // instances [i0, i1)
    int64_t r0, s0;            // first row of the group in the batch columns
    uint32_t rows_r, rows_s;
    uint32_t cap_units;
    uint64_t expect_rows;
    uint8_t *d_bits, *d_bshift;  // per instance of the group
    uint32_t *d_off[2];          // instance row offsets relative to the group (n + 1)
};

// Turns off launches for a scope and counts them (the plan's dry run).
struct DryRun {
    DryRun() {
        gj::g_dry_run = true;
        gj::g_dry_launches = 0;
    }
    ~DryRun() { gj::g_dry_run = false; }
};

struct VariantScope {
    explicit VariantScope(int v) { gj::set_scatter_variant(v); }
    ~VariantScope() { gj::set_scatter_variant(0); }
};

}  // namespace

struct gj_plan {
    int kind = 0;  // 0: join batch, 1: group-by batch
    gj_allocator alloc{};
    bool has_alloc = false;
    std::vector<void *> blocks;
    gj::Arena arena;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t launches = 0, output_bytes = 0, cap_units_total = 0;

    int n = 0, kb = 4, r_block = 4096, variant = 0;
    bool gfur = false;
    const void *rkey = nullptr, *skey = nullptr;
    int nrp = 0, nsp = 0;
    const void *rp[8]{}, *sp[8]{};
    int rw[8]{}, sw[8]{};
    uint64_t out_cap = 0;
    void *out_key = nullptr, *out_r[8]{}, *out_s[8]{};
    uint64_t *d_base = nullptr;      // groups + 1: first output row of each group
    uint64_t *d_total = nullptr;     // groups: output rows of each group
    uint32_t *d_units = nullptr;     // groups: work units of each group
    uint64_t *d_inst_off = nullptr;  // n + 1
    std::vector<Group> groups;
    // group-by batches (a Group's rows_r = rows, r0 = first row; S fields unused)
    const void *gkey = nullptr;
    const int32_t *gvals[8]{};
    int n_vals = 0, n_aggs = 0;
    gj_agg aggs[16]{};
    void *out_aggs[16]{};
    uint32_t *d_gstatus = nullptr;   // groups x 2: overflow flag, units
    uint32_t lds_bytes = 0;

    void *get(size_t bytes) {
        bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
        void *p = nullptr;
        if (has_alloc) p = alloc.alloc(bytes, alloc.ctx);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        if (!p) throw Error(GJ_ENOMEM, "plan: allocation of " + std::to_string(bytes) + " bytes failed");
        blocks.push_back(p);
        return p;
    }
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        for (void *p : blocks) {
            if (has_alloc) {
                if (alloc.free) alloc.free(p, alloc.ctx);
            } else {
                (void)hipFree(p);
            }
        }
        blocks.clear();
    }
};

namespace {

void enqueue_join(gj_plan *P, hipStream_t s) {
    VariantScope vs(P->variant);
    gj::fill_u64(s, P->d_base, 0ull, 1);
    for (size_t g = 0; g < P->groups.size(); ++g) {
        const Group &G = P->groups[g];
        const uint32_t ng = G.i1 - G.i0;
        P->arena.used = 0;  // groups run in stream order: each reuses the whole arena
        gj::Ctx ctx(&P->arena, s);
        gj::JoinSide side[2];
        for (int t = 0; t < 2; ++t) {
            const uint32_t rows = t ? G.rows_s : G.rows_r;
            const int64_t first = t ? G.s0 : G.r0;
            const int npay = t ? P->nsp : P->nrp;
            const int *w = t ? P->sw : P->rw;
            const void *const *pay = t ? P->sp : P->rp;
            const char *kin = static_cast<const char *>(t ? P->skey : P->rkey) + first * P->kb;
            gj::JoinSide &js = side[t];
            gj::PartCols pc;
            void *kout = ctx.scratch((size_t)rows * P->kb);
            js.key = kout;
            js.rows = rows;
            js.n_pay = npay;
            for (int i = 0; i < npay; ++i) js.width[i] = w[i];
            if (!P->gfur) {
                pc.n = npay;
                for (int i = 0; i < npay; ++i) {
                    pc.in[i] = static_cast<const char *>(pay[i]) + first * w[i];
                    pc.width[i] = w[i];
                    pc.out[i] = ctx.scratch((size_t)rows * w[i]);
                    js.pay[i] = pc.out[i];
                }
                js.rowid = nullptr;
            } else {
                pc.gen_rowid = true;
                pc.rowid_out = ctx.scratch((size_t)rows * 4);
                for (int i = 0; i < npay; ++i) js.pay[i] = static_cast<const char *>(pay[i]) + first * w[i];
                js.rowid = static_cast<const int32_t *>(pc.rowid_out);
            }
            uint32_t *poff = ctx.scratch_n<uint32_t>(((size_t)ng << 8) + 1);
            js.poff = poff;
            gj::partition_run_segments(ctx, P->kb, kin, kout, pc, rows, G.d_off[t], ng, G.d_bits, poff);
        }
        gj::JoinPlanned pl{};
        pl.cap_units = G.cap_units;
        pl.out_cap = P->out_cap;
        pl.out_base = P->d_base + g;
        pl.total = P->d_total + g;
        pl.next_base = P->d_base + g + 1;
        pl.out.key = P->out_key;
        for (int i = 0; i < P->nrp; ++i) pl.out.r[i] = P->out_r[i];
        for (int i = 0; i < P->nsp; ++i) pl.out.s[i] = P->out_s[i];
        pl.seg_bshift = G.d_bshift;
        pl.expect_rows = G.expect_rows;
        pl.units_out = P->d_units + g;
        gj::JoinOut jo{};
        gj::join_partitioned(ctx, P->kb, side[0], side[1], 0, P->r_block, P->gfur, &jo, G.d_bits, ng,
                             P->d_inst_off + G.i0, &pl);
    }
}

void enqueue_groupby(gj_plan *P, hipStream_t s) {
    VariantScope vs(P->variant);
    gj::fill_u64(s, P->d_base, 0ull, 1);
    for (size_t g = 0; g < P->groups.size(); ++g) {
        const Group &G = P->groups[g];
        P->arena.used = 0;
        gj::Ctx ctx(&P->arena, s);
        const char *k = static_cast<const char *>(P->gkey) + G.r0 * P->kb;
        const int32_t *v[8];
        for (int c = 0; c < P->n_vals; ++c) v[c] = P->gvals[c] + G.r0;
        gj::PgbPlanned pl{};
        pl.cap_units = G.cap_units;
        pl.out_base = P->d_base + g;
        pl.next_base = P->d_base + g + 1;
        pl.status = P->d_gstatus + 2 * g;
        pl.out_key = P->out_key;
        for (int j = 0; j < P->n_aggs; ++j) pl.out_aggs[j] = P->out_aggs[j];
        pl.out_cap = G.rows_r;
        pl.lds_bytes = P->lds_bytes;
        pl.inst_goff = P->d_inst_off + G.i0;
        gj::groupby_partition_segments(ctx, P->kb, k, v, P->n_vals, G.rows_r, P->aggs, P->n_aggs, P->gfur,
                                       G.d_off[0], G.i1 - G.i0, G.d_bits, pl);
    }
}

void enqueue(gj_plan *P, hipStream_t s) {
    if (P->kind == 0) enqueue_join(P, s);
    else enqueue_groupby(P, s);
}

void check_batch(const gj_rel_batch *R, const gj_rel_batch *S) {
    require(R && S, "null batch");
    const int32_t n = R->n_instances;
    require(n >= 1 && S->n_instances == n, "R and S need the same positive instance count");
    require(R->offsets && S->offsets, "null offsets");
    require(dtype_bytes(R->key.dtype) != 0 && R->key.dtype == S->key.dtype,
            "R.key and S.key need one dtype, GJ_I32 or GJ_I64");
    const gj_rel_batch *rel[2] = {R, S};
    for (int t = 0; t < 2; ++t) {
        const gj_rel_batch *X = rel[t];
        require(X->offsets[0] == 0, "offsets[0] must be 0");
        for (int i = 0; i < n; ++i) {
            require(X->offsets[i + 1] >= X->offsets[i], "offsets must not decrease");
            require(X->offsets[i + 1] - X->offsets[i] <= kMaxRows, "an instance has more than 2^31-1 rows",
                    GJ_EOVERFLOW);
        }
        require(X->n_payloads >= 0 && X->n_payloads <= 8, "0..8 payload columns");
        require(X->n_payloads == 0 || X->payloads, "null payload array");
        require(X->offsets[n] == 0 || X->key.data, "null key column");
        for (int i = 0; i < X->n_payloads; ++i) {
            require(dtype_bytes(X->payloads[i].dtype) != 0, "payload dtype must be GJ_I32 or GJ_I64");
            require(X->offsets[n] == 0 || X->payloads[i].data, "null payload column");
        }
    }
}

void check_tuning(const gj_join_tuning *t) {
    if (!t) return;
    for (int c = 0; c < GJ_TUNE_CLASSES; ++c) {
        require(t->part_log2[c] == 0 || (t->part_log2[c] >= 6 && t->part_log2[c] <= 12), "part_log2 must be 0 or 6..12");
        require(t->bucket_shift[c] == 0 || t->bucket_shift[c] == 1, "bucket_shift must be 0 or 1");
    }
    require(t->scatter_variant >= 0 && t->scatter_variant <= gj::kScatterVariants, "scatter_variant must be 0..14");
}

void build_join_plan(gj_plan *P, const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts,
                     const gj_join_tuning *tuning, int64_t out_capacity, hipStream_t st) {
    check_batch(R, S);
    check_tuning(tuning);
    gj_join_opts o{};
    if (opts) o = *opts;
    require(o.mat >= 0 && o.mat <= 2, "bad materialization");
    gj::check_join_lds_budget(o.lds_budget, dtype_bytes(R->key.dtype));
    require(o.flags == 0, "flags must be 0");
    require(o.algo == GJ_JOIN_AUTO || o.algo == GJ_JOIN_PHJ, "plans run the partitioned hash join only", GJ_EUNSUPPORTED);
    require(out_capacity >= 0, "negative output capacity");
    const int n = R->n_instances;
    P->n = n;
    P->kb = dtype_bytes(R->key.dtype);
    P->gfur = (o.mat == GJ_MAT_GFUR);
    P->r_block = o.lds_budget ? o.lds_budget : 4096;
    P->variant = tuning ? tuning->scatter_variant : 0;
    P->rkey = R->key.data;
    P->skey = S->key.data;
    P->nrp = R->n_payloads;
    P->nsp = S->n_payloads;
    for (int i = 0; i < P->nrp; ++i) {
        P->rp[i] = R->payloads[i].data;
        P->rw[i] = dtype_bytes(R->payloads[i].dtype);
    }
    for (int i = 0; i < P->nsp; ++i) {
        P->sp[i] = S->payloads[i].data;
        P->sw[i] = dtype_bytes(S->payloads[i].dtype);
    }
    uint64_t sum_s = (uint64_t)S->offsets[n];
    P->out_cap = out_capacity ? (uint64_t)out_capacity : sum_s;

    // per instance: partition bits and bucket shift from the size class
    std::vector<uint8_t> bits(n), bshift(n);
    for (int i = 0; i < n; ++i) {
        const uint64_t r = (uint64_t)(R->offsets[i + 1] - R->offsets[i]);
        const int c = r ? std::min(floor_log2(r), GJ_TUNE_CLASSES - 1) : 0;
        const int v = (tuning && tuning->part_log2[c]) ? tuning->part_log2[c] : kDefaultPartLog2;
        bits[i] = (uint8_t)std::max(0, std::min(8, ceil_log2(r) - v));
        bshift[i] = (uint8_t)(tuning ? tuning->bucket_shift[c] : 0);
    }
    // consecutive groups of at most kGroupRows rows per side (GJ_PLAN_GROUP_ROWS
    // lowers the limit, e.g. to exercise several groups on small batches)
    int64_t group_rows = kGroupRows;
    if (const char *e = getenv("GJ_PLAN_GROUP_ROWS")) {
        const long long v = atoll(e);
        if (v >= 1 && v < kGroupRows) group_rows = v;
    }
    P->groups.clear();
    for (int i = 0; i < n;) {
        Group G{};
        G.i0 = (uint32_t)i;
        G.r0 = R->offsets[i];
        G.s0 = S->offsets[i];
        uint64_t units = 0;
        int j = i;
        while (j < n) {
            const int64_t r = R->offsets[j + 1] - R->offsets[j], s = S->offsets[j + 1] - S->offsets[j];
            const int64_t nr = R->offsets[j + 1] - G.r0, ns = S->offsets[j + 1] - G.s0;
            if (j > i && (nr > group_rows || ns > group_rows)) break;
            if (r > 0 && s > 0) {
                const uint64_t a = std::min<uint64_t>(((uint64_t)r + P->r_block - 1) / P->r_block, kUnitFactor);
                const uint64_t piece = gj::join_s_piece(P->r_block);
                units += a * (((uint64_t)s + piece - 1) / piece + (1ull << bits[j]));
            }
            ++j;
        }
        G.i1 = (uint32_t)j;
        G.rows_r = (uint32_t)(R->offsets[j] - G.r0);
        G.rows_s = (uint32_t)(S->offsets[j] - G.s0);
        require(units < (1ull << 31), "too many work units in one group", GJ_EOVERFLOW);
        G.cap_units = (uint32_t)units;
        G.expect_rows = std::min<uint64_t>(G.rows_s, P->out_cap);
        P->cap_units_total += units;
        P->groups.push_back(G);
        i = j;
    }
    const int ng = (int)P->groups.size();

    // dry run: exact scratch size and launch count
    {
        gj::ProfPause pp;
        DryRun dr;
        P->arena = gj::Arena{};
        // placeholder addresses for the plan's own arrays (nothing is launched)
        char *ph = reinterpret_cast<char *>(uintptr_t(1) << 45);
        P->d_base = P->d_total = reinterpret_cast<uint64_t *>(ph);
        P->d_inst_off = reinterpret_cast<uint64_t *>(ph);
        P->d_units = reinterpret_cast<uint32_t *>(ph);
        P->out_key = ph;
        for (int i = 0; i < 8; ++i) P->out_r[i] = P->out_s[i] = ph;
        for (Group &G : P->groups) {
            G.d_bits = G.d_bshift = reinterpret_cast<uint8_t *>(ph);
            G.d_off[0] = G.d_off[1] = reinterpret_cast<uint32_t *>(ph);
        }
        enqueue_join(P, st);
        P->launches = gj::g_dry_launches;
    }
    const size_t scratch = P->arena.peak;

    // device memory: parameters, status words, outputs, scratch
    std::vector<size_t> poff_of(ng);
    size_t param_bytes = 0;
    for (int g = 0; g < ng; ++g) {
        const Group &G = P->groups[g];
        const size_t m = G.i1 - G.i0;
        poff_of[g] = param_bytes;
        param_bytes += ((2 * m + 3) & ~size_t(3)) + 8 * (m + 1);
    }
    param_bytes = (param_bytes + 7) & ~size_t(7);
    const size_t status_bytes = 8 * (size_t)(ng + 1) + 8 * (size_t)ng + 4 * (size_t)ng + 4 + 8 * (size_t)(n + 1);
    char *pb = static_cast<char *>(P->get(param_bytes + status_bytes));
    std::vector<char> host(param_bytes, 0);
    for (int g = 0; g < ng; ++g) {
        Group &G = P->groups[g];
        const size_t m = G.i1 - G.i0;
        char *h = host.data() + poff_of[g];
        char *d = pb + poff_of[g];
        memcpy(h, bits.data() + G.i0, m);
        memcpy(h + m, bshift.data() + G.i0, m);
        G.d_bits = reinterpret_cast<uint8_t *>(d);
        G.d_bshift = reinterpret_cast<uint8_t *>(d + m);
        const size_t o = (2 * m + 3) & ~size_t(3);
        uint32_t *ho[2] = {reinterpret_cast<uint32_t *>(h + o), reinterpret_cast<uint32_t *>(h + o + 4 * (m + 1))};
        for (size_t k = 0; k <= m; ++k) {
            ho[0][k] = (uint32_t)(R->offsets[G.i0 + k] - G.r0);
            ho[1][k] = (uint32_t)(S->offsets[G.i0 + k] - G.s0);
        }
        G.d_off[0] = reinterpret_cast<uint32_t *>(d + o);
        G.d_off[1] = reinterpret_cast<uint32_t *>(d + o + 4 * (m + 1));
    }
    char *sp = pb + param_bytes;
    P->d_base = reinterpret_cast<uint64_t *>(sp);
    P->d_total = P->d_base + (ng + 1);
    P->d_inst_off = P->d_total + ng;
    P->d_units = reinterpret_cast<uint32_t *>(P->d_inst_off + (n + 1));
    const uint64_t cap_rows = std::max<uint64_t>(P->out_cap, 1);
    P->out_key = P->get(cap_rows * P->kb);
    P->output_bytes = (int64_t)(cap_rows * P->kb);
    for (int i = 0; i < P->nrp; ++i) {
        P->out_r[i] = P->get(cap_rows * P->rw[i]);
        P->output_bytes += (int64_t)(cap_rows * P->rw[i]);
    }
    for (int i = 0; i < P->nsp; ++i) {
        P->out_s[i] = P->get(cap_rows * P->sw[i]);
        P->output_bytes += (int64_t)(cap_rows * P->sw[i]);
    }
    P->arena = gj::Arena{};
    P->arena.base = static_cast<char *>(P->get(scratch));
    P->arena.size = std::max<size_t>(scratch, 256);
    if (param_bytes) GJ_HIP(hipMemcpyAsync(pb, host.data(), param_bytes, hipMemcpyHostToDevice, st));
    GJ_HIP(hipMemsetAsync(sp, 0, status_bytes, st));  // a result read before any run sees zeros
    GJ_HIP(hipStreamSynchronize(st));
}

void build_groupby_plan(gj_plan *P, const gj_gb_batch *B, const gj_agg *aggs, int32_t n_aggs,
                        const gj_groupby_opts *opts, hipStream_t st) {
    require(B != nullptr, "null batch");
    const int32_t n = B->n_instances;
    require(n >= 1, "need at least one instance");
    require(B->offsets && B->offsets[0] == 0, "offsets[0] must be 0");
    for (int i = 0; i < n; ++i) {
        require(B->offsets[i + 1] >= B->offsets[i], "offsets must not decrease");
        require(B->offsets[i + 1] - B->offsets[i] <= kMaxRows, "an instance has more than 2^31-1 rows", GJ_EOVERFLOW);
    }
    const int64_t total = B->offsets[n];
    P->kb = dtype_bytes(B->key.dtype);
    require(P->kb != 0, "key dtype must be GJ_I32 or GJ_I64");
    require(total == 0 || B->key.data, "null key column");
    require(B->n_vals >= 0 && B->n_vals <= 8, "0..8 value columns");
    require(B->n_vals == 0 || B->vals, "null value array");
    for (int c = 0; c < B->n_vals; ++c) {
        require(B->vals[c].dtype == GJ_I32, "value columns must be GJ_I32");
        require(total == 0 || B->vals[c].data, "null value column");
        P->gvals[c] = static_cast<const int32_t *>(B->vals[c].data);
    }
    require(n_aggs >= 1 && n_aggs <= 16 && aggs, "1..16 aggregates");
    for (int j = 0; j < n_aggs; ++j) {
        require(aggs[j].op >= GJ_SUM && aggs[j].op <= GJ_MAX, "bad aggregate op");
        require(aggs[j].op == GJ_COUNT || (aggs[j].col >= 0 && aggs[j].col < B->n_vals), "aggregate column out of range");
        P->aggs[j] = aggs[j];
    }
    gj_groupby_opts o{};
    if (opts) o = *opts;
    require(o.algo == GJ_GB_AUTO || o.algo == GJ_GB_PARTITION, "group-by plans use the partition algorithm");
    require(o.mat >= 0 && o.mat <= 2, "bad materialization");
    require(o.radix_bits >= 0 && o.radix_bits <= 8, "radix_bits must be 0..8 for batches");
    P->kind = 1;
    P->n = n;
    P->gfur = (o.mat == GJ_MAT_GFUR);
    P->gkey = B->key.data;
    P->n_vals = B->n_vals;
    P->n_aggs = n_aggs;
    P->lds_bytes = gj::pgb_plan_lds_bytes(P->kb);
    std::vector<uint8_t> bits(n);
    for (int i = 0; i < n; ++i) {
        const uint64_t r = (uint64_t)(B->offsets[i + 1] - B->offsets[i]);
        bits[i] = (uint8_t)(o.radix_bits ? o.radix_bits : std::max(0, std::min(8, ceil_log2(r) - 10)));
    }
    int64_t group_rows = kGroupRows;
    if (const char *e = getenv("GJ_PLAN_GROUP_ROWS")) {
        const long long v = atoll(e);
        if (v >= 1 && v < kGroupRows) group_rows = v;
    }
    P->groups.clear();
    for (int i = 0; i < n;) {
        Group G{};
        G.i0 = (uint32_t)i;
        G.r0 = B->offsets[i];
        uint64_t units = 0;
        int j = i;
        while (j < n) {
            const int64_t r = B->offsets[j + 1] - B->offsets[j];
            if (j > i && B->offsets[j + 1] - G.r0 > group_rows) break;
            // aggregation units: sum over partitions of ceil(rows / 8192) <= rows / 8192 + partitions
            units += ((uint64_t)r + 8191) / 8192 + (r > 0 ? (1ull << bits[j]) : 0);
            ++j;
        }
        G.i1 = (uint32_t)j;
        G.rows_r = (uint32_t)(B->offsets[j] - G.r0);
        require(units < (1ull << 31), "too many work units in one group", GJ_EOVERFLOW);
        G.cap_units = (uint32_t)units;
        P->cap_units_total += units;
        P->groups.push_back(G);
        i = j;
    }
    const int ng = (int)P->groups.size();
    P->out_cap = (uint64_t)total;
    {
        gj::ProfPause pp;
        DryRun dr;
        P->arena = gj::Arena{};
        char *ph = reinterpret_cast<char *>(uintptr_t(1) << 45);
        P->d_base = reinterpret_cast<uint64_t *>(ph);
        P->d_inst_off = reinterpret_cast<uint64_t *>(ph);
        P->d_gstatus = reinterpret_cast<uint32_t *>(ph);
        P->out_key = ph;
        for (int j = 0; j < 16; ++j) P->out_aggs[j] = ph;
        for (Group &G : P->groups) {
            G.d_bits = reinterpret_cast<uint8_t *>(ph);
            G.d_off[0] = reinterpret_cast<uint32_t *>(ph);
        }
        enqueue_groupby(P, st);
        P->launches = gj::g_dry_launches;
    }
    const size_t scratch = P->arena.peak;
    std::vector<size_t> poff_of(ng);
    size_t param_bytes = 0;
    for (int g = 0; g < ng; ++g) {
        const size_t m = P->groups[g].i1 - P->groups[g].i0;
        poff_of[g] = param_bytes;
        param_bytes += ((m + 3) & ~size_t(3)) + 4 * (m + 1);
    }
    param_bytes = (param_bytes + 7) & ~size_t(7);
    const size_t status_bytes = 8 * (size_t)(ng + 1) + 8 * (size_t)(n + 1) + 8 * (size_t)ng;
    char *pb = static_cast<char *>(P->get(param_bytes + status_bytes));
    std::vector<char> host(param_bytes, 0);
    for (int g = 0; g < ng; ++g) {
        Group &G = P->groups[g];
        const size_t m = G.i1 - G.i0;
        char *h = host.data() + poff_of[g];
        char *d = pb + poff_of[g];
        memcpy(h, bits.data() + G.i0, m);
        G.d_bits = reinterpret_cast<uint8_t *>(d);
        const size_t o = (m + 3) & ~size_t(3);
        uint32_t *ho = reinterpret_cast<uint32_t *>(h + o);
        for (size_t k = 0; k <= m; ++k) ho[k] = (uint32_t)(B->offsets[G.i0 + k] - G.r0);
        G.d_off[0] = reinterpret_cast<uint32_t *>(d + o);
    }
    char *sp = pb + param_bytes;
    P->d_base = reinterpret_cast<uint64_t *>(sp);
    P->d_inst_off = P->d_base + (ng + 1);
    P->d_gstatus = reinterpret_cast<uint32_t *>(P->d_inst_off + (n + 1));
    const uint64_t cap_rows = std::max<uint64_t>(P->out_cap, 1);
    P->out_key = P->get(cap_rows * P->kb);
    P->output_bytes = (int64_t)(cap_rows * P->kb);
    for (int j = 0; j < n_aggs; ++j) {
        const int w = (aggs[j].op == GJ_SUM || aggs[j].op == GJ_COUNT) ? 8 : 4;
        P->out_aggs[j] = P->get(cap_rows * w);
        P->output_bytes += (int64_t)(cap_rows * w);
    }
    P->arena = gj::Arena{};
    P->arena.base = static_cast<char *>(P->get(scratch));
    P->arena.size = std::max<size_t>(scratch, 256);
    if (param_bytes) GJ_HIP(hipMemcpyAsync(pb, host.data(), param_bytes, hipMemcpyHostToDevice, st));
    GJ_HIP(hipMemsetAsync(sp, 0, status_bytes, st));
    GJ_HIP(hipStreamSynchronize(st));
}

int plan_error(int code, const std::string &msg) { return gj::fail(code, msg); }

float median(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.f : v[v.size() / 2];
}

}  // namespace

extern "C" {

int gj_join_plan_create(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts,
                        const gj_join_tuning *tuning, int64_t out_capacity, const gj_allocator *alloc,
                        void *stream, gj_plan **plan) {
    gj::clear_error();
    if (!plan) return plan_error(GJ_EINVAL, "null plan pointer");
    *plan = nullptr;
    gj_plan *P = new gj_plan();
    if (alloc && alloc->alloc) {
        P->alloc = *alloc;
        P->has_alloc = true;
    }
    try {
        build_join_plan(P, R, S, opts, tuning, out_capacity, (hipStream_t)stream);
        *plan = P;
        return GJ_OK;
    } catch (const Error &e) {
        P->release();
        delete P;
        return plan_error(e.code, e.what());
    } catch (const std::exception &e) {
        P->release();
        delete P;
        return plan_error(GJ_EHIP, e.what());
    }
}

int gj_groupby_plan_create(const gj_gb_batch *B, const gj_agg *aggs, int32_t n_aggs, const gj_groupby_opts *opts,
                           const gj_allocator *alloc, void *stream, gj_plan **plan) {
    gj::clear_error();
    if (!plan) return plan_error(GJ_EINVAL, "null plan pointer");
    *plan = nullptr;
    gj_plan *P = new gj_plan();
    if (alloc && alloc->alloc) {
        P->alloc = *alloc;
        P->has_alloc = true;
    }
    try {
        build_groupby_plan(P, B, aggs, n_aggs, opts, (hipStream_t)stream);
        *plan = P;
        return GJ_OK;
    } catch (const Error &e) {
        P->release();
        delete P;
        return plan_error(e.code, e.what());
    } catch (const std::exception &e) {
        P->release();
        delete P;
        return plan_error(GJ_EHIP, e.what());
    }
}

int gj_groupby_plan_result(gj_plan *P, void *stream, gj_groupby_out *out, int64_t *group_offsets) {
    gj::clear_error();
    if (!P || !out) return plan_error(GJ_EINVAL, "null argument");
    if (P->kind != 1) return plan_error(GJ_EINVAL, "not a group-by plan");
    try {
        GJ_HIP(hipStreamSynchronize((hipStream_t)stream));
        const int ng = (int)P->groups.size();
        std::vector<uint64_t> base(ng + 1);
        std::vector<uint32_t> status(2 * ng);
        GJ_HIP(hipMemcpy(base.data(), P->d_base, 8 * (ng + 1), hipMemcpyDeviceToHost));
        GJ_HIP(hipMemcpy(status.data(), P->d_gstatus, 8 * ng, hipMemcpyDeviceToHost));
        if (group_offsets) {
            std::vector<uint64_t> off(P->n + 1);
            GJ_HIP(hipMemcpy(off.data(), P->d_inst_off, 8 * (P->n + 1), hipMemcpyDeviceToHost));
            for (int i = 0; i <= P->n; ++i) group_offsets[i] = (int64_t)off[i];
        }
        out->n_groups = (int64_t)base[ng];
        out->key = P->out_key;
        if (out->aggs)
            for (int j = 0; j < P->n_aggs; ++j) out->aggs[j] = P->out_aggs[j];
        for (int g = 0; g < ng; ++g) {
            if (status[2 * g])
                return plan_error(GJ_ECAPACITY, "plan: a partition of group " + std::to_string(g) +
                                                    " holds more distinct keys than its LDS table");
            if (status[2 * g + 1] > P->groups[g].cap_units)
                return plan_error(GJ_ECAPACITY, "plan: aggregation units exceed the plan's room");
        }
        return GJ_OK;
    } catch (const Error &e) {
        return plan_error(e.code, e.what());
    }
}

int gj_plan_run(gj_plan *P, void *stream) {
    gj::clear_error();
    if (!P) return plan_error(GJ_EINVAL, "null plan");
    try {
        enqueue(P, (hipStream_t)stream);
        return GJ_OK;
    } catch (const Error &e) {
        return plan_error(e.code, e.what());
    }
}

int gj_plan_capture(gj_plan *P) {
    gj::clear_error();
    if (!P) return plan_error(GJ_EINVAL, "null plan");
    if (P->exec) return GJ_OK;
    hipStream_t cs = nullptr;
    try {
        gj::ProfPause pp;
        GJ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        GJ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue(P, cs);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        GJ_HIP(hipStreamEndCapture(cs, &P->graph));
        GJ_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        GJ_HIP(hipStreamDestroy(cs));
        return GJ_OK;
    } catch (const Error &e) {
        if (cs) (void)hipStreamDestroy(cs);
        return plan_error(e.code, e.what());
    }
}

int gj_plan_launch(gj_plan *P, void *stream) {
    gj::clear_error();
    if (!P) return plan_error(GJ_EINVAL, "null plan");
    if (!P->exec) return plan_error(GJ_EINVAL, "plan not captured");
    const hipError_t e = hipGraphLaunch(P->exec, (hipStream_t)stream);
    if (e != hipSuccess) return plan_error(GJ_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return GJ_OK;
}

int gj_join_plan_result(gj_plan *P, void *stream, gj_join_out *out, int64_t *out_offsets) {
    gj::clear_error();
    if (!P || !out) return plan_error(GJ_EINVAL, "null argument");
    if (P->kind != 0) return plan_error(GJ_EINVAL, "not a join plan");
    try {
        hipStream_t st = (hipStream_t)stream;
        GJ_HIP(hipStreamSynchronize(st));
        const int ng = (int)P->groups.size();
        std::vector<uint64_t> base(ng + 1);
        std::vector<uint32_t> units(ng);
        GJ_HIP(hipMemcpy(base.data(), P->d_base, 8 * (ng + 1), hipMemcpyDeviceToHost));
        GJ_HIP(hipMemcpy(units.data(), P->d_units, 4 * ng, hipMemcpyDeviceToHost));
        if (out_offsets) {
            std::vector<uint64_t> off(P->n + 1);
            GJ_HIP(hipMemcpy(off.data(), P->d_inst_off, 8 * (P->n + 1), hipMemcpyDeviceToHost));
            for (int i = 0; i <= P->n; ++i) out_offsets[i] = (int64_t)off[i];
        }
        const uint64_t T = base[ng];
        out->n_rows = (int64_t)T;
        out->key = P->out_key;
        for (int i = 0; i < P->nrp; ++i)
            if (out->r_payloads) out->r_payloads[i] = P->out_r[i];
        for (int i = 0; i < P->nsp; ++i)
            if (out->s_payloads) out->s_payloads[i] = P->out_s[i];
        for (int g = 0; g < ng; ++g)
            if (units[g] > P->groups[g].cap_units)
                return plan_error(GJ_ECAPACITY, "plan: group " + std::to_string(g) + " needed " +
                                                    std::to_string(units[g]) + " work units, room for " +
                                                    std::to_string(P->groups[g].cap_units));
        if (T > P->out_cap)
            return plan_error(GJ_ECAPACITY, "plan: " + std::to_string(T) + " output rows, capacity " +
                                                std::to_string(P->out_cap));
        return GJ_OK;
    } catch (const Error &e) {
        return plan_error(e.code, e.what());
    }
}

int gj_plan_get_info(const gj_plan *P, gj_plan_info *info) {
    if (!P || !info) return plan_error(GJ_EINVAL, "null argument");
    info->launches_per_run = P->launches;
    info->groups = (int64_t)P->groups.size();
    info->scratch_bytes = (int64_t)P->arena.size;
    info->output_bytes = P->output_bytes;
    info->unit_capacity = P->cap_units_total;
    return GJ_OK;
}

int gj_groupby_batch(const gj_gb_batch *B, const gj_agg *aggs, int32_t n_aggs, const gj_groupby_opts *opts,
                     const gj_allocator *alloc, void *stream, gj_groupby_out *out, int64_t *group_offsets) {
    gj::clear_error();
    if (!out) return plan_error(GJ_EINVAL, "null output");
    if (n_aggs > 0 && !out->aggs) return plan_error(GJ_EINVAL, "null aggs array");
    out->n_groups = 0;
    out->key = nullptr;
    gj_plan *P = nullptr;
    int rc = gj_groupby_plan_create(B, aggs, n_aggs, opts, alloc, stream, &P);
    if (rc != GJ_OK) return rc;
    try {
        rc = gj_plan_run(P, stream);
        void *pa[16] = {nullptr};
        gj_groupby_out po{};
        po.aggs = pa;
        if (rc == GJ_OK) rc = gj_groupby_plan_result(P, stream, &po, group_offsets);
        if (rc != GJ_OK) {
            const std::string msg = gj_last_error();
            gj_plan_destroy(P);
            return plan_error(rc, msg);
        }
        // the plan's columns hold sum(N_i) rows, the first n_groups of them used:
        // copy those into columns of the caller's allocator
        hipStream_t st = (hipStream_t)stream;
        gj::Ctx ctx(alloc, st);
        const uint64_t g = (uint64_t)po.n_groups;
        const size_t kbytes = (size_t)P->kb;
        void *okey = ctx.output(g * kbytes);
        if (g) GJ_HIP(hipMemcpyAsync(okey, po.key, g * kbytes, hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < n_aggs; ++j) {
            const size_t w = (aggs[j].op == GJ_SUM || aggs[j].op == GJ_COUNT) ? 8 : 4;
            void *o = ctx.output(g * w);
            if (g) GJ_HIP(hipMemcpyAsync(o, po.aggs[j], g * w, hipMemcpyDeviceToDevice, st));
            out->aggs[j] = o;
        }
        GJ_HIP(hipStreamSynchronize(st));  // the plan's columns are released next
        ctx.commit();
        out->key = okey;
        out->n_groups = (int64_t)g;
        gj_plan_destroy(P);
        return GJ_OK;
    } catch (const Error &e) {
        gj_plan_destroy(P);
        out->n_groups = 0;
        out->key = nullptr;
        return plan_error(e.code, e.what());
    }
}

int gj_plan_destroy(gj_plan *P) {
    if (!P) return GJ_OK;
    P->release();
    delete P;
    return GJ_OK;
}

int gj_join_autotune(const gj_rel_batch *R, const gj_rel_batch *S, const gj_join_opts *opts, int32_t reps,
                     const gj_allocator *alloc, void *stream, gj_join_tuning *out) {
    gj::clear_error();
    if (!out) return plan_error(GJ_EINVAL, "null output table");
    hipStream_t st = (hipStream_t)stream;
    std::vector<void *> staged;  // staging columns (released at the end)
    auto get = [&](size_t bytes) -> void * {
        bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
        void *p = nullptr;
        if (alloc && alloc->alloc) p = alloc->alloc(bytes, alloc->ctx);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        if (!p) throw Error(GJ_ENOMEM, "autotune: allocation failed");
        staged.push_back(p);
        return p;
    };
    auto put_all = [&]() {
        for (void *p : staged) {
            if (alloc && alloc->alloc) {
                if (alloc->free) alloc->free(p, alloc->ctx);
            } else {
                (void)hipFree(p);
            }
        }
        staged.clear();
    };
    hipEvent_t ea = nullptr, eb = nullptr;
    try {
        check_batch(R, S);
        require(reps >= 1 && reps <= 100, "reps must be 1..100");
        GJ_HIP(hipEventCreate(&ea));
        GJ_HIP(hipEventCreate(&eb));
        const int n = R->n_instances;
        gj_join_tuning best{};
        std::vector<std::vector<int>> members(GJ_TUNE_CLASSES);
        for (int i = 0; i < n; ++i) {
            const int64_t r = R->offsets[i + 1] - R->offsets[i], s = S->offsets[i + 1] - S->offsets[i];
            if (r > 0 && s > 0) members[std::min(floor_log2((uint64_t)r), GJ_TUNE_CLASSES - 1)].push_back(i);
        }
        // staging batch of up to 64 instances of one class (at most ~2^27 S rows)
        struct Staging {
            gj_col rk, sk;
            gj_col rp[8], sp[8];
            std::vector<int64_t> ro, so;
            gj_rel_batch Rb, Sb;
            int64_t rows = 0;
        };
        auto stage = [&](const std::vector<int> &idx, Staging &X) {
            std::vector<int> pick;
            const size_t want = std::min<size_t>(64, idx.size());
            int64_t srows = 0;
            for (size_t k = 0; k < want; ++k) {
                const int i = idx[k * idx.size() / want];
                const int64_t s = S->offsets[i + 1] - S->offsets[i];
                if (!pick.empty() && srows + s > (1LL << 27)) break;
                pick.push_back(i);
                srows += s;
            }
            X.ro.assign(1, 0);
            X.so.assign(1, 0);
            for (int i : pick) {
                X.ro.push_back(X.ro.back() + R->offsets[i + 1] - R->offsets[i]);
                X.so.push_back(X.so.back() + S->offsets[i + 1] - S->offsets[i]);
            }
            const gj_rel_batch *src[2] = {R, S};
            for (int t = 0; t < 2; ++t) {
                const gj_rel_batch *B = src[t];
                const std::vector<int64_t> &off = t ? X.so : X.ro;
                const int64_t rows = off.back();
                const int ncol = 1 + B->n_payloads;
                for (int c = 0; c < ncol; ++c) {
                    const gj_col &col = c == 0 ? B->key : B->payloads[c - 1];
                    const int w = dtype_bytes(col.dtype);
                    char *dst = static_cast<char *>(get((size_t)rows * w));
                    for (size_t k = 0; k < pick.size(); ++k) {
                        const int i = pick[k];
                        const int64_t len = B->offsets[i + 1] - B->offsets[i];
                        GJ_HIP(hipMemcpyAsync(dst + off[k] * w, static_cast<const char *>(col.data) + B->offsets[i] * w,
                                              (size_t)len * w, hipMemcpyDeviceToDevice, st));
                    }
                    gj_col nc{dst, col.dtype};
                    if (c == 0) (t ? X.sk : X.rk) = nc;
                    else (t ? X.sp : X.rp)[c - 1] = nc;
                }
            }
            X.Rb = gj_rel_batch{X.rk, X.rp, R->n_payloads, X.ro.data(), (int32_t)pick.size()};
            X.Sb = gj_rel_batch{X.sk, X.sp, S->n_payloads, X.so.data(), (int32_t)pick.size()};
            X.rows = X.ro.back() + X.so.back();
        };
        auto time_table = [&](const Staging &X, const gj_join_tuning &t) -> float {
            gj_plan *p = nullptr;
            int rc = gj_join_plan_create(&X.Rb, &X.Sb, opts, &t, 0, alloc, stream, &p);
            if (rc != GJ_OK) throw Error(rc, std::string("autotune: ") + gj_last_error());
            std::vector<float> ms;
            try {
                rc = gj_plan_capture(p);
                if (rc != GJ_OK) throw Error(rc, std::string("autotune: ") + gj_last_error());
                for (int k = 0; k <= reps; ++k) {
                    GJ_HIP(hipEventRecord(ea, st));
                    GJ_HIP(hipGraphLaunch(p->exec, st));
                    GJ_HIP(hipEventRecord(eb, st));
                    GJ_HIP(hipEventSynchronize(eb));
                    float x = 0.f;
                    GJ_HIP(hipEventElapsedTime(&x, ea, eb));
                    if (k > 0) ms.push_back(x);  // the first launch warms up
                }
                gj_join_out o{};
                void *rr[8], *ss[8];
                o.r_payloads = rr;
                o.s_payloads = ss;
                rc = gj_join_plan_result(p, stream, &o, nullptr);
                if (rc != GJ_OK) throw Error(rc, std::string("autotune: ") + gj_last_error());
            } catch (...) {
                gj_plan_destroy(p);
                throw;
            }
            gj_plan_destroy(p);
            return median(ms);
        };
        int big_class = -1;
        int64_t big_rows = -1;
        for (int c = 0; c < GJ_TUNE_CLASSES; ++c) {
            if (members[c].empty()) continue;
            Staging X;
            stage(members[c], X);
            float tbest = INFINITY;
            int8_t bv = 0, bs = 0;
            for (int v = 9; v <= 12; ++v) {
                for (int sh = 0; sh <= 1; ++sh) {
                    gj_join_tuning t = best;
                    t.part_log2[c] = (int8_t)v;
                    t.bucket_shift[c] = (int8_t)sh;
                    const float x = time_table(X, t);
                    if (x < tbest) {
                        tbest = x;
                        bv = (int8_t)v;
                        bs = (int8_t)sh;
                    }
                }
            }
            best.part_log2[c] = bv;
            best.bucket_shift[c] = bs;
            if (X.rows > big_rows) {
                big_rows = X.rows;
                big_class = c;
            }
            put_all();
        }
        if (big_class >= 0) {
            Staging X;
            stage(members[big_class], X);
            float tbest = INFINITY;
            int bvar = 0;
            for (int v = 0; v <= gj::kScatterVariants; ++v) {
                gj_join_tuning t = best;
                t.scatter_variant = v;
                const float x = time_table(X, t);
                if (x < tbest) {
                    tbest = x;
                    bvar = v;
                }
            }
            best.scatter_variant = bvar;
            put_all();
        }
        *out = best;
        (void)hipEventDestroy(ea);
        (void)hipEventDestroy(eb);
        return GJ_OK;
    } catch (const Error &e) {
        (void)hipStreamSynchronize(st);
        put_all();
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        return plan_error(e.code, e.what());
    }
}

}  // extern "C"
