// Algorithm selection: an analytical bandwidth cost model (the paper's models of
// Sections 4.1.3, 4.1.4 and 4.4 applied to this implementation's passes, with
// constants measured on MI355X) and a small learned network over the same
// workload features. The network decides when trained weights are loaded and
// finite; the cost model decides otherwise. Either way only speed changes:
// every algorithm computes the same result.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace gj {
namespace {

// MI355X constants, measured with the library's own kernels (the clustered and
// unclustered gathers of Section 4.1.1, 2^27 4-byte values): B_G is the stream
// copy's read + write rate, 5.16 TB/s; the unclustered gather took 5.86 times
// as long as the clustered one, so B_G / B_R = (12 * 5.86 - 8) / 4 = 15.6 (the
// paper's A100 figure is 24). Global atomics: scattered 64-bit updates per
// second.
struct Consts {
    double seq = 5.16e12;
    double rand_ratio = 15.6;
    double atomic_rate = 2.5e10;
};
Consts g_c;

constexpr double kLdsBytes = 160.0 * 1024.0;  // per compute unit (and per workgroup)

struct Workload {
    bool join;
    double nr, ns, g, w, cr, cs, alpha, mr, key_bytes_varying;
};

Workload decode(const float *f) {
    Workload x{};
    x.join = f[0] > 0.5f;
    x.nr = exp2(32.0 * f[1]);
    x.ns = exp2(32.0 * f[2]);
    x.g = exp2(32.0 * f[3]);
    x.w = 8.0 * f[4];
    x.cr = std::max(0.0, std::round(8.0 * f[5]));
    x.cs = x.join ? std::max(0.0, std::round(8.0 * f[6])) : 0.0;
    x.key_bytes_varying = x.join ? x.w : std::max(1.0, std::round(8.0 * f[6]));
    x.alpha = 1.2 * f[7];
    x.mr = f[8];
    return x;
}

int passes_for(double rows) {
    const int bits = std::max(1, (int)std::ceil(std::log2(std::max(1.0, rows / 2048.0))));
    return std::min(bits, 16) > 8 ? 2 : 1;
}

// Partition passes of a join over R rows with the default build block.
int join_passes_for(double rows, int key_bytes, int r_pay_bytes) {
    const uint64_t n = (uint64_t)std::max(1.0, rows);
    return join_default_bits(n, join_default_r_block(n, key_bytes, false, r_pay_bytes)) > 8 ? 2 : 1;
}

// Classes: 0 partitioned GFTR, 1 partitioned GFUR, 6 sort-merge GFTR (the paper's
// models of Section 4.1.4 over this implementation's passes).
void cost_join(const Workload &x, double *t) {
    const double R = x.nr, S = x.ns, w = x.w;
    const double T = x.mr * S;  // PK-FK
    const double P = join_passes_for(R, w > 4.0 ? 8 : 4, (int)(4.0 * x.cr));
    const double r = 4.0 * x.cr, s = 4.0 * x.cs;
    const double hist = P * w * (R + S), count = w * (R + S);
    const double gftr = hist + 2 * P * ((w + r) * R + (w + s) * S) + count + w * (R + S) + r * R + s * S +
                        T * (w + r + s);
    const double gfur_seq = hist + 2 * P * (w + 4) * (R + S) + count + w * (R + S) + 4 * (R + S) + T * (w + r + s);
    const double gfur_rand = T * (r + s) * g_c.rand_ratio;  // each gathered byte at B_G / ratio
    // sort-merge: LSD passes over the key bytes that vary (dense keys below 2^24
    // leave the top byte constant), the Merge Path read of both key columns,
    // bounds, counts and offsets per S row, then a write pass whose R reads only
    // move forward (clustered)
    const double ps = w > 4.0 ? 8.0 : (std::max(R, S) < 16777216.0 ? 3.0 : 4.0);
    const double smj = ps * (w * (R + S) + 2 * ((w + r) * R + (w + s) * S)) + w * (R + S) + 24 * S + r * R + s * S +
                       T * (w + r + s);
    for (int c = 0; c < 7; ++c) t[c] = INFINITY;
    t[0] = gftr / g_c.seq;
    t[1] = (gfur_seq + gfur_rand) / g_c.seq;
    t[6] = smj / g_c.seq;
}

// Classes: 2 hash, 3 sort, 4 partition, 5 sort on dictionary-encoded keys.
void cost_groupby(const Workload &x, double *t) {
    const double N = x.nr, g = std::min(x.g, x.nr), w = x.w, v = x.cr;
    const double rec = 8 + 16 * v;  // count + (sum, min, max) per value column
    const double out = g * (w + rec);
    // hash: table fill and insert stream; aggregation in LDS when the ids, cut
    // into at most 64 ranges, fit a workgroup's LDS per range (several ranges
    // resolve every row's id once and re-read it, mostly from L2), else global
    // atomics for the rows of groups beyond 64 KB of records
    const double table = 1.5 * N * (w == 4 ? 8 : 4);
    const double ins = table + N * (w + 8);
    const double slices = std::ceil(g * (rec + 4) / kLdsBytes);
    double th = (ins + N * (4 + 4 * v) + out) / g_c.seq;
    if (slices <= 64) th += (slices > 1 ? 12 * N : 0.0) / g_c.seq + (slices - 1) * N * 4 / (4 * g_c.seq);
    else th += N * (1 + 3 * v) * (1.0 - std::min(1.0, 65536.0 / (g * (rec + 4)))) / g_c.atomic_rate;
    if (g * 16 > 32e6) th += N * 64 * 2 / g_c.seq;  // table probes miss the caches
    // sort: LSD passes over the key bytes that vary, then the segmented reduction
    const double sp = std::max(1.0, x.key_bytes_varying);
    const double ts = (w * N + sp * (w * N + 2 * (w + 4 * v) * N) + (w + 4 * v) * N + out) / g_c.seq;
    // sort on codes (Section 4.4): the encoding is the hash table's insert, the
    // code write and the rank lookup; then ceil(log2 g / 8) passes over 4-byte codes
    const double cp = std::max(1.0, std::ceil(std::log2(std::max(2.0, g)) / 8.0));
    const double tde = (ins + 8 * N + 4 * N + cp * (4 * N + 2 * (4 + 4 * v) * N) + (4 + 4 * v) * N + out) / g_c.seq;
    // partition: hashed partitioning, discovery (two key reads), aggregation
    const double P = passes_for(N);
    double tp = (P * w * N + 2 * P * (w + 4 * v) * N + 2 * w * N + (w + 4 * v) * N + out) / g_c.seq;
    if (g < 256) tp *= 1.0 + 256.0 / std::max(1.0, g) * 0.05;  // few busy partitions
    for (int c = 0; c < 7; ++c) t[c] = INFINITY;
    t[2] = th;
    t[3] = ts;
    t[4] = tp;
    t[5] = tde;
}

// ---- the learned network, evaluated on the host for one sample ----
constexpr int F = 12, H = 64, C = 7;
std::mutex g_mu;
std::vector<float> g_w;  // empty = no trained weights

void mlp_probs(const float *theta, const float *x, const float *mask, float *p) {
    const float *W1 = theta, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + C * H;
    float h1[H], h2[H], z[C];
    for (int i = 0; i < H; ++i) {
        float a = 0.f;
        for (int k = 0; k < F; ++k) a = fmaf(x[k], W1[i * F + k], a);
        h1[i] = std::max(a + b1[i], 0.f);
    }
    for (int i = 0; i < H; ++i) {
        float a = 0.f;
        for (int k = 0; k < H; ++k) a = fmaf(h1[k], W2[i * H + k], a);
        h2[i] = std::max(a + b2[i], 0.f);
    }
    float mx = -INFINITY;
    for (int c = 0; c < C; ++c) {
        float a = 0.f;
        for (int k = 0; k < H; ++k) a = fmaf(h2[k], W3[c * H + k], a);
        z[c] = a + b3[c];
        if (mask[c] > 0.f) mx = std::max(mx, z[c]);
    }
    float sum = 0.f;
    for (int c = 0; c < C; ++c) {
        p[c] = mask[c] > 0.f ? expf(z[c] - mx) : 0.f;
        sum += p[c];
    }
    for (int c = 0; c < C; ++c) p[c] /= sum;
}

}  // namespace

int select_algorithm(const float *features, int op_kind, float *probs_out) {
    const Workload x = decode(features);
    float mask[C] = {0, 0, 0, 0, 0, 0, 0};
    if (op_kind == 0) mask[0] = mask[1] = mask[6] = 1;
    else mask[2] = mask[3] = mask[4] = mask[5] = 1;
    std::vector<float> w;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        w = g_w;
    }
    if (!w.empty()) {
        float p[C];
        mlp_probs(w.data(), features, mask, p);
        bool ok = true;
        for (int c = 0; c < C; ++c) ok &= std::isfinite(p[c]);
        if (ok) {
            int best = -1;
            for (int c = 0; c < C; ++c)
                if (mask[c] > 0 && (best < 0 || p[c] > p[best])) best = c;
            if (probs_out) memcpy(probs_out, p, sizeof(p));
            return best;
        }
    }
    double t[C];
    if (x.join) cost_join(x, t);
    else cost_groupby(x, t);
    int best = -1;
    for (int c = 0; c < C; ++c)
        if (mask[c] > 0 && (best < 0 || t[c] < t[best])) best = c;
    if (probs_out)
        for (int c = 0; c < C; ++c) probs_out[c] = (c == best) ? 1.f : 0.f;
    return best;
}

void features_join(float *f, double nr, double ns, int key_bytes, int cr, int cs, float mr_hint, float skew_hint) {
    memset(f, 0, 12 * sizeof(float));
    // the match ratio and the skew of the foreign keys are unknown before the
    // join runs: the caller's hints, else every probe row matching and uniform keys
    const double mr = mr_hint > 0.f ? std::min(1.0, (double)mr_hint) : 1.0;
    const double alpha = skew_hint > 0.f ? (double)skew_hint : 0.0;
    f[0] = 1.f;
    f[1] = (float)(std::log2(std::max(1.0, nr)) / 32.0);
    f[2] = (float)(std::log2(std::max(1.0, ns)) / 32.0);
    f[3] = f[1];
    f[4] = key_bytes / 8.f;
    f[5] = cr / 8.f;
    f[6] = cs / 8.f;
    f[7] = (float)(alpha / 1.2);
    f[8] = (float)mr;
    f[9] = (float)(std::log2(std::max(1.0, ns) / std::max(1.0, nr)) / 32.0);
    f[10] = (float)(std::log2(std::max(1.0, mr * ns)) / 32.0);
    f[11] = (float)(std::log2(std::max(1.0, nr * (key_bytes + 4.0 * cr) + ns * (key_bytes + 4.0 * cs))) / 48.0);
}

void features_groupby(float *f, double n, int key_bytes, int nv, double g_est, int varying_bytes, float skew_hint,
                      double rec_bytes) {
    memset(f, 0, 12 * sizeof(float));
    f[0] = 0.f;
    f[1] = (float)(std::log2(std::max(1.0, n)) / 32.0);
    // the group count is unknown before the call (Section 2.2): the estimate,
    // else about n / 16
    const double g = std::max(1.0, g_est > 0.0 ? g_est : n / 16.0);
    f[3] = (float)(std::log2(g) / 32.0);
    f[4] = key_bytes / 8.f;
    f[5] = nv / 8.f;
    // key bytes that vary between rows (a plain radix sort's passes), else all
    f[6] = (varying_bytes > 0 ? varying_bytes : key_bytes) / 8.f;
    f[7] = skew_hint > 0.f ? (float)(skew_hint / 1.2) : 0.f;
    f[8] = 1.f;
    f[9] = (float)(std::log2(std::max(1.0, n / g)) / 32.0);
    // the LDS the hash group-by's records of all groups take: whether they fit one
    // workgroup (Algorithm 1's is_smem_enough) depends on the aggregates, not on g alone
    f[10] = (float)(std::log2(std::max(1.0, g * std::max(4.0, rec_bytes))) / 32.0);
    f[11] = (float)(std::log2(std::max(1.0, n * (key_bytes + 4.0 * nv))) / 48.0);
}

}  // namespace gj

extern "C" {

int gj_cost_model(const float features[12], int32_t op_kind, double predicted_seconds[7]) {
    if (!features || !predicted_seconds || op_kind < 0 || op_kind > 1) return GJ_EINVAL;
    const gj::Workload x = gj::decode(features);
    if (op_kind == 0) gj::cost_join(x, predicted_seconds);
    else gj::cost_groupby(x, predicted_seconds);
    return GJ_OK;
}

int gj_select(const float features[12], int32_t op_kind, int32_t *choice, float probs[7]) {
    if (!features || !choice || op_kind < 0 || op_kind > 1) return GJ_EINVAL;
    *choice = gj::select_algorithm(features, op_kind, probs);
    return GJ_OK;
}

int gj_selector_set_weights(const float *params, int32_t n) {
    std::lock_guard<std::mutex> lk(gj::g_mu);
    if (!params || n == 0) {
        gj::g_w.clear();
        return GJ_OK;
    }
    if (n != GJ_MLP_PARAMS) return GJ_EINVAL;
    gj::g_w.assign(params, params + n);
    return GJ_OK;
}

int gj_get_cost_constants(double *seq_bytes_per_s, double *rand_ratio, double *atomic_rate) {
    if (!seq_bytes_per_s || !rand_ratio || !atomic_rate) return GJ_EINVAL;
    *seq_bytes_per_s = gj::g_c.seq;
    *rand_ratio = gj::g_c.rand_ratio;
    *atomic_rate = gj::g_c.atomic_rate;
    return GJ_OK;
}

int gj_set_cost_constants(double seq_bytes_per_s, double rand_ratio, double atomic_rate) {
    if (!(seq_bytes_per_s > 0) || !(rand_ratio >= 1) || !(atomic_rate > 0)) return GJ_EINVAL;
    gj::g_c.seq = seq_bytes_per_s;
    gj::g_c.rand_ratio = rand_ratio;
    gj::g_c.atomic_rate = atomic_rate;
    return GJ_OK;
}

}  // extern "C"
