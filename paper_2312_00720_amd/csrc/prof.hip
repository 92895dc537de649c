// Per-launch timing with HIP events, for the benchmark's roofline accounting
// and per-phase breakdowns. Off unless gj_profile_start() was called on the
// thread; then each launch costs two event records on its own stream.
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "internal.hpp"

namespace gj {
namespace {

struct Rec {
    std::string name;
    double bytes;
    hipEvent_t a, b;
};

struct Prof {
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        GJ_HIP(hipEventCreate(&e));
        return e;
    }
};

thread_local Prof g_prof;

}  // namespace

ProfPause::ProfPause() : was(g_prof.on) { g_prof.on = false; }
ProfPause::~ProfPause() { g_prof.on = was; }

void prof_before(const char *name, double alg_bytes, hipStream_t s) {
    if (!g_prof.on) return;
    Rec r{name, alg_bytes, g_prof.take(), g_prof.take()};
    GJ_HIP(hipEventRecord(r.a, s));
    g_prof.recs.push_back(r);
}

void prof_after(hipStream_t s) {
    if (!g_prof.on || g_prof.recs.empty()) return;
    GJ_HIP(hipEventRecord(g_prof.recs.back().b, s));
}

}  // namespace gj

extern "C" {

int gj_profile_start(void) {
    gj::g_prof.on = true;
    gj::g_prof.recs.clear();
    return GJ_OK;
}

int gj_profile_stop(gj_kernel_stat *stats, int32_t cap, int32_t *n_out) {
    gj::Prof &P = gj::g_prof;
    P.on = false;
    struct Acc {
        int64_t launches = 0;
        double ms = 0, bytes = 0;
    };
    std::map<std::string, Acc> acc;
    int rc = GJ_OK;
    for (auto &r : P.recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) rc = GJ_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = GJ_EHIP;
        Acc &x = acc[r.name];
        x.launches += 1;
        x.ms += ms;
        x.bytes += r.bytes;
        P.pool.push_back(r.a);
        P.pool.push_back(r.b);
    }
    P.recs.clear();
    int32_t n = 0;
    for (auto &kv : acc) {
        if (stats && n < cap) {
            gj_kernel_stat &s = stats[n];
            memset(&s, 0, sizeof(s));
            strncpy(s.name, kv.first.c_str(), sizeof(s.name) - 1);
            s.launches = kv.second.launches;
            s.total_ms = kv.second.ms;
            s.alg_bytes = kv.second.bytes;
        }
        ++n;
    }
    if (n_out) *n_out = n;
    return rc;
}

}  // extern "C"
