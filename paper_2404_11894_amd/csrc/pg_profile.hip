// pg_profile.hip -- optional per-step timing with HIP events recorded on the
// stream each step is launched on.  Host code.
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "pg_api_common.h"

namespace pg {

namespace {
struct Rec {
    std::string name;
    hipEvent_t a, b;
};
struct Recorder {
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
thread_local Recorder g_rec;
}  // namespace

ProfScope::ProfScope(hipStream_t stream, const char* name) : s(stream) {
    if (!g_rec.on) return;
    Rec r{name, g_rec.get(), g_rec.get()};
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    g_rec.recs.push_back(r);
    slot = (int)g_rec.recs.size() - 1;
}

ProfScope::~ProfScope() {
    if (slot >= 0 && slot < (int)g_rec.recs.size()) (void)hipEventRecord(g_rec.recs[slot].b, s);
}

}  // namespace pg

using namespace pg;

extern "C" {

pg_status pg_profile_start(void) {
    g_error.clear();
    for (auto& r : g_rec.recs) {
        g_rec.pool.push_back(r.a);
        g_rec.pool.push_back(r.b);
    }
    g_rec.recs.clear();
    g_rec.on = true;
    return PG_OK;
}

pg_status pg_profile_stop(int32_t max_entries, pg_profile_entry* out, int32_t* n_entries) {
    g_error.clear();
    g_rec.on = false;
    std::map<std::string, pg_profile_entry> agg;
    std::vector<std::string> order;
    for (auto& r : g_rec.recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(PG_ERR_HIP, "hipEventSynchronize failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(PG_ERR_HIP, "hipEventElapsedTime failed");
        auto it = agg.find(r.name);
        if (it == agg.end()) {
            pg_profile_entry e{};
            std::strncpy(e.name, r.name.c_str(), sizeof e.name - 1);
            it = agg.emplace(r.name, e).first;
            order.push_back(r.name);
        }
        it->second.count += 1;
        it->second.total_ms += ms;
        if (ms > it->second.max_ms) it->second.max_ms = ms;
    }
    int32_t n = 0;
    for (auto& name : order) {
        if (out && n < max_entries) out[n] = agg[name];
        ++n;
    }
    if (n_entries) *n_entries = n;
    return PG_OK;
}

}  // extern "C"
