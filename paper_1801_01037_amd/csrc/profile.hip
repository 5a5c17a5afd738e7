// Per-launch timing with HIP events on the handle's stream: each profiled
// launch is bracketed by two events, and sv_profile_read sums the elapsed
// times per kernel class together with the algorithmic bytes and flops the
// launches had to move and compute.
#include <cstring>

#include "sv_internal.h"

namespace svk {

const char *class_name(int cls)
{
    static const char *names[KC_COUNT] = {"init", "pair", "pair_ctrl", "swap", "diag",
                                          "tile", "dense", "norm", "probs", "batch",
                                          "sample", "graph"};
    return (cls >= 0 && cls < KC_COUNT) ? names[cls] : "?";
}

static hipEvent_t take_event(Profiler &p)
{
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(sv_state s)
{
    if (!s->prof.on) return -1;
    ProfRec r{};
    r.start = take_event(s->prof);
    r.stop = take_event(s->prof);
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, s->stream) != hipSuccess) return -1;
    s->prof.recs.push_back(r);
    return int(s->prof.recs.size() - 1);
}

void prof_end(sv_state s, int token, int cls, double bytes, double flops)
{
    if (token < 0 || size_t(token) >= s->prof.recs.size()) return;
    ProfRec &r = s->prof.recs[token];
    r.cls = cls;
    r.bytes = bytes;
    r.flops = flops;
    (void)hipEventRecord(r.stop, s->stream);
}

static void recycle(Profiler &p)
{
    for (ProfRec &r : p.recs) {
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.recs.clear();
}

void prof_release(sv_state s)
{
    recycle(s->prof);
    for (hipEvent_t e : s->prof.pool) (void)hipEventDestroy(e);
    s->prof.pool.clear();
}

}  // namespace svk

extern "C" {

sv_status sv_profile(sv_state s, int enable)
{
    if (!s) return SV_EINVAL;
    if (enable) {
        (void)hipStreamSynchronize(s->stream);
        svk::recycle(s->prof);
    }
    s->prof.on = enable != 0;
    return SV_OK;
}

sv_status sv_profile_read(sv_state s, sv_prof_entry *out, int max_entries, int *n_entries)
{
    if (!s || !n_entries || (max_entries > 0 && !out)) return SV_EINVAL;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return SV_EDEVICE;
    sv_prof_entry agg[svk::KC_COUNT];
    std::memset(agg, 0, sizeof agg);
    for (int c = 0; c < svk::KC_COUNT; ++c)
        std::strncpy(agg[c].name, svk::class_name(c), sizeof agg[c].name - 1);
    for (const svk::ProfRec &r : s->prof.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) continue;
        sv_prof_entry &e = agg[r.cls];
        e.launches += 1;
        e.total_ms += ms;
        e.bytes += r.bytes;
        e.flops += r.flops;
    }
    int k = 0;
    for (int c = 0; c < svk::KC_COUNT; ++c) {
        if (agg[c].launches == 0) continue;
        if (k < max_entries) out[k] = agg[c];
        ++k;
    }
    *n_entries = k;
    return SV_OK;
}

}  // extern "C"
