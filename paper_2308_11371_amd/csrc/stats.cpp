// Kernel statistics and HIP-event timing of individual launches.
#include <cstring>

#include "common.hpp"

namespace ifeti {

static int stat_id(ifeti_ctx *c, const char *name) {
    for (size_t i = 0; i < c->kstats.size(); ++i)
        if (c->kstats[i].name == name) return (int)i;
    c->kstats.push_back(KernelStat{name});
    return (int)c->kstats.size() - 1;
}

static hipEvent_t get_event(ifeti_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    IFETI_HIP(hipEventCreate(&e));
    return e;
}

Prof::Prof(ifeti_ctx *c, const char *name, double flops, double bytes) : c_(c), id_(stat_id(c, name)) {
    KernelStat &k = c->kstats[id_];
    k.launches += 1;
    k.flops += flops;
    k.bytes += bytes;
    if (c->opt.timing && (c->opt.timing_filter.empty() || c->opt.timing_filter == name)) {
        a_ = get_event(c);
        IFETI_HIP(hipEventRecord(a_, c->stream));
    }
}

Prof::~Prof() {
    if (!a_) return;
    hipEvent_t b = nullptr;
    try {
        b = get_event(c_);
    } catch (...) {
        return;
    }
    if (hipEventRecord(b, c_->stream) == hipSuccess) c_->pending.push_back(PendingEvent{id_, a_, b});
    if (c_->pending.size() > 20000) flush_events(c_);
}

void flush_events(ifeti_ctx *c) {
    if (c->pending.empty()) return;
    IFETI_HIP(hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) c->kstats[p.id].ms += ms;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

void release_events(ifeti_ctx *c) {
    (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    c->pending.clear();
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
}

}  // namespace ifeti
