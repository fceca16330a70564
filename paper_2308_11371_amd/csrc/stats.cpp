// Kernel statistics and HIP-event timing of individual launches.
#include <algorithm>
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

// timing filter: empty = every family, else a comma-separated list of family names
static bool filter_match(const std::string &filter, const char *name) {
    if (filter.empty()) return true;
    const size_t n = std::strlen(name);
    size_t p = 0;
    while (p <= filter.size()) {
        size_t e = filter.find(',', p);
        if (e == std::string::npos) e = filter.size();
        if (e - p == n && filter.compare(p, n, name) == 0) return true;
        p = e + 1;
    }
    return false;
}

Prof::Prof(ifeti_ctx *c, const char *name, double flops, double bytes, bool in_packet)
    : c_(c), id_(c->no_alloc ? -1 : stat_id(c, name)), in_packet_(in_packet) {
    if (id_ < 0) return;  // allocation-free call: no statistics entries, no events
    KernelStat &k = c->kstats[id_];
    k.launches += 1;
    k.flops += flops;
    k.bytes += bytes;
    if (c->opt.timing && !c->capturing && filter_match(c->opt.timing_filter, name) &&
        (k.launches - 1) % std::max(1, c->opt.timing_every) == 0) {
        k.timed += 1;
        a_ = get_event(c);
        b_ = get_event(c);
        if (!in_packet_) IFETI_HIP(hipEventRecord(a_, c->stream));
    }
}

Prof::~Prof() {
    if (!a_) return;
    if (in_packet_ || hipEventRecord(b_, c_->stream) == hipSuccess) c_->pending.push_back(PendingEvent{id_, a_, b_});
    if (c_->pending.size() > 20000) {
        try {
            flush_events(c_);
        } catch (...) {
        }
    }
}

void flush_events(ifeti_ctx *c) {
    if (c->pending.empty()) return;
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
            c->kstats[p.id].ms += ms;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

const void *read_back(ifeti_ctx *c, const void *dev, size_t bytes) {
    if (bytes > c->h_pin_bytes) {
        IFETI_HIP(hipStreamSynchronize(c->stream));
        if (c->h_pin) (void)hipHostFree(c->h_pin);
        c->h_pin = nullptr;
        c->h_pin_bytes = 0;
        const size_t want = std::max<size_t>(bytes, 1 << 16);
        IFETI_HIP(hipHostMalloc(&c->h_pin, want, hipHostMallocDefault));
        c->h_pin_bytes = want;
    }
    if (!c->ev_poll) IFETI_HIP(hipEventCreateWithFlags(&c->ev_poll, hipEventDisableTiming));
    IFETI_HIP(hipMemcpyAsync(c->h_pin, dev, bytes, hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipEventRecord(c->ev_poll, c->stream));
    for (;;) {
        const hipError_t e = hipEventQuery(c->ev_poll);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) IFETI_HIP(e);
    }
    return c->h_pin;
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
