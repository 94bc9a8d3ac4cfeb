// Launch profiler: each timed launch stamps a pair of HIP events with the
// kernel's start and end; durations are aggregated by kernel name with the
// algorithmic bytes each launch moves.  Off unless enabled.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"

namespace ces {

Profiler& Profiler::get() {
    static Profiler p;
    return p;
}

hipEvent_t Profiler::event() {
    if (used_ < pool_.size()) return pool_[used_++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool_.push_back(e);
    ++used_;
    return e;
}

Profiler::Slot Profiler::begin(const char* name) {
    Slot s;
    if (!on_) return s;
    std::lock_guard<std::mutex> g(mu_);
    if (!only_.empty() && (!name || only_ != name)) return s;
    Rec r;
    r.a = event();
    r.b = event();
    if (!r.a || !r.b) return s;
    recs_.push_back(r);
    s.idx = (int)recs_.size() - 1;
    s.a = r.a;
    s.b = r.b;
    return s;
}

void Profiler::end(const Slot& s, const char* name, double bytes_per_sample, int samples) {
    std::lock_guard<std::mutex> g(mu_);
    if (s.idx < 0 || s.idx >= (int)recs_.size()) return;
    Rec& r = recs_[s.idx];
    r.name = name;
    r.bps = bytes_per_sample;
    r.samples = samples;
}

void Profiler::set_samples(int idx, int samples) {
    std::lock_guard<std::mutex> g(mu_);
    if (idx >= 0 && idx < (int)recs_.size()) recs_[idx].samples = samples;
}

void Profiler::only(const char* name) {
    std::lock_guard<std::mutex> g(mu_);
    only_ = name ? name : "";
}

void Profiler::enable(bool on) {
    std::lock_guard<std::mutex> g(mu_);
    on_ = on;
    recs_.clear();
    used_ = 0;
}

int Profiler::read(std::vector<Entry>& out) {
    std::lock_guard<std::mutex> g(mu_);
    out.clear();
    std::map<std::string, Entry> agg;
    for (const Rec& r : recs_) {
        if (hipEventSynchronize(r.b) != hipSuccess) return -1;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
        Entry& e = agg[r.name ? r.name : "?"];
        e.name = r.name ? r.name : "?";
        e.launches += 1;
        e.ms += ms;
        e.bytes += r.bps * (double)r.samples;
    }
    for (auto& kv : agg) out.push_back(kv.second);
    std::sort(out.begin(), out.end(), [](const Entry& a, const Entry& b) { return a.ms > b.ms; });
    recs_.clear();
    used_ = 0;
    return 0;
}

}  // namespace ces
