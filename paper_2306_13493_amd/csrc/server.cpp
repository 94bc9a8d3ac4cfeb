// Serving loop behind ces_server_*: continuous batching of level-sample
// requests with device-memory admission.
//
// Threads: the caller submits; a planner thread runs the plan set-up of
// each new descriptor (Algorithm 1 steps 1-3 on the device, on its own
// stream) and queues the request as ready; the loop thread admits ready
// requests while their memory fits the budget, adds each to a Scheduler
// that runs continuously (new lanes start while others are mid-solve),
// advances the lanes, and completes a request once its done event has
// passed (its results were copied to pinned host memory by then), copying
// them to the caller's buffers.  All device memory comes from one caching
// pool, so completing a request never frees (and never synchronises the
// device) while others run.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>
#include <unordered_map>

#include "plan.hpp"

namespace ces {
namespace {

using Clock = std::chrono::steady_clock;

// Pinned host staging buffers in power-of-two size classes, recycled until
// the server ends.
class PinnedCache {
public:
    ~PinnedCache() {
        for (void* p : all_) (void)hipHostFree(p);
    }
    void* get(size_t bytes) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        {
            std::lock_guard<std::mutex> g(mu_);
            auto& v = free_[c];
            if (!v.empty()) {
                void* p = v.back();
                v.pop_back();
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> g(mu_);
        all_.push_back(p);
        cls_[p] = c;
        return p;
    }
    void put(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu_);
        free_[cls_[p]].push_back(p);
    }

private:
    std::mutex mu_;
    std::map<size_t, std::vector<void*>> free_;
    std::map<void*, size_t> cls_;
    std::vector<void*> all_;
};

struct PlanRef {
    std::string key;
    ces_plan p = nullptr;
    int refs = 0;      // requests holding the plan
    int running = 0;   // of those, admitted and not complete
};

struct Request {
    int64_t id = 0;
    ces_level_desc d{};
    uint64_t seed = 0, first = 0;
    int64_t count = 0;
    double* y_user = nullptr;
    int32_t* st_user = nullptr;
    Clock::time_point t_submit, t_done;
    std::atomic<int> state{0};   // 0 queued, 1 admitted, 2 done, < 0 error
    PlanRef* plan = nullptr;
    double* y_dev = nullptr;
    int32_t* st_dev = nullptr;
    double* y_pin = nullptr;
    int32_t* st_pin = nullptr;
    hipEvent_t done = nullptr;
    std::atomic<int> recorded{0};   // done has been recorded (may be polled)
};

std::string desc_key(const ces_level_desc& d) {
    return std::string(reinterpret_cast<const char*>(&d), sizeof(d));
}

}  // namespace
}  // namespace ces

using namespace ces;

struct ces_server_s {
    ces_context ctx = nullptr;
    size_t budget = 0;
    int max_inflight = 64;
    DevicePool pool;
    PinnedCache pinned;
    StreamPool planner_streams, loop_streams, lane_streams;

    std::mutex mu;
    std::condition_variable cv_plan, cv_loop, cv_done;
    bool stop = false;
    int64_t next_id = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request*> submitted, ready;
    std::list<Request*> running;
    std::unordered_map<std::string, std::unique_ptr<PlanRef>> plans;
    std::list<PlanRef*> idle_plans;   // refs == 0, oldest first
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_admitted_now = 0, samples_done = 0;
    size_t mem_peak = 0;
    int loop_error = CES_OK;
    std::string loop_msg;
    // bytes promised to allocations in progress outside mu (a plan set-up
    // on the planner, a request's workspace and outputs on the loop)
    size_t reserved = 0;

    std::thread planner, loop;

    static constexpr size_t kMaxReady = 8;        // planned ahead of admission
    static constexpr size_t kMaxIdlePlans = 16;   // kept for repeated descriptors

    // the pool can take `need` more bytes within the budget (caller holds mu)
    bool fits(size_t need) const { return pool.in_use() + reserved + need <= budget; }

    // Make room for `need` bytes (caller holds mu): destroy idle plans, then
    // drop the workspaces of plans whose requests are all still queued
    // (they make new ones when admitted), `keep` excepted.
    void evict_for(size_t need, const PlanRef* keep = nullptr) {
        while (!fits(need) && !idle_plans.empty() && evict_one()) {
        }
        for (auto it = plans.begin(); it != plans.end() && !fits(need); ++it) {
            PlanRef* ref = it->second.get();
            if (ref != keep && ref->running == 0 && ref->p->sf) drop_workspace(ref->p);
        }
    }

    void finish_request(Request* r, int state) {
        // caller holds mu
        r->t_done = Clock::now();
        r->state.store(state);
        if (state == 2) {
            ++n_completed;
            samples_done += r->count;
        } else {
            ++n_failed;
        }
        cv_done.notify_all();
        cv_plan.notify_all();   // memory may have come free for a set-up
    }

    void release_plan(PlanRef* ref) {
        // caller holds mu
        if (--ref->refs > 0) return;
        idle_plans.push_back(ref);
        while (idle_plans.size() > kMaxIdlePlans) evict_one();
    }

    bool evict_one() {
        // caller holds mu; only plans without requests (their lanes retired
        // and their work complete) are destroyed
        if (idle_plans.empty()) return false;
        PlanRef* ref = idle_plans.front();
        idle_plans.pop_front();
        ces_plan p = ref->p;
        plans.erase(ref->key);
        ces_plan_destroy(p);
        return true;
    }

    // Once the loop has stopped on an error nothing will run again: every
    // request not yet finished fails with that error (caller holds mu).
    void fail_unfinished() {
        for (Request* r : ready) {
            release_plan(r->plan);
            finish_request(r, loop_error);
        }
        ready.clear();
        for (Request* r : submitted) finish_request(r, loop_error);
        submitted.clear();
    }

    void planner_main() {
        (void)hipSetDevice(ctx->device);
        hipStream_t st = nullptr;
        const bool have_stream = planner_streams.stream(0, &st) == hipSuccess;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_plan.wait(lk, [&] {
                return stop || (!submitted.empty() && (ready.size() < kMaxReady || loop_error != CES_OK));
            });
            if (loop_error != CES_OK) fail_unfinished();
            if (submitted.empty()) {
                if (stop) return;
                continue;
            }
            Request* r = submitted.front();
            const std::string key = desc_key(r->d);
            auto it = plans.find(key);
            if (it != plans.end()) {
                submitted.pop_front();
                PlanRef* ref = it->second.get();
                if (ref->refs == 0) idle_plans.remove(ref);
                ++ref->refs;
                r->plan = ref;
            } else {
                // the set-up's buffers must fit in the budget next to what
                // runs; with nothing admitted, waiting or being set up it
                // goes ahead regardless, so that the stream always moves
                const size_t sb = plan_setup_bytes(&r->d);
                evict_for(sb);
                if (!fits(sb) && !(n_admitted_now == 0 && ready.empty() && reserved == 0)) {
                    cv_plan.wait_for(lk, std::chrono::milliseconds(20));
                    continue;
                }
                submitted.pop_front();
                reserved += sb;
                lk.unlock();
                ces_plan p = nullptr;
                const int rc = have_stream ? plan_create(ctx, &r->d, &pool, st, &p, false) : CES_ERR_DEVICE;
                lk.lock();
                reserved -= sb;
                cv_loop.notify_all();
                if (rc != CES_OK) {
                    finish_request(r, rc);
                    continue;
                }
                auto ref = std::make_unique<PlanRef>();
                ref->key = key;
                ref->p = p;
                ref->refs = 1;
                r->plan = ref.get();
                plans[key] = std::move(ref);
            }
            if (loop_error != CES_OK) {
                // the loop stopped while this request was being planned
                release_plan(r->plan);
                finish_request(r, loop_error);
                continue;
            }
            ready.push_back(r);
            cv_loop.notify_all();
        }
    }

    // device bytes a ready request needs beyond what its plan holds
    size_t need_bytes(const Request* r) const {
        size_t b = DevicePool::charged((size_t)r->count * 8) + DevicePool::charged((size_t)r->count * 4);
        // the workspace's buffers (about twenty), each possibly a slightly
        // larger cached block
        if (!r->plan->p->sf) b += DevicePool::charged(workspace_bytes(r->plan->p, r->count)) + 32 * 256;
        return b;
    }

    int admit(Scheduler& S, Request* r, hipEvent_t ev) {
        void* yd = nullptr;
        void* sd = nullptr;
        CES_HIP(pool.alloc((size_t)r->count * 8, &yd), "request outputs");
        r->y_dev = static_cast<double*>(yd);
        CES_HIP(pool.alloc((size_t)r->count * 4, &sd), "request outputs");
        r->st_dev = static_cast<int32_t*>(sd);
        r->y_pin = static_cast<double*>(pinned.get((size_t)r->count * 8));
        r->st_pin = static_cast<int32_t*>(pinned.get((size_t)r->count * 4));
        if (!r->y_pin || !r->st_pin) return fail(CES_ERR_NOMEM, "pinned staging");
        r->done = ev;
        r->recorded.store(0);
        ces_request q{r->plan->p, r->seed, r->first, r->count, r->y_dev, nullptr, nullptr, nullptr, r->st_dev};
        return S.add(q, ev, r->count, r->y_pin, r->st_pin, &r->recorded);
    }

    void free_request_buffers(Request* r) {
        if (r->y_dev) pool.release(r->y_dev);
        if (r->st_dev) pool.release(r->st_dev);
        pinned.put(r->y_pin);
        pinned.put(r->st_pin);
        r->y_dev = nullptr;
        r->st_dev = nullptr;
        r->y_pin = nullptr;
        r->st_pin = nullptr;
    }

    void loop_main() {
        (void)hipSetDevice(ctx->device);
        hipStream_t caller = nullptr;
        if (loop_streams.stream(0, &caller) != hipSuccess) {
            std::lock_guard<std::mutex> g(mu);
            loop_error = CES_ERR_DEVICE;
            return;
        }
        ces_schedule sched = ctx->sched;
        Scheduler S(lane_streams, caller, sched);
        std::vector<hipEvent_t> free_events;
        size_t next_event = 1;
        auto get_event = [&](hipEvent_t* e) -> hipError_t {
            if (!free_events.empty()) {
                *e = free_events.back();
                free_events.pop_back();
                return hipSuccess;
            }
            return loop_streams.event(next_event++, e);
        };
        std::vector<ces_plan> released;
        for (;;) {
            bool did = false;
            // admission: memory and in-flight limits; always admit when
            // nothing runs so that one oversized request still proceeds
            {
                std::unique_lock<std::mutex> lk(mu);
                while (!ready.empty() && n_admitted_now < max_inflight) {
                    Request* r = ready.front();
                    const size_t need = need_bytes(r);
                    evict_for(need, r->plan);
                    if (!fits(need) && (n_admitted_now > 0 || reserved > 0)) break;
                    ready.pop_front();
                    cv_plan.notify_all();
                    hipEvent_t ev = nullptr;
                    reserved += need;
                    ++r->plan->running;   // its workspace is in use from here on
                    lk.unlock();
                    int rc = get_event(&ev) == hipSuccess ? admit(S, r, ev) : CES_ERR_DEVICE;
                    lk.lock();
                    reserved -= need;
                    if (rc != CES_OK) {
                        free_request_buffers(r);
                        if (ev) free_events.push_back(ev);
                        --r->plan->running;
                        release_plan(r->plan);
                        finish_request(r, rc);
                        continue;
                    }
                    r->state.store(1);
                    ++n_admitted_now;
                    running.push_back(r);
                    mem_peak = std::max(mem_peak, pool.in_use());
                    did = true;
                }
            }
            bool prog = false;
            int rc = S.step(&prog);
            if (rc == CES_OK) rc = S.retire(&released);
            released.clear();
            if (rc != CES_OK) {
                const std::string msg = ces_last_error();
                // end the scheduler's use of the plans before their
                // references go, so that none is destroyed under a lane
                (void)S.join();
                std::lock_guard<std::mutex> g(mu);
                loop_error = rc;
                loop_msg = msg;
                for (Request* r : running) {
                    --r->plan->running;
                    release_plan(r->plan);
                    --n_admitted_now;
                    finish_request(r, rc);
                }
                running.clear();
                fail_unfinished();
                cv_plan.notify_all();
                return;
            }
            did = did || prog;
            // completions: results are in pinned memory once `done` passed
            for (auto it = running.begin(); it != running.end();) {
                Request* r = *it;
                if (!r->recorded.load()) {
                    ++it;
                    continue;
                }
                const hipError_t q = hipEventQuery(r->done);
                if (q == hipErrorNotReady) {
                    (void)hipGetLastError();
                    ++it;
                    continue;
                }
                std::memcpy(r->y_user, r->y_pin, (size_t)r->count * 8);
                bool ok = q == hipSuccess;
                if (r->st_user) std::memcpy(r->st_user, r->st_pin, (size_t)r->count * 4);
                std::lock_guard<std::mutex> g(mu);
                free_request_buffers(r);
                free_events.push_back(r->done);
                r->done = nullptr;
                --r->plan->running;
                release_plan(r->plan);
                --n_admitted_now;
                finish_request(r, ok ? 2 : CES_ERR_DEVICE);
                it = running.erase(it);
                did = true;
            }
            if (did) continue;
            std::unique_lock<std::mutex> lk(mu);
            if (running.empty() && ready.empty()) {
                if (stop && submitted.empty()) return;
                cv_loop.wait_for(lk, std::chrono::milliseconds(50));
            } else if (!running.empty() && S.pending_solves() == 0) {
                // only copies and finalizes in flight
                lk.unlock();
                std::this_thread::yield();
            } else {
                lk.unlock();
                std::this_thread::yield();
            }
        }
    }
};

extern "C" {

int ces_server_create(ces_context ctx, size_t mem_budget_bytes, int32_t max_inflight, ces_server* out) {
    if (!ctx || !out) return fail(CES_ERR_ARG, "context or out is NULL");
    *out = nullptr;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    auto* s = new ces_server_s;
    s->ctx = ctx;
    s->budget = mem_budget_bytes ? mem_budget_bytes : (size_t)(0.9 * (double)ctx->budget);
    s->max_inflight = max_inflight > 0 ? max_inflight : 64;
    s->planner = std::thread([s] { s->planner_main(); });
    s->loop = std::thread([s] { s->loop_main(); });
    *out = s;
    return CES_OK;
}

int ces_server_submit(ces_server s, const ces_level_desc* desc, uint64_t seed, uint64_t first, int64_t count,
                      double* y_host, int32_t* status_host, int64_t* request_id) {
    if (!s || !request_id) return fail(CES_ERR_ARG, "server or request_id is NULL");
    int rc = validate_desc(desc);
    if (rc != CES_OK) return rc;
    if (count <= 0) return fail(CES_ERR_ARG, "count must be > 0");
    if (!y_host) return fail(CES_ERR_ARG, "y_host is NULL");
    if (first + (uint64_t)count < first) return fail(CES_ERR_ARG, "sample range overflows");
    auto r = std::make_unique<Request>();
    r->d = *desc;
    r->seed = seed;
    r->first = first;
    r->count = count;
    r->y_user = y_host;
    r->st_user = status_host;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(CES_ERR_BUSY, "server is shutting down");
    if (s->loop_error != CES_OK) return fail(s->loop_error, "server loop stopped: " + s->loop_msg);
    r->id = s->next_id++;
    *request_id = r->id;
    s->submitted.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    ++s->n_submitted;
    s->cv_plan.notify_all();
    return CES_OK;
}

int ces_server_poll(ces_server s, int64_t id, int32_t* state, double* latency_s) {
    if (!s || !state) return fail(CES_ERR_ARG, "server or state is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(CES_ERR_ARG, "unknown request id");
    Request* r = it->second.get();
    const int st = r->state.load();
    *state = st;
    if (latency_s) {
        const auto end = (st == 2 || st < 0) ? r->t_done : Clock::now();
        *latency_s = std::chrono::duration<double>(end - r->t_submit).count();
    }
    return CES_OK;
}

int ces_server_drain(ces_server s) {
    if (!s) return fail(CES_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->n_completed + s->n_failed == s->n_submitted; });
    if (s->loop_error != CES_OK) return fail(s->loop_error, "server loop stopped: " + s->loop_msg);
    return CES_OK;
}

int ces_server_get_stats(ces_server s, ces_server_stats* out) {
    if (!s || !out) return fail(CES_ERR_ARG, "server or out is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->failed = s->n_failed;
    out->admitted = s->n_admitted_now;
    out->queued = s->n_submitted - s->n_completed - s->n_failed - s->n_admitted_now;
    out->samples_done = s->samples_done;
    out->mem_in_use = s->pool.in_use();
    out->mem_peak = s->mem_peak;
    out->plans_cached = (int32_t)s->plans.size();
    return CES_OK;
}

int ces_server_destroy(ces_server s) {
    if (!s) return CES_OK;
    (void)ces_server_drain(s);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_plan.notify_all();
    s->cv_loop.notify_all();
    s->planner.join();
    s->loop.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : s->plans) ces_plan_destroy(kv.second->p);
    s->plans.clear();
    delete s;
    return CES_OK;
}

}  // extern "C"
