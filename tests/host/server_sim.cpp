// Scenarios for the serving loop and the batch scheduler on the host (test
// infrastructure): the library's server.cpp and exec.cpp, compiled
// unchanged, run over the stand-in device layer of fake_device.cpp and the
// stand-in HIP runtime of fake_hip.cpp, under ASan and UBSan.
//
//   server_sim <scenario>      prints "ok <scenario>" and exits 0, or
//                              prints the failed check and exits 1
//
// A watchdog aborts a scenario that runs longer than 120 s (a hung drain).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include <unistd.h>

#include "plan.hpp"

extern "C" {
void fake_hip_set_capacity(size_t bytes);
size_t fake_hip_live_bytes();
void fake_device_fail_after(long long n);
void fake_device_set_iteration_delay_us(int us);
int fake_device_max_concurrent_solves();
void fake_device_reset_counters();
long long fake_device_solves();
}

namespace {

using Clock = std::chrono::steady_clock;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                         ces_last_error());                                          \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

// Y of sample i under the stand-in device layer (see fake_device.cpp)
double expected_y(const ces_level_desc& d, uint64_t seed, uint64_t i) {
    const double im = (double)(i % (seed >= 1000000 ? 16 : 100000));
    const double fine = 3.0 * im + (double)(seed % 7) + 11.0 * d.stream + d.m_fine;
    return d.level_kind == CES_LEVEL_PAIR ? fine - (im + d.m_fine / 2) : fine;
}

ces_level_desc desc(int m, bool pair, int prec = CES_PREC_MIXED, int field = CES_FIELD_PAIR, uint32_t tag = 0) {
    ces_level_desc d;
    ces_level_desc_default(&d);
    d.m_fine = m;
    d.level_kind = pair ? CES_LEVEL_PAIR : CES_LEVEL_SINGLE;
    d.precision = prec;
    d.field_mode = field;
    d.stream = tag;
    return d;
}

ces_context make_ctx(size_t budget) {
    auto* c = new ces_context_s;
    c->budget = budget;
    c->sched.depth = 2;
    return c;
}

struct Req {
    ces_level_desc d;
    uint64_t seed = 0, first = 0;
    int64_t count = 0;
    std::vector<double> y;
    std::vector<int32_t> status;
    int64_t id = 0;
};

void submit(ces_server s, Req& r) {
    r.y.assign(r.count, -1.0);
    r.status.assign(r.count, 99);
    CHECK(ces_server_submit(s, &r.d, r.seed, r.first, r.count, r.y.data(), r.status.data(), &r.id) == CES_OK);
}

void check_result(const Req& r) {
    for (int64_t t = 0; t < r.count; ++t) {
        if (r.y[t] != expected_y(r.d, r.seed, r.first + t) || r.status[t] != 0) {
            std::fprintf(stderr, "request %lld sample %lld: y %.17g expected %.17g status %d\n", (long long)r.id,
                         (long long)t, r.y[t], expected_y(r.d, r.seed, r.first + t), r.status[t]);
            std::exit(1);
        }
    }
}

int state_of(ces_server s, const Req& r, double* lat = nullptr) {
    int32_t st = 0;
    CHECK(ces_server_poll(s, r.id, &st, lat) == CES_OK);
    return st;
}

std::vector<Req> random_requests(int n, unsigned seed, int mmax, bool fail_some = false) {
    std::mt19937_64 g(seed);
    std::vector<Req> v(n);
    const int ms[] = {8, 16, 32, 64, 128, 256, 512};
    for (int i = 0; i < n; ++i) {
        int m = ms[g() % 7];
        while (m > mmax) m /= 2;
        const bool pair = m >= 16 && (g() % 4) != 0;
        v[i].d = desc(m, pair, (g() % 3) ? CES_PREC_MIXED : CES_PREC_FP64,
                      (g() % 3) ? CES_FIELD_PAIR : CES_FIELD_HARTLEY, (uint32_t)(g() % 3));
        if (fail_some && i % 7 == 3) {
            v[i].d.psd_policy = CES_PSD_FAIL;
            v[i].d.lambda = 2.0;
        }
        v[i].seed = g() % 1000;
        v[i].first = g() % 5000;
        v[i].count = 1 + (int64_t)(g() % 256);
    }
    return v;
}

// ---------------------------------------------------------------- batch --
// ces_sample_batch: every request's outputs by sample index, whatever the
// chunking; a plan may appear in several requests.
void scenario_batch() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    std::vector<ces_level_desc> ds = {desc(16, false), desc(32, true, CES_PREC_FP64, CES_FIELD_PAIR, 1),
                                      desc(64, true, CES_PREC_MIXED, CES_FIELD_HARTLEY, 2),
                                      desc(128, true, CES_PREC_MIXED, CES_FIELD_PAIR, 3)};
    std::vector<ces_plan> plans;
    for (auto& d : ds) {
        ces_plan p = nullptr;
        CHECK(ces::plan_create(ctx, &d, ces::default_allocator(), nullptr, &p) == CES_OK);
        plans.push_back(p);
    }
    for (long long chunk : {0LL, 7LL, 64LL}) {
        ces_schedule sc{};
        sc.depth = chunk == 7 ? 1 : 3;
        sc.max_lanes = chunk == 64 ? 1 : 0;
        sc.chunk_samples = chunk;
        CHECK(ces_schedule_set(ctx, &sc) == CES_OK);
        struct Out { int plan; uint64_t first; int64_t count; double* y; int32_t* st; };
        std::vector<Out> outs;
        std::vector<ces_request> reqs;
        const int64_t counts[] = {1, 33, 200, 0, 5, 77};
        for (int i = 0; i < 6; ++i) {
            Out o{i % 4, (uint64_t)(3 * i + 1), counts[i], nullptr, nullptr};
            void* y = nullptr;
            void* st = nullptr;
            CHECK(hipMalloc(&y, 8 * (size_t)std::max<int64_t>(o.count, 1)) == hipSuccess);
            CHECK(hipMalloc(&st, 4 * (size_t)std::max<int64_t>(o.count, 1)) == hipSuccess);
            o.y = (double*)y;
            o.st = (int32_t*)st;
            outs.push_back(o);
            reqs.push_back(ces_request{plans[o.plan], 42, o.first, o.count, o.y, nullptr, nullptr, nullptr, o.st});
        }
        CHECK(ces_sample_batch(ctx, reqs.data(), (int32_t)reqs.size(), nullptr) == CES_OK);
        for (auto& o : outs) {
            for (int64_t t = 0; t < o.count; ++t) {
                CHECK(o.y[t] == expected_y(ds[o.plan], 42, o.first + t));
                CHECK(o.st[t] == 0);
            }
            CHECK(hipFree(o.y) == hipSuccess);
            CHECK(hipFree(o.st) == hipSuccess);
        }
    }
    // a plan in two concurrent calls is refused, not corrupted
    CHECK(plans[0]->busy.load() == 0);
    for (ces_plan p : plans) ces_plan_destroy(p);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

// ces_autotune with CESMLMC_AUTOTUNE_CACHE: the first call tunes and
// stores its choice; a second call on the same batch applies the stored
// choice and runs the batch once, outputs complete.
void scenario_autotune_cache() {
    char path[64];
    std::snprintf(path, sizeof(path), "/tmp/ces_autotune_%d.txt", (int)getpid());
    std::remove(path);
    setenv("CESMLMC_AUTOTUNE_CACHE", path, 1);
    ces_context ctx = make_ctx((size_t)8 << 30);
    std::vector<ces_level_desc> ds = {desc(16, false), desc(64, true, CES_PREC_MIXED, CES_FIELD_PAIR, 1),
                                      desc(128, true, CES_PREC_MIXED, CES_FIELD_PAIR, 2)};
    std::vector<ces_plan> plans;
    for (auto& d : ds) {
        ces_plan p = nullptr;
        CHECK(ces::plan_create(ctx, &d, ces::default_allocator(), nullptr, &p) == CES_OK);
        plans.push_back(p);
    }
    const int64_t counts[] = {300, 40, 9};
    std::vector<ces_request> reqs;
    for (int i = 0; i < 3; ++i) {
        void* y = nullptr;
        CHECK(hipMalloc(&y, 8 * (size_t)counts[i]) == hipSuccess);
        reqs.push_back(ces_request{plans[i], 9, 0, counts[i], (double*)y, nullptr, nullptr, nullptr, nullptr});
    }
    auto check_outputs = [&] {
        for (int i = 0; i < 3; ++i)
            for (int64_t t = 0; t < counts[i]; ++t) CHECK(reqs[i].y[t] == expected_y(ds[i], 9, (uint64_t)t));
    };
    // solves of one plain run of the batch
    fake_device_reset_counters();
    CHECK(ces_sample_batch(ctx, reqs.data(), 3, nullptr) == CES_OK);
    const long long one_run = fake_device_solves();
    ces_schedule s1{}, s2{};
    double ms1 = 0.0, ms2 = 0.0;
    fake_device_reset_counters();
    CHECK(ces_autotune(ctx, reqs.data(), 3, nullptr, &s1, &ms1) == CES_OK);
    CHECK(fake_device_solves() > 3 * one_run);   // tuned: many runs
    check_outputs();
    for (auto& r : reqs) std::memset(r.y, 0, 8 * (size_t)r.count);
    ces_schedule def{};
    def.depth = 2;
    CHECK(ces_schedule_set(ctx, &def) == CES_OK);
    fake_device_reset_counters();
    CHECK(ces_autotune(ctx, reqs.data(), 3, nullptr, &s2, &ms2) == CES_OK);
    CHECK(fake_device_solves() == one_run);      // stored: one run
    check_outputs();
    CHECK(s2.depth == s1.depth && s2.max_lanes == s1.max_lanes && s2.chunk_samples == s1.chunk_samples &&
          s2.graphs == s1.graphs);
    CHECK(std::fabs(ms2 - ms1) <= 1e-4 + 1e-6 * ms1);
    ces_schedule now{};
    CHECK(ces_schedule_get(ctx, &now) == CES_OK && now.depth == s1.depth && now.chunk_samples == s1.chunk_samples);
    // another batch (other counts) is not served from the stored choice
    reqs[0].count = 200;
    fake_device_reset_counters();
    CHECK(ces_autotune(ctx, reqs.data(), 3, nullptr, &s2, &ms2) == CES_OK);
    CHECK(fake_device_solves() > 3 * one_run);
    FILE* f = std::fopen(path, "r");
    CHECK(f != nullptr);
    int lines = 0;
    char buf[256];
    while (std::fgets(buf, sizeof(buf), f)) ++lines;
    std::fclose(f);
    CHECK(lines == 2);
    std::remove(path);
    unsetenv("CESMLMC_AUTOTUNE_CACHE");
    for (auto& r : reqs) CHECK(hipFree(r.y) == hipSuccess);
    for (ces_plan p : plans) ces_plan_destroy(p);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

// ces_mlmc_run_checkpointed: a run stopped after every round and resumed
// from its checkpoint file gives the uninterrupted run's result bit for bit;
// a checkpoint of other options is refused.
void scenario_mlmc_checkpoint() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    std::vector<ces_plan> plans;
    for (int l = 0; l < 4; ++l) {
        ces_level_desc d = desc(16 << l, l > 0, CES_PREC_MIXED, CES_FIELD_PAIR, (uint32_t)l);
        ces_plan p = nullptr;
        CHECK(ces::plan_create(ctx, &d, ces::default_allocator(), nullptr, &p) == CES_OK);
        plans.push_back(p);
    }
    ces_mlmc_opts o;
    ces_mlmc_opts_default(&o);
    o.eps = 2.0;
    o.l_start = 1;
    o.n_pilot = 6;
    o.max_rounds = 12;
    o.seed = 1000003;   // bounded level variances (fake_device.cpp)
    ces_mlmc_result a{}, b{};
    CHECK(ces_mlmc_run(ctx, plans.data(), nullptr, 4, &o, nullptr, &a) == CES_OK);
    CHECK(a.rounds >= 3);
    char path[64];
    std::snprintf(path, sizeof(path), "/tmp/ces_mlmc_ckpt_%d.json", (int)getpid());
    std::remove(path);
    int calls = 0, last = -1;
    for (;;) {
        std::memset(&b, 0, sizeof(b));
        CHECK(ces_mlmc_run_checkpointed(ctx, plans.data(), nullptr, 4, &o, path, 1, nullptr, &b) == CES_OK);
        ++calls;
        if (b.rounds == last) break;   // nothing left to do
        last = b.rounds;
        CHECK(calls < 100);
    }
    CHECK(calls == a.rounds + 1);
    CHECK(std::memcmp(&a, &b, sizeof(a)) == 0);
    // the finished checkpoint of other options (another seed) is refused
    ces_mlmc_opts o2 = o;
    o2.seed = 1000004;
    CHECK(ces_mlmc_run_checkpointed(ctx, plans.data(), nullptr, 4, &o2, path, 0, nullptr, &b) == CES_ERR_ARG);
    std::remove(path);
    for (ces_plan p : plans) ces_plan_destroy(p);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

// ------------------------------------------------------------- serving --
// Mixed requests, shared descriptors, results equal to the per-sample
// formula; every device byte is back once the server is gone.
void scenario_serve_mix() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, 0, 0, &s) == CES_OK);
    auto reqs = random_requests(120, 1, 256);
    for (auto& r : reqs) submit(s, r);
    CHECK(ces_server_drain(s) == CES_OK);
    for (auto& r : reqs) {
        CHECK(state_of(s, r) == 2);
        check_result(r);
    }
    ces_server_stats st{};
    CHECK(ces_server_get_stats(s, &st) == CES_OK);
    CHECK(st.completed == 120 && st.failed == 0 && st.queued == 0 && st.admitted == 0);
    CHECK(ces_server_destroy(s) == CES_OK);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

// Admission by memory: the pool never holds more than the budget while
// more than one request runs, requests still overlap, and a request larger
// than the budget runs alone.
void scenario_admission() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    fake_device_set_iteration_delay_us(200);
    ces_level_desc d = desc(64, true);
    ces_plan probe = nullptr;
    CHECK(ces::plan_create(ctx, &d, ces::default_allocator(), nullptr, &probe) == CES_OK);
    const size_t one = ces::workspace_bytes(probe, 64) + 64 * 12 + 512;
    ces_plan_destroy(probe);
    // room for about three requests of 64 samples (plans take a little more)
    const size_t budget = 3 * one + one / 2;
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, budget, 0, &s) == CES_OK);
    fake_device_reset_counters();
    std::vector<Req> reqs(24);
    for (int i = 0; i < 24; ++i) {
        // each request its own descriptor, so each needs its own workspace
        reqs[i].d = desc(64, true, CES_PREC_MIXED, CES_FIELD_PAIR, (uint32_t)i);
        reqs[i].seed = (uint64_t)i;
        reqs[i].count = 64;
        submit(s, reqs[i]);
    }
    int max_admitted = 0, max_queued = 0;
    for (;;) {
        ces_server_stats st{};
        CHECK(ces_server_get_stats(s, &st) == CES_OK);
        max_admitted = std::max<int>(max_admitted, (int)st.admitted);
        max_queued = std::max<int>(max_queued, (int)st.queued);
        if (st.completed + st.failed == 24) break;
        std::this_thread::sleep_for(std::chrono::microseconds(300));
    }
    CHECK(ces_server_drain(s) == CES_OK);
    for (auto& r : reqs) check_result(r);
    ces_server_stats st{};
    CHECK(ces_server_get_stats(s, &st) == CES_OK);
    CHECK(st.mem_peak <= budget);
    CHECK(max_admitted >= 2 && max_admitted <= 3);
    CHECK(max_queued >= 10);
    CHECK(fake_device_max_concurrent_solves() >= 2);
    // one request needing more than the whole budget still runs, alone
    Req big;
    big.d = desc(64, true);
    big.count = 400;
    submit(s, big);
    CHECK(ces_server_drain(s) == CES_OK);
    check_result(big);
    CHECK(ces_server_destroy(s) == CES_OK);
    CHECK(fake_hip_live_bytes() == 0);
    fake_device_set_iteration_delay_us(0);
    delete ctx;
}

// Continuous batching: a request submitted while a long one is running is
// admitted at once and completes while the long one is still running.
void scenario_continuous() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    fake_device_set_iteration_delay_us(2000);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, 0, 0, &s) == CES_OK);
    Req a;
    a.d = desc(512, true);   // 66 + 34 iterations of 2 ms on two streams
    a.count = 4;
    submit(s, a);
    const auto t0 = Clock::now();
    while (state_of(s, a) == 0) {
        CHECK(Clock::now() - t0 < std::chrono::seconds(20));
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    std::vector<Req> small(3);
    for (int i = 0; i < 3; ++i) {
        small[i].d = desc(16 << i, i > 0, CES_PREC_MIXED, CES_FIELD_PAIR, (uint32_t)(1 + i));
        small[i].seed = 5;
        small[i].count = 10;
        submit(s, small[i]);
    }
    for (auto& r : small) {
        while (state_of(s, r) != 2) {
            CHECK(state_of(s, r) >= 0);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        check_result(r);
    }
    CHECK(state_of(s, a) == 1);   // still running: the small ones overtook it
    CHECK(ces_server_drain(s) == CES_OK);
    check_result(a);
    double la = 0, lb = 0;
    state_of(s, a, &la);
    state_of(s, small[0], &lb);
    CHECK(lb < la);
    CHECK(ces_server_destroy(s) == CES_OK);
    fake_device_set_iteration_delay_us(0);
    delete ctx;
}

// Overload: many more requests than may run at once, submitted from four
// threads; the in-flight cap holds and everything completes.
void scenario_overload() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    fake_device_set_iteration_delay_us(20);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, (size_t)1 << 30, 4, &s) == CES_OK);
    fake_device_reset_counters();
    std::vector<std::vector<Req>> per(4);
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t) {
        per[t] = random_requests(100, 10 + t, 128);
        th.emplace_back([&, t] {
            for (auto& r : per[t]) submit(s, r);
        });
    }
    int max_admitted = 0;
    for (;;) {
        ces_server_stats st{};
        CHECK(ces_server_get_stats(s, &st) == CES_OK);
        max_admitted = std::max<int>(max_admitted, (int)st.admitted);
        if (st.submitted == 400 && st.completed + st.failed == 400) break;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    for (auto& x : th) x.join();
    CHECK(ces_server_drain(s) == CES_OK);
    for (auto& v : per)
        for (auto& r : v) check_result(r);
    CHECK(max_admitted <= 4);
    CHECK(fake_device_max_concurrent_solves() <= 8);   // fine + coarse per request
    ces_server_stats st{};
    CHECK(ces_server_get_stats(s, &st) == CES_OK);
    CHECK(st.mem_peak <= ((size_t)1 << 30));
    CHECK(ces_server_destroy(s) == CES_OK);
    CHECK(fake_hip_live_bytes() == 0);
    fake_device_set_iteration_delay_us(0);
    delete ctx;
}

// Failure isolation: a request whose plan cannot be made, and one whose
// workspace cannot be allocated, fail alone.
void scenario_isolation() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, 0, 2, &s) == CES_OK);
    auto reqs = random_requests(40, 3, 128, true);
    for (auto& r : reqs) submit(s, r);
    CHECK(ces_server_drain(s) == CES_OK);
    int failed = 0;
    for (auto& r : reqs) {
        if (r.d.psd_policy == CES_PSD_FAIL) {
            CHECK(state_of(s, r) == CES_ERR_NOT_PSD);
            ++failed;
        } else {
            CHECK(state_of(s, r) == 2);
            check_result(r);
        }
    }
    CHECK(failed >= 5);
    // device memory exhausted for one request: it fails, later ones run
    fake_hip_set_capacity(fake_hip_live_bytes() + ((size_t)64 << 20));
    Req huge;
    huge.d = desc(512, true, CES_PREC_FP64);
    huge.count = 256;
    submit(s, huge);
    CHECK(ces_server_drain(s) == CES_OK);
    CHECK(state_of(s, huge) == CES_ERR_NOMEM);
    fake_hip_set_capacity((size_t)1 << 40);
    Req after;
    after.d = desc(32, true);
    after.count = 9;
    submit(s, after);
    CHECK(ces_server_drain(s) == CES_OK);
    check_result(after);
    ces_server_stats st{};
    CHECK(ces_server_get_stats(s, &st) == CES_OK);
    CHECK(st.failed == failed + 1 && st.completed == (int64_t)reqs.size() - failed + 1);
    CHECK(ces_server_destroy(s) == CES_OK);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

// A device error in the loop stops it: every request not complete fails
// with the error (those still queued or being planned too), drain and
// destroy return, and new submissions are refused.
void scenario_loop_error() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    fake_device_set_iteration_delay_us(300);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, 0, 2, &s) == CES_OK);
    auto reqs = random_requests(60, 4, 128);
    for (auto& r : reqs) submit(s, r);
    fake_device_fail_after(12);
    CHECK(ces_server_drain(s) == CES_ERR_DEVICE);
    int done = 0, failed = 0;
    for (auto& r : reqs) {
        const int st = state_of(s, r);
        CHECK(st == 2 || st == CES_ERR_DEVICE);
        if (st == 2) {
            check_result(r);
            ++done;
        } else {
            ++failed;
        }
    }
    CHECK(failed >= 40 && done + failed == 60);
    ces_server_stats st{};
    CHECK(ces_server_get_stats(s, &st) == CES_OK);
    CHECK(st.completed == done && st.failed == failed && st.admitted == 0 && st.queued == 0);
    Req late;
    late.d = desc(16, false);
    late.count = 1;
    late.y.assign(1, 0.0);
    int64_t id = 0;
    CHECK(ces_server_submit(s, &late.d, 0, 0, 1, late.y.data(), nullptr, &id) == CES_ERR_DEVICE);
    CHECK(ces_server_destroy(s) == CES_OK);
    CHECK(fake_hip_live_bytes() == 0);
    fake_device_set_iteration_delay_us(0);
    delete ctx;
}

// Destroy right after submitting drains first.
void scenario_destroy_pending() {
    ces_context ctx = make_ctx((size_t)8 << 30);
    ces_server s = nullptr;
    CHECK(ces_server_create(ctx, 0, 0, &s) == CES_OK);
    auto reqs = random_requests(30, 5, 256);
    for (auto& r : reqs) submit(s, r);
    CHECK(ces_server_destroy(s) == CES_OK);
    for (auto& r : reqs) check_result(r);
    CHECK(fake_hip_live_bytes() == 0);
    delete ctx;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: server_sim <scenario>\n");
        return 2;
    }
    const std::string sc = argv[1];
    std::thread([sc] {
        std::this_thread::sleep_for(std::chrono::seconds(120));
        std::fprintf(stderr, "watchdog: scenario %s still running after 120 s\n", sc.c_str());
        std::_Exit(3);
    }).detach();
    if (sc == "batch") scenario_batch();
    else if (sc == "autotune_cache") scenario_autotune_cache();
    else if (sc == "mlmc_checkpoint") scenario_mlmc_checkpoint();
    else if (sc == "serve_mix") scenario_serve_mix();
    else if (sc == "admission") scenario_admission();
    else if (sc == "continuous") scenario_continuous();
    else if (sc == "overload") scenario_overload();
    else if (sc == "isolation") scenario_isolation();
    else if (sc == "loop_error") scenario_loop_error();
    else if (sc == "destroy_pending") scenario_destroy_pending();
    else {
        std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
        return 2;
    }
    std::printf("ok %s\n", sc.c_str());
    return 0;
}
