// Host stand-ins for the library's device layer (test infrastructure):
// plan set-up, the field kernels, the solver and the finalize kernel are
// replaced by host code with known results, so that the scheduler and the
// serving loop (compiled unchanged) can be checked on a machine without a
// GPU.
//
// Field: sample i of a plan with seed s, level tag t and mesh m writes
//   fine   k = 3 (i mod P) + (s mod 7) + 11 t + m
//   coarse k =   (i mod P) + m / 2
// (P = 100000, or 16 for seeds of at least 10^6: bounded sample variances)
// into the first value of its coefficient slot; the solver returns that
// value as the QoI.  So Y = 2 (i mod P) + (s mod 7) + 11 t + m/2 for a
// pair level and 3 (i mod P) + (s mod 7) + 11 t + m for a single one,
// all exact in float.
//
// A solve of mesh m takes 2 + m/8 iterations (one per advance call), each
// delayed by fake_device_set_iteration_delay_us.  fake_device_fail_after(n)
// makes the n-th advance call from now fail with a device error.  A
// descriptor with psd_policy FAIL and lambda > 1 fails plan creation with
// CES_ERR_NOT_PSD.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>

#include "plan.hpp"

namespace {

std::atomic<long long> g_fail_after{-1};
std::atomic<int> g_delay_us{0};
std::atomic<int> g_active{0}, g_active_max{0};
std::atomic<long long> g_solves{0};

}  // namespace

extern "C" {
void fake_device_fail_after(long long n) { g_fail_after.store(n); }
void fake_device_set_iteration_delay_us(int us) { g_delay_us.store(us); }
int fake_device_max_concurrent_solves() { return g_active_max.load(); }
void fake_device_reset_counters() {
    g_active_max.store(g_active.load());
    g_solves.store(0);
}
long long fake_device_solves() { return g_solves.load(); }

int ces_plan_destroy(ces_plan p) {
    if (!p) return CES_OK;
    p->ctx->used -= std::min(p->ctx->used.load(), p->ws_bytes);
    delete p;
    return CES_OK;
}
}

namespace ces {

int plan_create(ces_context ctx, const ces_level_desc* desc, DeviceAllocator* A, hipStream_t, ces_plan* out,
                bool) {
    int rc = validate_desc(desc);
    if (rc != CES_OK) return rc;
    if (desc->psd_policy == CES_PSD_FAIL && desc->lambda > 1.0)
        return fail(CES_ERR_NOT_PSD, "no nonnegative embedding (fake)");
    auto* p = new ces_plan_s;
    p->ctx = ctx;
    p->d = *desc;
    p->alloc = A;
    p->n = 2 * desc->m_fine;
    p->is_double = desc->precision == CES_PREC_FP64;
    p->nf = 1;
    const size_t tb = p->is_double ? 8 : 4;
    // the amplitudes, as the real plan holds them
    if (A->alloc((size_t)p->n * p->n * tb, &p->af.p) != hipSuccess) {
        delete p;
        return fail(CES_ERR_NOMEM, "amplitudes (fake)");
    }
    p->af.a = A;
    p->af.bytes = (size_t)p->n * p->n * tb;
    *out = p;
    return CES_OK;
}

template <typename T>
hipError_t launch_field(const FieldBatch<T>& b, hipStream_t) {
    const bool pair = b.mode == MODE_PAIR;
    for (int u = 0; u < b.units; ++u)
        for (int c = 0; c < (pair ? 2 : 1); ++c) {
            const uint64_t i = pair ? 2 * (b.q0 + u) + c : b.q0 + u;
            const int slot = pair ? 2 * u + c : u;
            const double im = (double)(i % (b.seed >= 1000000 ? 16 : 100000));
            if (b.n_src > 0) {
                // coarse field of an EMBED pair, written as that plan's
                // fine field (b.m is the coarse mesh here)
                b.kf[(size_t)slot * b.kf_stride] = (T)(im + b.m);
                continue;
            }
            b.kf[(size_t)slot * b.kf_stride] = (T)(3.0 * im + (double)(b.seed % 7) + 11.0 * b.stream + b.m);
            if (b.coarse) b.kc[(size_t)slot * b.kc_stride] = (T)(im + b.m / 2);
        }
    return hipSuccess;
}
template hipError_t launch_field<float>(const FieldBatch<float>&, hipStream_t);
template hipError_t launch_field<double>(const FieldBatch<double>&, hipStream_t);

hipError_t launch_convert_d2f(const double* in, float* out, long long count, hipStream_t) {
    for (long long i = 0; i < count; ++i) out[i] = (float)in[i];
    return hipSuccess;
}

hipError_t launch_finalize(const double* qf, const double* qc, const int* itf, const int* itc, int slot0,
                           int nslots, long long out0, double* y, double* yf, double* yc, int* iters, int* status,
                           hipStream_t) {
    for (int t = 0; t < nslots; ++t) {
        const int s = slot0 + t;
        y[out0 + t] = qf[s] - (qc ? qc[s] : 0.0);
        if (yf) yf[out0 + t] = qf[s];
        if (yc) yc[out0 + t] = qc ? qc[s] : 0.0;
        if (iters) iters[out0 + t] = itf[s];
        if (status) status[out0 + t] = (itf[s] < 0 || (itc && itc[s] < 0)) ? CES_ERR_NOCONV : 0;
    }
    return hipSuccess;
}

namespace {

class FakeSolver final : public Solver {
public:
    FakeSolver(const SolverCfg& c, int cap, bool dbl, DeviceAllocator* A) : cfg_(c), cap_(cap), dbl_(dbl), A_(A) {}
    ~FakeSolver() override {
        if (solving_) --g_active;
        if (buf_) A_->release(buf_);
    }
    // as much memory as the library's solver of this mesh takes, so that
    // the serving loop's admission sees the real sizes
    hipError_t init() {
        const int m = cfg_.m;
        const size_t tb = dbl_ ? 8 : 4;
        size_t per = lvl_stride(m) * 8 + 64 + 16;
        if (m > 32) {
            per = lvl_stride(m) * (6 * 8 + tb) + 64 * 8;
            for (int l = m / 2; l >= 2; l /= 2) per += lvl_stride(l) * 5 * tb;
        }
        bytes_ = (size_t)cap_ * per;
        return A_->alloc(bytes_, &buf_);
    }
    int capacity() const override { return cap_; }
    size_t bytes() const override { return bytes_; }
    int mg_levels() const override { return 1; }
    hipError_t begin(const void* k, long long kstride, int S, hipStream_t, bool) override {
        if (S < 0 || S > cap_) return hipErrorInvalidValue;
        if (solving_) return hipErrorInvalidValue;   // a solve was begun twice
        solving_ = true;
        const int now = ++g_active;
        int seen = g_active_max.load();
        while (now > seen && !g_active_max.compare_exchange_weak(seen, now)) {
        }
        ++g_solves;
        k_ = k;
        kstride_ = kstride;
        S_ = S;
        it_ = 0;
        return hipSuccess;
    }
    hipError_t advance(hipStream_t, int depth, bool, bool* done, bool* progressed) override {
        if (depth < 1 || depth > 4) return hipErrorInvalidValue;
        if (!solving_) return hipErrorInvalidValue;
        const long long f = g_fail_after.load();
        if (f >= 0) {
            if (f == 0) {
                g_fail_after.store(-1);
                return hipErrorLaunchFailure;
            }
            g_fail_after.store(f - 1);
        }
        if (const int us = g_delay_us.load()) std::this_thread::sleep_for(std::chrono::microseconds(us));
        ++it_;
        *progressed = true;
        *done = it_ >= 2 + cfg_.m / 8;
        return hipSuccess;
    }
    hipError_t wait() override { return hipSuccess; }
    hipError_t finish(hipStream_t) override {
        if (!solving_) return hipErrorInvalidValue;
        solving_ = false;
        --g_active;
        return hipSuccess;
    }
    hipError_t qoi(const void* k, long long kstride, int S, double* q, int* iters, hipStream_t) override {
        if (k != k_ || kstride != kstride_ || S != S_) return hipErrorInvalidValue;
        for (int s = 0; s < S; ++s) {
            const double v = dbl_ ? static_cast<const double*>(k)[(size_t)s * kstride]
                                  : (double)static_cast<const float*>(k)[(size_t)s * kstride];
            if (q) q[s] = v;
            if (iters) iters[s] = it_;
        }
        return hipSuccess;
    }
    const double* x() const override { return nullptr; }
    long long xstride() const override { return 0; }

private:
    SolverCfg cfg_;
    int cap_;
    bool dbl_;
    DeviceAllocator* A_;
    void* buf_ = nullptr;
    size_t bytes_ = 0;
    const void* k_ = nullptr;
    long long kstride_ = 0;
    int S_ = 0, it_ = 0;
    bool solving_ = false;
};

}  // namespace

std::unique_ptr<Solver> make_solver(const SolverCfg& cfg, int capacity, bool is_double, DeviceAllocator* alloc,
                                    hipStream_t, std::string* err, bool) {
    auto s = std::make_unique<FakeSolver>(cfg, capacity, is_double, alloc);
    if (s->init() != hipSuccess) {
        *err = "solver workspace (fake)";
        return nullptr;
    }
    return s;
}

}  // namespace ces
