// Sample workspaces and the sampling scheduler behind ces_sample,
// ces_sample_batch, ces_autotune and the serving loop: Algorithm 1 step 4
// for every sample of a request and the level difference of Section 3.4,
// for many requests of different mesh sizes at once.
#include <algorithm>
#include <chrono>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "plan.hpp"

namespace ces {

StreamPool::~StreamPool() {
    for (auto s : streams_) (void)hipStreamDestroy(s);
    for (auto e : events_) (void)hipEventDestroy(e);
}

hipError_t StreamPool::stream(size_t i, hipStream_t* out) {
    while (streams_.size() <= i) {
        hipStream_t s = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        streams_.push_back(s);
    }
    *out = streams_[i];
    return hipSuccess;
}

hipError_t StreamPool::event(size_t i, hipEvent_t* out) {
    while (events_.size() <= i) {
        hipEvent_t v = nullptr;
        hipError_t e = hipEventCreateWithFlags(&v, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        events_.push_back(v);
    }
    *out = events_[i];
    return hipSuccess;
}

namespace {

class HipAllocator final : public DeviceAllocator {
public:
    hipError_t alloc(size_t bytes, void** p) override { return hipMalloc(p, bytes); }
    void release(void* p) override { (void)hipFree(p); }
};

struct PinnedSlots {
    std::mutex mu;
    std::vector<int*> free;
    std::vector<void*> slabs;
};
PinnedSlots& pinned() {
    static PinnedSlots* s = new PinnedSlots;   // lives until the process ends
    return *s;
}

}  // namespace

DeviceAllocator* default_allocator() {
    static HipAllocator a;
    return &a;
}

int* pinned_slot_acquire() {
    PinnedSlots& P = pinned();
    std::lock_guard<std::mutex> g(P.mu);
    if (P.free.empty()) {
        constexpr int kSlots = 256, kInts = 16;   // 64-byte slots
        void* slab = nullptr;
        if (hipHostMalloc(&slab, (size_t)kSlots * kInts * sizeof(int), hipHostMallocDefault) != hipSuccess)
            return nullptr;
        P.slabs.push_back(slab);
        for (int i = 0; i < kSlots; ++i) P.free.push_back(reinterpret_cast<int*>(slab) + i * kInts);
    }
    int* s = P.free.back();
    P.free.pop_back();
    return s;
}

void pinned_slot_release(int* slot) {
    if (!slot) return;
    PinnedSlots& P = pinned();
    std::lock_guard<std::mutex> g(P.mu);
    P.free.push_back(slot);
}

DevicePool::~DevicePool() {
    trim();
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : size_) (void)hipFree(kv.first);
    size_.clear();
}

hipError_t DevicePool::alloc(size_t bytes, void** p) {
    const size_t b = std::max<size_t>(256, (bytes + 255) / 256 * 256);
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = free_.lower_bound(b);
        if (it != free_.end() && it->first <= b + b / kReuseSlack) {
            *p = it->second;
            cached_ -= it->first;
            in_use_ += it->first;
            free_.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, b);
    if (e != hipSuccess) {
        // give the cached blocks back and try once more
        trim();
        e = hipMalloc(p, b);
        if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> g(mu_);
    size_[*p] = b;
    in_use_ += b;
    return hipSuccess;
}

void DevicePool::release(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    free_.emplace(it->second, p);
    in_use_ -= it->second;
    cached_ += it->second;
}

void DevicePool::trim() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : free_) {
        (void)hipFree(kv.second);
        size_.erase(kv.second);
    }
    free_.clear();
    cached_ = 0;
}

size_t DevicePool::in_use() const {
    std::lock_guard<std::mutex> g(mu_);
    return in_use_;
}

size_t DevicePool::cached() const {
    std::lock_guard<std::mutex> g(mu_);
    return cached_;
}

size_t lvl_stride(int m) { return ((size_t)(m + 1) * (m + 1) + 63) / 64 * 64; }

size_t slot_bytes(const ces_plan p) {
    const int m = p->d.m_fine;
    const size_t tb = p->is_double ? 8 : 4;
    auto solver_bytes = [&](int mm) {
        if (mm <= 32) return lvl_stride(mm) * 8 + 64 + 16;
        size_t b = lvl_stride(mm) * (6 * 8 + tb);
        for (int l = mm / 2; l >= 2; l /= 2) b += lvl_stride(l) * 5 * tb;
        return b + 64 * 8;
    };
    size_t b = solver_bytes(m) + lvl_stride(m) * tb;
    if (p->d.level_kind == CES_LEVEL_PAIR) b += solver_bytes(m / 2) + lvl_stride(m / 2) * tb;
    const size_t per_unit = (size_t)p->nf * (m + 1) * p->n * 2 * tb;
    b += p->d.field_mode == CES_FIELD_PAIR ? per_unit / 2 : per_unit;
    return b + 32;
}

namespace {

long long workspace_slots(const ces_plan p, long long max_slots) {
    const int m = p->d.m_fine;
    const bool pair_field = p->d.field_mode == CES_FIELD_PAIR;
    const size_t per_slot = slot_bytes(p);
    // 9 GiB (3% of the device; 257^2 single level: 2060 samples per chunk,
    // 4096-sample calls in 2 chunks instead of 4: +1.7% samples/s), but
    // room for at least 64 samples: on meshes of about 300 MB per sample the
    // per-chunk overheads (one host round trip per CG iteration) dominate
    // small chunks (2049^2 flow cell, 1024 samples per call: 13 per chunk
    // 781 samples/s, 55 per chunk 845, 138 per chunk 857)
    size_t target = std::max((size_t)9 << 30, 64 * per_slot);
    if (const char* env = std::getenv("CESMLMC_WORKSPACE_MB")) target = (size_t)std::atoll(env) << 20;
    const size_t used = p->ctx->used.load();
    if (p->ctx->budget && p->ctx->budget - std::min(p->ctx->budget, used) < target)
        target = p->ctx->budget - std::min(p->ctx->budget, used);
    long long slots = (long long)(target / per_slot);
    // samples per chunk: small meshes solve in one launch per chunk, so
    // allow more of them; larger meshes fill the device well before 8192
    slots = std::min<long long>(slots, m <= 32 ? 65536 : 8192);
    if (max_slots > 0) slots = std::min(slots, pair_field ? (max_slots + 1) / 2 * 2 : max_slots);
    if (pair_field) slots &= ~1LL;
    return slots;
}

}  // namespace

SolverCfg solver_cfg(const ces_plan p, bool coarse) {
    const int m = p->d.m_fine;
    SolverCfg cfg;
    cfg.m = coarse ? m / 2 : m;
    cfg.bc = p->d.bc;
    cfg.f = p->d.f_value;
    cfg.rtol = p->d.cg_rtol;
    cfg.maxit = p->d.cg_max_iter;
    cfg.qoi = p->d.qoi;
    cfg.qx = p->d.qoi_x;
    cfg.qy = p->d.qoi_y;
    // single levels (plain Monte Carlo, the coarsest MLMC level) run the
    // most samples per chunk: there the second visit of level 1 pays when
    // it saves enough iterations, which needs a field that the coarse
    // levels resolve: the length scale ell (lambda / sqrt(2 nu) for Matern,
    // lambda for the separable exponential) spanning at least 8 fine cells.
    // Measured at 257^2 (Matern nu = 1): lambda = 0.1 (ell = 18 cells)
    // 9.96 -> 8.01 iterations, +7% samples/s; lambda = 0.02 (3.6 cells)
    // 11.0 -> 10.0 iterations but -3%; Matern 3/2 at lambda = 0.01 more
    // iterations (11.4 -> 11.9) and -15%.
    const double ell = p->d.cov_kind == CES_COV_MATERN ? p->d.lambda / std::sqrt(2.0 * p->d.nu) : p->d.lambda;
    const bool w1 = p->d.mg_cycle == CES_CYCLE_W1;
    cfg.twice1 = w1 || (!coarse && p->d.mg_cycle == CES_CYCLE_AUTO && p->d.level_kind == CES_LEVEL_SINGLE &&
                        ell * m >= 8.0);
    return cfg;
}

size_t workspace_bytes(const ces_plan p, long long max_slots) {
    const long long slots = workspace_slots(p, max_slots);
    return slots > 0 ? (size_t)slots * slot_bytes(p) : 0;
}

int ensure_workspace(ces_plan p, long long max_slots, hipStream_t st) {
    if (p->sf) return CES_OK;
    const int m = p->d.m_fine;
    const bool pair_field = p->d.field_mode == CES_FIELD_PAIR;
    const long long slots = workspace_slots(p, max_slots);
    if (slots < (pair_field ? 2 : 1))
        return fail(CES_ERR_NOMEM, "device memory budget too small for one sample of this plan");
    p->chunk_slots = (int)slots;
    p->chunk_units = pair_field ? (int)slots / 2 : (int)slots;
    const size_t tb = p->is_double ? 8 : 4;
    DeviceAllocator* A = p->alloc;
    p->kf_ss = (long long)lvl_stride(m);
    p->kc_ss = (long long)lvl_stride(m / 2);
    CES_HIP(p->work.alloc((size_t)p->nf * p->chunk_units * (m + 1) * p->n * 2 * tb, A), "field workspace");
    CES_HIP(p->kf.alloc((size_t)slots * p->kf_ss * tb, A), "coefficient workspace");
    CES_HIP(hipMemsetAsync(p->kf.p, 0, p->kf.bytes, st), "coefficient workspace");
    if (p->d.level_kind == CES_LEVEL_PAIR) {
        CES_HIP(p->kc.alloc((size_t)slots * p->kc_ss * tb, A), "coefficient workspace");
        CES_HIP(hipMemsetAsync(p->kc.p, 0, p->kc.bytes, st), "coefficient workspace");
    }
    CES_HIP(p->qf.alloc((size_t)slots * 8, A), "qoi workspace");
    CES_HIP(p->qc.alloc((size_t)slots * 8, A), "qoi workspace");
    CES_HIP(p->itf.alloc((size_t)slots * 4, A), "qoi workspace");
    CES_HIP(p->itc.alloc((size_t)slots * 4, A), "qoi workspace");
    std::string err;
    p->sf = make_solver(solver_cfg(p, false), (int)slots, p->is_double, A, st, &err);
    if (!p->sf) return fail(CES_ERR_NOMEM, err);
    if (p->d.level_kind == CES_LEVEL_PAIR) {
        p->sc = make_solver(solver_cfg(p, true), (int)slots, p->is_double, A, st, &err);
        if (!p->sc) return fail(CES_ERR_NOMEM, err);
    }
    p->ws_bytes = p->work.bytes + p->kf.bytes + p->kc.bytes + p->sf->bytes() + (p->sc ? p->sc->bytes() : 0);
    p->ctx->used += p->ws_bytes;
    return CES_OK;
}

void drop_workspace(ces_plan p) {
    p->sf.reset();
    p->sc.reset();
    for (DevBuf* b : {&p->work, &p->kf, &p->kc, &p->qf, &p->qc, &p->itf, &p->itc, &p->zf, &p->zc}) b->reset();
    p->ctx->used -= std::min(p->ctx->used.load(), p->ws_bytes);
    p->ws_bytes = 0;
    p->chunk_slots = p->chunk_units = 0;
}

namespace {

template <typename T>
void set_lattice(FieldBatch<T>& b, const ces_plan p) {
    if (p->q_s <= 0) return;
    b.qrank = p->q_rank.as<int32_t>();
    b.qz = p->q_z.as<uint32_t>();
    b.qshifts = p->q_shifts;
}

}  // namespace

template <typename T>
FieldBatch<T> make_field_batch(ces_plan p, const WsBufs& w, uint64_t seed, uint64_t q0, int units) {
    FieldBatch<T> b;
    b.n = p->n;
    b.m = p->d.m_fine;
    b.mode = p->d.field_mode == CES_FIELD_PAIR ? MODE_PAIR : MODE_HARTLEY;
    b.nf = p->nf;
    // EMBED pairs draw the coarse field in a second batch (make_embedded_batch)
    b.coarse = p->d.level_kind == CES_LEVEL_PAIR && !p->cpl;
    b.af = p->af.as<T>();
    b.ac = p->nf == 2 ? p->ac.as<T>() : p->af.as<T>();
    b.tw = p->tw.as<cplx<T>>();
    b.fp = p->fp;
    b.seed = seed;
    b.q0 = q0;
    b.stream = p->d.stream;
    b.units = units;
    b.work = static_cast<cplx<T>*>(w.work);
    b.kf = static_cast<T*>(w.kf);
    b.kf_stride = w.kf_ss;
    b.kc = static_cast<T*>(w.kc);
    b.kc_stride = w.kc_ss;
    set_lattice(b, p);
    return b;
}

template <typename T>
FieldBatch<T> make_embedded_batch(ces_plan p, const WsBufs& w, uint64_t seed, uint64_t q0, int units) {
    const ces_plan c = p->cpl.get();
    FieldBatch<T> b;
    b.n = c->n;
    b.m = c->d.m_fine;
    b.mode = p->d.field_mode == CES_FIELD_PAIR ? MODE_PAIR : MODE_HARTLEY;
    b.nf = 1;
    b.coarse = false;
    b.af = c->af.as<T>();
    b.ac = b.af;
    b.tw = c->tw.as<cplx<T>>();
    b.fp = c->fp;
    b.seed = seed;
    b.q0 = q0;
    b.stream = p->d.stream;
    b.units = units;
    b.work = static_cast<cplx<T>*>(w.work);
    b.kf = static_cast<T*>(w.kc);
    b.kf_stride = w.kc_ss;
    b.n_src = p->n;
    set_lattice(b, p);   // counters are the fine embedding's
    return b;
}

template FieldBatch<float> make_field_batch<float>(ces_plan, const WsBufs&, uint64_t, uint64_t, int);
template FieldBatch<double> make_field_batch<double>(ces_plan, const WsBufs&, uint64_t, uint64_t, int);
template FieldBatch<float> make_embedded_batch<float>(ces_plan, const WsBufs&, uint64_t, uint64_t, int);
template FieldBatch<double> make_embedded_batch<double>(ces_plan, const WsBufs&, uint64_t, uint64_t, int);

namespace {


WsBufs plan_ws(const ces_plan p) { return WsBufs{p->work.p, p->kf.p, p->kc.p, p->kf_ss, p->kc_ss}; }

template <typename T>
FieldBatch<T> field_batch(ces_plan p, uint64_t seed, uint64_t q0, int units) {
    return make_field_batch<T>(p, plan_ws(p), seed, q0, units);
}

template <typename T>
FieldBatch<T> embedded_batch(ces_plan p, uint64_t seed, uint64_t q0, int units) {
    return make_embedded_batch<T>(p, plan_ws(p), seed, q0, units);
}

template <typename T>
int field_t(ces_plan p, uint64_t seed, uint64_t sample, double* zf, double* zc, hipStream_t st) {
    const bool pair_field = p->d.field_mode == CES_FIELD_PAIR;
    const int m = p->d.m_fine;
    const size_t nf = (size_t)(m + 1) * (m + 1), nc = (size_t)(m / 2 + 1) * (m / 2 + 1);
    if (!p->zf.p) {
        CES_HIP(p->zf.alloc(2 * nf * 8, p->alloc), "field hook buffers");
        CES_HIP(p->zc.alloc(2 * nc * 8, p->alloc), "field hook buffers");
    }
    FieldBatch<T> b = field_batch<T>(p, seed, pair_field ? sample / 2 : sample, 1);
    b.zf = p->zf.as<double>();
    b.zc = p->zc.as<double>();
    CES_HIP(launch_field<T>(b, st), "field kernels");
    if (p->cpl) {
        FieldBatch<T> c = embedded_batch<T>(p, seed, pair_field ? sample / 2 : sample, 1);
        c.zf = p->zc.as<double>();
        CES_HIP(launch_field<T>(c, st), "coarse field kernels");
    }
    const int comp = pair_field ? (int)(sample % 2) : 0;
    CES_HIP(hipMemcpyAsync(zf, p->zf.as<double>() + comp * nf, nf * 8, hipMemcpyDeviceToDevice, st), "copy field");
    if (zc && p->d.level_kind == CES_LEVEL_PAIR)
        CES_HIP(hipMemcpyAsync(zc, p->zc.as<double>() + comp * nc, nc * 8, hipMemcpyDeviceToDevice, st), "copy field");
    return CES_OK;
}

template <typename T>
int solve_t(ces_plan p, int grid, int64_t count, const double* k, double* u, int32_t* iters, hipStream_t st) {
    Solver* S = grid == 0 ? p->sf.get() : p->sc.get();
    DevBuf& kb = grid == 0 ? p->kf : p->kc;
    const long long kss = grid == 0 ? p->kf_ss : p->kc_ss;
    const int m = grid == 0 ? p->d.m_fine : p->d.m_fine / 2;
    const size_t nn = (size_t)(m + 1) * (m + 1);
    for (int64_t c0 = 0; c0 < count; c0 += S->capacity()) {
        const int ns = (int)std::min<int64_t>(S->capacity(), count - c0);
        for (int i = 0; i < ns; ++i) {
            const double* src = k + (size_t)(c0 + i) * nn;
            T* dst = kb.as<T>() + (size_t)i * kss;
            if (sizeof(T) == 8)
                CES_HIP(hipMemcpyAsync(dst, src, nn * 8, hipMemcpyDeviceToDevice, st), "copy k");
            else
                CES_HIP(launch_convert_d2f(src, reinterpret_cast<float*>(dst), (long long)nn, st), "convert k");
        }
        CES_HIP(S->solve(kb.p, kss, ns, st), "solve");
        CES_HIP(S->qoi(kb.p, kss, ns, nullptr, iters ? iters + c0 : nullptr, st), "solve status");
        CES_HIP(hipMemcpy2DAsync(u + (size_t)c0 * nn, nn * 8, S->x(), (size_t)S->xstride() * 8, nn * 8, ns,
                                 hipMemcpyDeviceToDevice, st),
                "copy solution");
    }
    return CES_OK;
}

// marks a plan's workspace as taken for the lifetime of the guard
struct BusyGuard {
    ces_plan p = nullptr;
    explicit BusyGuard(ces_plan q) {
        int z = 0;
        if (q->busy.compare_exchange_strong(z, 1)) p = q;
    }
    ~BusyGuard() {
        if (p) p->busy.store(0);
    }
    bool ok() const { return p != nullptr; }
};

}  // namespace

// Records the plan's workspace-free event on the stream that ran the last
// work using the workspace (a lane's coarse stream joins its main stream
// before every finalize, so for a lane that is its main stream).
static hipError_t mark_workspace_free(ces_plan p, hipStream_t st) {
    if (!p->ws_free) {
        hipError_t e = hipEventCreateWithFlags(&p->ws_free, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(p->ws_free, st);
}

int field_impl(ces_plan p, uint64_t seed, uint64_t sample, double* zf, double* zc, hipStream_t st) {
    int rc = ensure_workspace(p, 0, st);
    if (rc != CES_OK) return rc;
    BusyGuard g(p);
    if (!g.ok()) return fail(CES_ERR_BUSY, "plan is in use by another call");
    if (p->ws_free) CES_HIP(hipStreamWaitEvent(st, p->ws_free, 0), "workspace");
    rc = p->is_double ? field_t<double>(p, seed, sample, zf, zc, st) : field_t<float>(p, seed, sample, zf, zc, st);
    if (rc == CES_OK) CES_HIP(mark_workspace_free(p, st), "workspace");
    return rc;
}

int solve_impl(ces_plan p, int grid, int64_t count, const double* k, double* u, int32_t* iters, hipStream_t st) {
    int rc = ensure_workspace(p, 0, st);
    if (rc != CES_OK) return rc;
    BusyGuard g(p);
    if (!g.ok()) return fail(CES_ERR_BUSY, "plan is in use by another call");
    if (p->ws_free) CES_HIP(hipStreamWaitEvent(st, p->ws_free, 0), "workspace");
    rc = p->is_double ? solve_t<double>(p, grid, count, k, u, iters, st)
                      : solve_t<float>(p, grid, count, k, u, iters, st);
    if (rc == CES_OK) CES_HIP(mark_workspace_free(p, st), "workspace");
    return rc;
}

// ------------------------------------------------------------ scheduler
Scheduler::Scheduler(StreamPool& pool, hipStream_t caller, const ces_schedule& s)
    : pool_(pool), caller_(caller), s_(s) {
    if (s_.depth <= 0) s_.depth = 2;
    s_.depth = std::min(s_.depth, 4);
}

Scheduler::~Scheduler() {
    (void)join();
}

int Scheduler::lane_of(ces_plan p, Lane** out) {
    for (auto& L : lanes_)
        if (L->p == p) {
            *out = L.get();
            return CES_OK;
        }
    int z = 0;
    if (!p->busy.compare_exchange_strong(z, 1)) return fail(CES_ERR_BUSY, "plan is in use by another call");
    lanes_.emplace_back(new Lane);
    lanes_.back()->p = p;
    *out = lanes_.back().get();
    return CES_OK;
}

hipError_t Scheduler::get_stream(hipStream_t* out) {
    if (!free_streams_.empty()) {
        *out = free_streams_.back();
        free_streams_.pop_back();
        return hipSuccess;
    }
    return pool_.stream(next_stream_++, out);
}

hipError_t Scheduler::get_event(hipEvent_t* out) {
    if (!free_events_.empty()) {
        *out = free_events_.back();
        free_events_.pop_back();
        return hipSuccess;
    }
    return pool_.event(next_event_++, out);
}

int Scheduler::add(const ces_request& r, hipEvent_t done_event, long long max_slots, double* y_host,
                   int32_t* status_host, std::atomic<int>* recorded) {
    ces_plan p = r.plan;
    if (!p) return fail(CES_ERR_ARG, "request plan is NULL");
    if (r.count < 0) return fail(CES_ERR_ARG, "count < 0");
    if (r.count > 0 && !r.y) return fail(CES_ERR_ARG, "y is NULL");
    if (r.first_sample + (uint64_t)r.count < r.first_sample) return fail(CES_ERR_ARG, "sample range overflows");
    if (p->q_s > 0 && r.first_sample + (uint64_t)r.count > (1ull << 63))
        return fail(CES_ERR_ARG, "sample indices of a lattice plan must stay below 2^63");
    if (joined_) return fail(CES_ERR_ARG, "scheduler already joined");
    if (r.count == 0) {
        if (done_event) CES_HIP(hipEventRecord(done_event, caller_), "request event");
        if (recorded) recorded->store(1);
        return CES_OK;
    }
    Lane* L = nullptr;
    int rc = lane_of(p, &L);
    if (rc != CES_OK) return rc;
    if ((rc = ensure_workspace(p, max_slots, caller_)) != CES_OK) return rc;
    const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
    long long cu = p->chunk_units;
    if (s_.chunk_samples > 0) cu = std::max<long long>(1, std::min<long long>(cu, s_.chunk_samples / per_unit));
    const uint64_t first = r.first_sample, last = first + (uint64_t)r.count - 1;
    const uint64_t u_begin = first / per_unit, u_end = last / per_unit + 1;
    // as few chunks as the workspace allows, of equal size (no short tail chunk)
    const uint64_t nch = (u_end - u_begin + (uint64_t)cu - 1) / (uint64_t)cu;
    cu = (long long)((u_end - u_begin + nch - 1) / nch);
    for (uint64_t u0 = u_begin; u0 < u_end; u0 += (uint64_t)cu) {
        Job j;
        j.seed = r.seed;
        j.u0 = u0;
        j.units = (int)std::min<uint64_t>((uint64_t)cu, u_end - u0);
        j.first = first;
        const uint64_t s0 = u0 * per_unit;
        j.lo = std::max(first, s0);
        j.hi = std::min(last + 1, s0 + (uint64_t)j.units * per_unit);
        j.y = r.y;
        j.yf = r.q_fine;
        j.yc = r.q_coarse;
        j.iters = r.iters;
        j.status = r.status;
        const bool last = u0 + (uint64_t)cu >= u_end;
        j.done_event = last ? done_event : nullptr;
        j.count = r.count;
        j.y_host = last ? y_host : nullptr;
        j.status_host = last ? status_host : nullptr;
        j.recorded = last ? recorded : nullptr;
        L->jobs.push_back(j);
    }
    return CES_OK;
}

template <typename T>
int Scheduler::start_t(Lane& L, const Job& j) {
    ces_plan p = L.p;
    const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
    const int nslots = j.units * per_unit;
    FieldBatch<T> b = field_batch<T>(p, j.seed, j.u0, j.units);
    CES_HIP(launch_field<T>(b, L.sa), "field kernels");
    if (p->cpl) CES_HIP(launch_field<T>(embedded_batch<T>(p, j.seed, j.u0, j.units), L.sa), "coarse field kernels");
    CES_HIP(p->sf->begin(p->kf.p, p->kf_ss, nslots, L.sa, false), "fine solve");
    if (p->sc) {
        CES_HIP(hipEventRecord(L.ev_f, L.sa), "lane event");
        CES_HIP(hipStreamWaitEvent(L.sb, L.ev_f, 0), "lane event");
        CES_HIP(p->sc->begin(p->kc.p, p->kc_ss, nslots, L.sb, false), "coarse solve");
    }
    L.solving = true;
    L.fdone = L.cdone = false;
    return CES_OK;
}

int Scheduler::start(Lane& L) {
    if (!L.forked) {
        // the lane's streams start after everything the caller's stream
        // holds now (workspace zeroing included)
        CES_HIP(get_stream(&L.sa), "lane stream");
        CES_HIP(get_stream(&L.sb), "lane stream");
        CES_HIP(get_event(&L.ev_f), "lane event");
        CES_HIP(get_event(&L.ev_c), "lane event");
        CES_HIP(get_event(&L.ev_fork), "lane event");
        CES_HIP(hipEventRecord(L.ev_fork, caller_), "fork");
        CES_HIP(hipStreamWaitEvent(L.sa, L.ev_fork, 0), "fork");
        CES_HIP(hipStreamWaitEvent(L.sb, L.ev_fork, 0), "fork");
        if (L.p->ws_free) {
            CES_HIP(hipStreamWaitEvent(L.sa, L.p->ws_free, 0), "workspace");
            CES_HIP(hipStreamWaitEvent(L.sb, L.p->ws_free, 0), "workspace");
        }
        L.forked = true;
    }
    const Job& j = L.jobs[L.next];
    return L.p->is_double ? start_t<double>(L, j) : start_t<float>(L, j);
}

int Scheduler::finish(Lane& L) {
    ces_plan p = L.p;
    const Job& j = L.jobs[L.next];
    const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
    const int nslots = j.units * per_unit;
    CES_HIP(p->sf->finish(L.sa), "fine solve");
    CES_HIP(p->sf->qoi(p->kf.p, p->kf_ss, nslots, p->qf.as<double>(), p->itf.as<int>(), L.sa), "fine qoi");
    if (p->sc) {
        CES_HIP(p->sc->finish(L.sb), "coarse solve");
        CES_HIP(p->sc->qoi(p->kc.p, p->kc_ss, nslots, p->qc.as<double>(), p->itc.as<int>(), L.sb), "coarse qoi");
        CES_HIP(hipEventRecord(L.ev_c, L.sb), "lane event");
        CES_HIP(hipStreamWaitEvent(L.sa, L.ev_c, 0), "lane event");
    }
    const uint64_t s0 = j.u0 * per_unit;
    CES_HIP(launch_finalize(p->qf.as<double>(), p->sc ? p->qc.as<double>() : nullptr, p->itf.as<int>(),
                            p->sc ? p->itc.as<int>() : nullptr, (int)(j.lo - s0), (int)(j.hi - j.lo),
                            (long long)(j.lo - j.first), j.y, j.yf, j.yc, j.iters, j.status, L.sa),
            "finalize");
    if (j.y_host)
        CES_HIP(hipMemcpyAsync(j.y_host, j.y, (size_t)j.count * 8, hipMemcpyDeviceToHost, L.sa), "copy results");
    if (j.status_host && j.status)
        CES_HIP(hipMemcpyAsync(j.status_host, j.status, (size_t)j.count * 4, hipMemcpyDeviceToHost, L.sa),
                "copy results");
    if (j.done_event) CES_HIP(hipEventRecord(j.done_event, L.sa), "request event");
    if (j.recorded) j.recorded->store(1);
    ++L.next;
    L.solving = false;
    return CES_OK;
}

int Scheduler::step(bool* progressed) {
    *progressed = false;
    int busy = 0;
    for (auto& L : lanes_) busy += L->solving ? 1 : 0;
    for (auto& Lp : lanes_) {
        Lane& L = *Lp;
        if (!L.solving) {
            if (L.next < L.jobs.size() && (s_.max_lanes <= 0 || busy < s_.max_lanes)) {
                int rc = start(L);
                if (rc != CES_OK) return rc;
                ++busy;
                *progressed = true;
            }
            continue;
        }
        bool pf = false, pc = false;
        const bool g = s_.graphs != 0;
        if (!L.fdone) CES_HIP(L.p->sf->advance(L.sa, s_.depth, g, &L.fdone, &pf), "fine solve");
        if (L.p->sc && !L.cdone) CES_HIP(L.p->sc->advance(L.sb, s_.depth, g, &L.cdone, &pc), "coarse solve");
        if (pf || pc) *progressed = true;
        if (L.fdone && (L.cdone || !L.p->sc)) {
            int rc = finish(L);
            if (rc != CES_OK) return rc;
            --busy;
            *progressed = true;
        }
    }
    return CES_OK;
}

bool Scheduler::idle() const {
    for (auto& L : lanes_)
        if (L->solving || L->next < L->jobs.size()) return false;
    return true;
}

int Scheduler::run() {
    while (!idle()) {
        bool prog = false;
        int rc = step(&prog);
        if (rc != CES_OK) return rc;
        if (prog) continue;
        // nothing could be enqueued: every solve has `depth` iterations in
        // flight.  Block when one solve is pending, else poll again.
        Solver* only = nullptr;
        int pending = 0;
        for (auto& L : lanes_) {
            if (!L->solving) continue;
            if (!L->fdone) { only = L->p->sf.get(); ++pending; }
            if (L->p->sc && !L->cdone) { only = L->p->sc.get(); ++pending; }
        }
        if (pending == 1) CES_HIP(only->wait(), "solve wait");
        else std::this_thread::yield();
    }
    return CES_OK;
}

int Scheduler::join() {
    if (joined_) return CES_OK;
    joined_ = true;
    int rc = CES_OK;
    for (auto& L : lanes_) {
        if (L->forked) {
            for (hipStream_t s : {L->sa, L->sb}) {
                hipEvent_t e = nullptr;
                hipError_t err = get_event(&e);
                if (err == hipSuccess) err = hipEventRecord(e, s);
                if (err == hipSuccess) err = hipStreamWaitEvent(caller_, e, 0);
                if (err != hipSuccess && rc == CES_OK) rc = hip_fail(err, "join");
            }
            hipError_t err = mark_workspace_free(L->p, L->sa);
            if (err != hipSuccess && rc == CES_OK) rc = hip_fail(err, "join");
        }
        L->p->busy.store(0);
    }
    return rc;
}

int Scheduler::retire(std::vector<ces_plan>* released) {
    std::vector<std::unique_ptr<Lane>> keep;
    int rc = CES_OK;
    for (auto& L : lanes_) {
        if (L->solving || L->next < L->jobs.size()) {
            keep.push_back(std::move(L));
            continue;
        }
        if (L->forked) {
            hipError_t err = mark_workspace_free(L->p, L->sa);
            if (err != hipSuccess && rc == CES_OK) rc = hip_fail(err, "retire");
            // later work on these streams only depends on what is enqueued
            // after it, so they can serve another lane at once
            free_streams_.push_back(L->sa);
            free_streams_.push_back(L->sb);
            free_events_.push_back(L->ev_f);
            free_events_.push_back(L->ev_c);
            free_events_.push_back(L->ev_fork);
        }
        L->p->busy.store(0);
        released->push_back(L->p);
    }
    lanes_.swap(keep);
    return rc;
}

int Scheduler::pending_solves() const {
    int n = 0;
    for (auto& L : lanes_) {
        if (!L->solving) continue;
        n += L->fdone ? 0 : 1;
        n += (L->p->sc && !L->cdone) ? 1 : 0;
    }
    return n;
}

}  // namespace ces

using namespace ces;

namespace {

int run_batch(ces_context ctx, const ces_request* reqs, int32_t nreq, hipStream_t st, const ces_schedule& s) {
    Scheduler S(ctx->pool, st, s);
    for (int32_t i = 0; i < nreq; ++i) {
        if (reqs[i].plan && reqs[i].plan->ctx != ctx) return fail(CES_ERR_ARG, "request plan belongs to another context");
        int rc = S.add(reqs[i], nullptr);
        if (rc != CES_OK) return rc;
    }
    int rc = S.run();
    int rj = S.join();
    return rc != CES_OK ? rc : rj;
}

// ---- persisted autotuner choices (file named by CESMLMC_AUTOTUNE_CACHE) --
// One line per tuned batch: "<key> depth max_lanes chunk_samples graphs
// best_ms".  The key is an FNV-1a hash of the device's architecture name
// and, per distinct plan in request order, its descriptor bytes and the
// batch's sample count on it.
uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    return h;
}

uint64_t batch_key(ces_context ctx, const ces_request* reqs, int32_t nreq) {
    uint64_t h = 1469598103934665603ull;
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess)
        h = fnv1a(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
    for (int32_t i = 0; i < nreq; ++i) {
        bool seen = false;
        for (int32_t j = 0; j < i; ++j) seen = seen || reqs[j].plan == reqs[i].plan;
        if (seen || !reqs[i].plan) continue;
        int64_t total = 0;
        for (int32_t j = i; j < nreq; ++j)
            if (reqs[j].plan == reqs[i].plan) total += reqs[j].count;
        h = fnv1a(h, &reqs[i].plan->d, sizeof(ces_level_desc));
        h = fnv1a(h, &total, sizeof(total));
    }
    return h;
}

bool cache_lookup(const char* path, uint64_t key, ces_schedule* s, double* ms) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        uint64_t k = 0;
        int depth = 0, lanes = 0, graphs = 0;
        long long chunk = 0;
        double t = 0.0;
        if (std::sscanf(line, "%" SCNx64 " %d %d %lld %d %lf", &k, &depth, &lanes, &chunk, &graphs, &t) == 6 &&
            k == key && depth >= 1 && depth <= 4 && lanes >= 0 && chunk >= 0 && (graphs == 0 || graphs == 1)) {
            *s = ces_schedule{};
            s->depth = depth;
            s->max_lanes = lanes;
            s->chunk_samples = chunk;
            s->graphs = graphs;
            *ms = t;
            found = true;   // the last entry for a key wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, uint64_t key, const ces_schedule& s, double ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%016" PRIx64 " %d %d %lld %d %.4f\n", key, s.depth, s.max_lanes, (long long)s.chunk_samples,
                 s.graphs, ms);
    std::fclose(f);
}

}  // namespace

extern "C" {

int ces_sample(ces_plan p, uint64_t seed, uint64_t first, int64_t count, double* y, double* yf, double* yc,
               int32_t* iters, int32_t* status, void* stream) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    if (count < 0) return fail(CES_ERR_ARG, "count < 0");
    if (count == 0) return CES_OK;
    if (!y) return fail(CES_ERR_ARG, "y is NULL");
    if (first + (uint64_t)count < first) return fail(CES_ERR_ARG, "sample range overflows");
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    ces_request r{p, seed, first, count, y, yf, yc, iters, status};
    return run_batch(p->ctx, &r, 1, reinterpret_cast<hipStream_t>(stream), p->ctx->sched);
}

int ces_sample_batch(ces_context ctx, const ces_request* reqs, int32_t nreq, void* stream) {
    if (!ctx) return fail(CES_ERR_ARG, "context is NULL");
    if (nreq < 0 || (nreq > 0 && !reqs)) return fail(CES_ERR_ARG, "requests");
    if (nreq == 0) return CES_OK;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return run_batch(ctx, reqs, nreq, reinterpret_cast<hipStream_t>(stream), ctx->sched);
}

int ces_schedule_get(ces_context ctx, ces_schedule* out) {
    if (!ctx || !out) return fail(CES_ERR_ARG, "context or out is NULL");
    *out = ctx->sched;
    if (out->depth <= 0) out->depth = 2;
    return CES_OK;
}

int ces_schedule_set(ces_context ctx, const ces_schedule* s) {
    if (!ctx || !s) return fail(CES_ERR_ARG, "context or schedule is NULL");
    if (s->depth < 0 || s->depth > 4) return fail(CES_ERR_ARG, "depth must be in 0..4");
    if (s->graphs != 0 && s->graphs != 1) return fail(CES_ERR_ARG, "graphs must be 0 or 1");
    if (s->max_lanes < 0 || s->chunk_samples < 0) return fail(CES_ERR_ARG, "max_lanes / chunk_samples < 0");
    ctx->sched = *s;
    if (ctx->sched.depth == 0) ctx->sched.depth = 2;
    return CES_OK;
}

int ces_autotune(ces_context ctx, const ces_request* reqs, int32_t nreq, void* stream, ces_schedule* chosen,
                 double* best_ms) {
    if (!ctx) return fail(CES_ERR_ARG, "context is NULL");
    if (nreq <= 0 || !reqs) return fail(CES_ERR_ARG, "requests");
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // a choice persisted for this batch: apply it and run the batch once
    const char* cache = std::getenv("CESMLMC_AUTOTUNE_CACHE");
    const uint64_t key = cache && *cache ? batch_key(ctx, reqs, nreq) : 0;
    if (cache && *cache) {
        ces_schedule c{};
        double ms = 0.0;
        if (cache_lookup(cache, key, &c, &ms)) {
            int rc = run_batch(ctx, reqs, nreq, st, c);
            if (rc != CES_OK) return rc;
            ctx->sched = c;
            if (chosen) *chosen = c;
            if (best_ms) *best_ms = ms;
            return CES_OK;
        }
    }
    auto timed = [&](const ces_schedule& s, double* ms) -> int {
        double best = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            CES_HIP(hipStreamSynchronize(st), "autotune sync");
            const auto t0 = std::chrono::steady_clock::now();
            int rc = run_batch(ctx, reqs, nreq, st, s);
            if (rc != CES_OK) return rc;
            CES_HIP(hipStreamSynchronize(st), "autotune sync");
            best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        *ms = best;
        return CES_OK;
    };
    int nplans = 0;
    for (int32_t i = 0; i < nreq; ++i) {
        bool seen = false;
        for (int32_t j = 0; j < i; ++j) seen = seen || reqs[j].plan == reqs[i].plan;
        nplans += seen ? 0 : 1;
    }
    ces_schedule best = ctx->sched;
    if (best.depth <= 0) best.depth = 2;
    int rc = run_batch(ctx, reqs, nreq, st, best);   // warm-up, allocates workspaces
    if (rc != CES_OK) return rc;
    double tbest = 0.0;
    if ((rc = timed(best, &tbest)) != CES_OK) return rc;
    auto consider = [&](ces_schedule c) -> int {
        double t = 0.0;
        int r = timed(c, &t);
        if (r != CES_OK) return r;
        if (t < 0.97 * tbest) {
            best = c;
            tbest = t;
        }
        return CES_OK;
    };
    // coordinate search: in-flight depth, concurrent lanes, chunk size
    for (int d = 1; d <= 4; ++d)
        if (d != best.depth) {
            ces_schedule c = best;
            c.depth = d;
            if ((rc = consider(c)) != CES_OK) return rc;
        }
    for (int lanes : {0, 1, 2, 4})
        if (lanes != best.max_lanes && lanes < nplans) {
            ces_schedule c = best;
            c.max_lanes = lanes;
            if ((rc = consider(c)) != CES_OK) return rc;
        }
    for (long long ch : {0LL, 2048LL, 512LL})
        if (ch != best.chunk_samples) {
            ces_schedule c = best;
            c.chunk_samples = ch;
            if ((rc = consider(c)) != CES_OK) return rc;
        }
    {
        ces_schedule c = best;
        c.graphs = best.graphs ? 0 : 1;
        if ((rc = consider(c)) != CES_OK) return rc;
    }
    ctx->sched = best;
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = tbest;
    if (cache && *cache) cache_store(cache, key, best, tbest);
    return CES_OK;
}

}  // extern "C"
