// Library-private state behind the C ABI handles and the interfaces
// between api.cpp (plan set-up, parity hooks), exec.cpp (workspaces and
// the sampling scheduler) and server.cpp (the serving loop).
#pragma once

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cesmlmc.h"
#include "internal.hpp"

namespace ces {

// Sets the calling thread's ces_last_error() message; returns code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define CES_HIP(call, what)                                \
    do {                                                   \
        hipError_t e__ = (call);                           \
        if (e__ != hipSuccess) return ces::hip_fail(e__, what); \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DeviceAllocator* a = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) a->release(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b, DeviceAllocator* from = nullptr) {
        reset();
        a = from ? from : default_allocator();
        bytes = b;
        return b ? a->alloc(b, &p) : hipSuccess;
    }
    template <typename U>
    U* as() const { return reinterpret_cast<U*>(p); }
};

// Caching device allocator: released blocks are kept (keyed by size) and
// handed out again for requests they fit within 25% (kReuseSlack); nothing
// is returned to HIP until trim() or destruction.  Thread-safe.
class DevicePool final : public DeviceAllocator {
public:
    // a cached block of b' bytes serves a request of b (rounded up to 256)
    // when b' <= b (1 + 1/kReuseSlack)
    static constexpr size_t kReuseSlack = 4;
    // bytes the pool may count against its user for a request of `bytes`
    static size_t charged(size_t bytes) {
        const size_t b = (bytes + 255) / 256 * 256;
        return b + b / kReuseSlack;
    }
    DevicePool() = default;
    DevicePool(const DevicePool&) = delete;
    DevicePool& operator=(const DevicePool&) = delete;
    ~DevicePool() override;
    hipError_t alloc(size_t bytes, void** p) override;
    void release(void* p) override;
    void trim();                 // frees every cached block (synchronises)
    size_t in_use() const;       // bytes handed out
    size_t cached() const;       // bytes kept for reuse

private:
    mutable std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::map<void*, size_t> size_;
    size_t in_use_ = 0, cached_ = 0;
};

// Streams (default priority, non-blocking) and events, created on first
// use and kept until the owner goes away.  One pool per host thread that
// schedules work (a context's caller, a server's loop).
class StreamPool {
public:
    StreamPool() = default;
    StreamPool(const StreamPool&) = delete;
    StreamPool& operator=(const StreamPool&) = delete;
    ~StreamPool();
    hipError_t stream(size_t i, hipStream_t* out);
    hipError_t event(size_t i, hipEvent_t* out);

private:
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> events_;
};

size_t lvl_stride(int m);

// Bump allocator over a caller-given device range: consecutive 256-byte
// aligned blocks, release does nothing (the range is reused as a whole).
class ArenaAllocator final : public DeviceAllocator {
public:
    ArenaAllocator(void* base, size_t bytes) : base_(static_cast<char*>(base)), size_(bytes) {}
    hipError_t alloc(size_t bytes, void** p) override {
        const size_t b = (bytes + 255) / 256 * 256;
        if (b > size_ - off_) return hipErrorOutOfMemory;
        *p = base_ + off_;
        off_ += b;
        return hipSuccess;
    }
    void release(void*) override {}
    size_t used() const { return off_; }

private:
    char* base_;
    size_t size_, off_ = 0;
};

// Device buffers of one sample workspace: the field DFT intermediate and
// the coefficient slots of the fine and coarse meshes.
struct WsBufs {
    void* work = nullptr;
    void* kf = nullptr;
    void* kc = nullptr;
    long long kf_ss = 0, kc_ss = 0;
};

// Workspace of ces_sample_noalloc: every buffer lies at a fixed offset of
// the library's static device array (see noalloc.hip), set up with the plan;
// the solvers keep only host state here.
struct StaticWs {
    int device = -1;
    int units = 0, slots = 0;
    size_t bytes = 0;              // extent of the static array this layout covers
    WsBufs w;
    double *qf = nullptr, *qc = nullptr;
    int *itf = nullptr, *itc = nullptr;
    std::unique_ptr<ArenaAllocator> arena;   // declared before the solvers: outlives them
    std::unique_ptr<Solver> sf, sc;
};

}  // namespace ces

struct ces_context_s {
    int device = 0;
    size_t budget = 0;
    std::atomic<size_t> used{0};
    ces_schedule sched{};
    ces::StreamPool pool;
};

struct ces_plan_s {
    ces_context ctx = nullptr;
    ces_level_desc d{};
    ces::DeviceAllocator* alloc = nullptr;   // source of every device buffer of the plan
    int n = 0, J = 0;
    int64_t tau_f = 0, tau_c = 0;
    double lam_min = 0, lam_max = 0, gap = 0, imag_max = 0;
    int64_t n_clamped = 0;
    ces::DevBuf lam;                    // symmetrised, clamped eigenvalues (n*n doubles)
    std::vector<uint8_t> keep_f, keep_c;  // masks; empty = every eigenvalue kept
    bool is_double = false;
    int nf = 1;                         // DFTs per unit
    ces::FftPlan fp{};
    ces::DevBuf af, ac, tw;
    // sample workspace
    int chunk_units = 0, chunk_slots = 0;
    ces::DevBuf work, kf, kc, qf, qc, itf, itc, zf, zc;
    long long kf_ss = 0, kc_ss = 0;
    std::unique_ptr<ces::Solver> sf, sc;
    size_t ws_bytes = 0;
    // CES_COUPLE_EMBED: the coarse mesh's own embedding (a SINGLE plan of
    // mesh 2h with the coarse drop count); its amplitudes drive the coarse
    // field, its workspace is never used
    std::unique_ptr<ces_plan_s> cpl;
    // quasi-Monte Carlo lattice (HARTLEY plans): q_s coordinates, generating
    // vector q_z (q_s uint32), coordinate of each fine normal counter q_rank
    // (n*n int32, -1 = Philox), q_shifts random shifts; q_s = 0: none
    int32_t q_s = 0, q_shifts = 0;
    ces::DevBuf q_z, q_rank;
    // layout of ces_sample_noalloc (null when a sample unit does not fit)
    std::unique_ptr<ces::StaticWs> sws;
    std::atomic<int> busy{0};           // a scheduler is using the workspace
    // recorded after the last work that used the workspace; the next lane
    // of this plan waits for it (lanes of successive calls may run on
    // different streams)
    hipEvent_t ws_free = nullptr;
    ~ces_plan_s() {
        if (ws_free) (void)hipEventDestroy(ws_free);
    }
};

namespace ces {

// Device bytes per in-flight sample of a plan's workspace.
size_t slot_bytes(const ces_plan p);

// The levels of one estimator must draw independent normals (the variance
// of eq. (mlmc-estimator) is the sum of the level variances only for
// independent levels).  Sample indices restart at 0 on every level and all
// levels share the seed, so the level tag (fourth Philox counter word) is
// what keeps them apart: CES_ERR_ARG unless the tags of level l (levels[l]
// and finest[l], which may share one) differ from those of every other level.
int check_level_tags(const ces_plan* levels, const ces_plan* finest, int nlevels);

// Plan set-up (Algorithm 1 steps 1-3 and the masks of Algorithm 2) with
// device buffers from `alloc`, device work on stream st (synchronised).
// keep_eigenvalues = false drops the n*n eigenvalue array once the
// amplitudes exist (ces_plan_eigenvalues then fails).
int plan_create(ces_context ctx, const ces_level_desc* desc, DeviceAllocator* alloc, hipStream_t st,
                ces_plan* out, bool keep_eigenvalues = true);
int validate_desc(const ces_level_desc* d);
// Upper bound on the device bytes plan_create(d) holds at once (the
// eigenvalue set-up at the largest embedding GROW may try, the masks and
// amplitudes, the coarse plan of an EMBED pair), allowing for the caching
// pool's reuse of slightly larger blocks.
size_t plan_setup_bytes(const ces_level_desc* d);

// Allocates the plan's sample workspace on first use (zeroed on stream st).
// max_slots > 0 caps the samples per chunk (the serving loop sizes
// workspaces per request); 0 sizes it for throughput (about 4.5 GiB, at
// most 8192 samples, 65536 for m <= 32).
int ensure_workspace(ces_plan p, long long max_slots, hipStream_t st);
// Gives the sample workspace back to the plan's allocator (the next
// sampling call makes a new one).  The caller guarantees that no enqueued
// work still uses it.
void drop_workspace(ces_plan p);
// Device bytes ensure_workspace(p, max_slots) would allocate.
size_t workspace_bytes(const ces_plan p, long long max_slots);
// Solver settings of the plan's fine (coarse = false) or coarse mesh.
SolverCfg solver_cfg(const ces_plan p, bool coarse);
// Field batches of units q0 .. q0+units-1 into the workspace buffers w (the
// coarse field of an EMBED pair: make_embedded_batch, enqueued after the
// fine batch on the same stream, since it reuses w.work).
template <typename T>
FieldBatch<T> make_field_batch(ces_plan p, const WsBufs& w, uint64_t seed, uint64_t q0, int units);
template <typename T>
FieldBatch<T> make_embedded_batch(ces_plan p, const WsBufs& w, uint64_t seed, uint64_t q0, int units);

// The static device array behind ces_sample_noalloc (noalloc.hip).
// scratch_init: with `device` current, looks up the array's address on
// that device once (later calls return at once).  scratch_layout: sets up
// p->sws when a sample unit of p fits (no error otherwise: the entry
// point reports it).
int scratch_init(int device);
int scratch_layout(ces_plan p, hipStream_t st);

// Gaussian field of one sample into z_fine / z_coarse (parity hook).
int field_impl(ces_plan p, uint64_t seed, uint64_t sample, double* zf, double* zc, hipStream_t st);
// Solve for caller-given coefficients (parity hook).
int solve_impl(ces_plan p, int grid, int64_t count, const double* k, double* u, int32_t* iters,
               hipStream_t st);

// The sampling scheduler: requests are split into chunks of their plan's
// workspace capacity; each distinct plan is a lane with two streams
// (field + fine solve + finalize, coarse solve) forked from the caller's
// stream when the lane starts; one host thread interleaves the lanes,
// keeping up to `depth` CG iterations of every solve in flight.  A batch
// call joins every lane back into the caller's stream; the serving loop
// instead retires lanes whose work is all enqueued and reuses their
// streams.
class Scheduler {
public:
    Scheduler(StreamPool& pool, hipStream_t caller, const ces_schedule& s);
    ~Scheduler();
    // Queue one request; done_event (may be null) is recorded once all of
    // its results are written.  max_slots > 0 sizes a new workspace for at
    // most that many samples per chunk.
    // y_host / status_host (pinned, may be null): the request's outputs are
    // also copied there before done_event.  *recorded (may be null) is set
    // to 1 once done_event has been recorded: an event that was never
    // recorded counts as complete, so it must not be polled before that.
    int add(const ces_request& r, hipEvent_t done_event, long long max_slots = 0, double* y_host = nullptr,
            int32_t* status_host = nullptr, std::atomic<int>* recorded = nullptr);
    // One pass over the lanes; *progressed = some work was enqueued.
    int step(bool* progressed);
    bool idle() const;
    // step() until idle, waiting on the device when nothing can progress
    int run();
    // make the caller's stream wait for every lane (ends the scheduler's use
    // of the plans)
    int join();
    // Drop the lanes whose queued jobs are all enqueued; their plans are
    // appended to *released (no longer used by the scheduler).
    int retire(std::vector<ces_plan>* released);
    int lanes() const { return (int)lanes_.size(); }
    // solves in progress (for an idle wait of the serving loop)
    int pending_solves() const;

private:
    struct Job {
        uint64_t seed, u0, first, lo, hi;
        int units;
        double *y, *yf, *yc;
        int32_t *iters, *status;
        hipEvent_t done_event;
        // last chunk of a request: copies of its outputs to host memory
        int64_t count;
        double* y_host;
        int32_t* status_host;
        std::atomic<int>* recorded;
    };
    struct Lane {
        ces_plan p = nullptr;
        std::vector<Job> jobs;
        size_t next = 0;
        bool solving = false, fdone = false, cdone = false, forked = false;
        hipStream_t sa = nullptr, sb = nullptr;
        hipEvent_t ev_f = nullptr, ev_c = nullptr, ev_fork = nullptr;
    };
    int lane_of(ces_plan p, Lane** out);
    int start(Lane& L);
    int finish(Lane& L);
    template <typename T>
    int start_t(Lane& L, const Job& j);
    hipError_t get_stream(hipStream_t* s);
    hipError_t get_event(hipEvent_t* e);

    StreamPool& pool_;
    hipStream_t caller_;
    ces_schedule s_;
    std::vector<std::unique_ptr<Lane>> lanes_;
    std::vector<hipStream_t> free_streams_;
    std::vector<hipEvent_t> free_events_;
    size_t next_stream_ = 0, next_event_ = 0;
    bool joined_ = false;
};

}  // namespace ces
