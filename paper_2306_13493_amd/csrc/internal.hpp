// Host-side interfaces between the translation units of the library.
#pragma once

#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "fft_lds.hpp"

namespace ces {

enum { MODE_PAIR = 0, MODE_HARTLEY = 1 };
enum { BC_DIRICHLET0 = 0, BC_FLOWCELL = 1 };
enum { Q_INTEGRAL = 0, Q_POINT = 1, Q_L2 = 2, Q_OUTFLUX = 3 };
enum { COV_MATERN = 0, COV_SEPEXP = 1 };
enum { PERIOD_EUCLID = 0, PERIOD_INF = 1 };

// ------------------------------------------------------ device memory --
// Source of the library's device workspaces: plain hipMalloc/hipFree, or
// a caching pool that keeps released blocks for reuse, so that a serving
// loop never frees (and so never synchronises the device) while other
// streams run.
class DeviceAllocator {
public:
    virtual ~DeviceAllocator() = default;
    virtual hipError_t alloc(size_t bytes, void** p) = 0;
    virtual void release(void* p) = 0;
};
DeviceAllocator* default_allocator();

// Pinned host slots of 4 ints for convergence read-backs, recycled for the
// life of the process (freeing pinned memory would synchronise the device).
int* pinned_slot_acquire();
void pinned_slot_release(int* slot);

// ---------------------------------------------------------- plan set-up --
// Covariance model (Section 2.1): Matern with smoothness nu (pref =
// sigma2 2^(1-nu) / Gamma(nu)), or the separable exponential.
struct CovParams {
    int kind = COV_MATERN;
    double nu = 0.5, lam = 0.1, sigma2 = 1.0, pref = 1.0;
};
// First column of the n x n embedding (Algorithm 1 step 2; n = 2(m + J)),
// index [j2][j1]: C at the minimum-image offsets for J = 0, the smoothly
// periodised covariance of Section 2.2 for J > 0 (cutoff norm `reading`).
hipError_t launch_cov_column(double* s, int n, int m, int J, int reading, const CovParams& c,
                             hipStream_t st);
// out[k] = lam[rep(k)] with rep the orbit representative (min(k, n-k) per
// axis, pair sorted); per-block minimum, maximum and count of negatives.
// nblk receives the number of blocks.
hipError_t launch_symmetrise(const double* lam, double* out, int n, double* bmin, double* bmax,
                             int* bneg, int* nblk, hipStream_t st);
int symmetrise_blocks(int n);
// lam <- max(lam, 0); af = sqrt(lam)/n masked by keep_f (null = all kept),
// ac likewise with keep_c (ac may be null).
template <typename T>
hipError_t launch_amplitudes(double* lam, int n, const uint8_t* keep_f, const uint8_t* keep_c, T* af,
                             T* ac, hipStream_t st);

// ---------------------------------------------------------------- field --
// One batch of DFT units (pairs in PAIR mode, samples in HARTLEY mode):
// xi from Philox/Box-Muller, w = a (.) xi, 2-D DFT pruned to the first m+1
// outputs per axis, Z restricted to the fine nodes and to the even (coarse)
// nodes, k = exp(Z).
template <typename T>
struct FieldBatch {
    int n = 0, m = 0;
    int mode = MODE_PAIR;
    int nf = 1;              // DFTs per unit: 1, or 2 when fine/coarse masks differ
    bool coarse = false;     // also write the coarse-mesh field
    const T* af = nullptr;   // amplitudes sqrt(Lambda)/n (fine mask), n*n
    const T* ac = nullptr;   // amplitudes of the coarse mask (nf == 2)
    const cplx<T>* tw = nullptr;
    FftPlan fp{};
    uint64_t seed = 0;
    uint64_t q0 = 0;         // first unit index of the batch
    uint32_t stream = 0;
    int units = 0;           // units in this batch
    cplx<T>* work = nullptr; // nf * units * (m+1) * n
    // outputs per slot (slot = 2u + c in PAIR mode, u in HARTLEY mode)
    T* kf = nullptr; long long kf_stride = 0;   // exp(Z) on (m+1)^2 nodes
    T* kc = nullptr; long long kc_stride = 0;   // exp(Z) on (m/2+1)^2 nodes
    double* zf = nullptr;    // if set: Z (not exp) as double, stride (m+1)^2
    double* zc = nullptr;    // if set: Z coarse as double, stride (m/2+1)^2
    // > 0: draw the normals of the embedding of size n_src of the mesh with
    // half this one's spacing, at the nearest signed frequencies
    int n_src = 0;
    // lattice (HARTLEY only): qrank[e] = coordinate of normal counter e or
    // -1; qz = generating vector; unit q is point q / qshifts of shift
    // q mod qshifts.  qrank = nullptr: Philox normals everywhere
    const int32_t* qrank = nullptr;
    const uint32_t* qz = nullptr;
    int qshifts = 0;
};
template <typename T>
hipError_t launch_field(const FieldBatch<T>& b, hipStream_t st);

// FP64 2-D DFT (+ sign) of a real n x n array s (Algorithm 1 step 3):
// lam = Re(DFT s), imag_blk[blk] = per-block max |Im|.  work: n*n complex.
hipError_t launch_eigen_fft(const double* s, int n, const FftPlan& fp, const cplx<double>* tw,
                            cplx<double>* work, double* lam, double* imag_blk, int* nblk,
                            hipStream_t st);

hipError_t launch_normals(uint64_t seed, uint64_t q, uint32_t stream, uint64_t first_e,
                          long long count, double* out, hipStream_t st);

hipError_t launch_convert_d2f(const double* in, float* out, long long count, hipStream_t st);

// --------------------------------------------------------------- solver --
struct SolverCfg {
    int m = 0;          // intervals per side of the mesh
    int bc = BC_DIRICHLET0;
    double f = 1.0;
    double rtol = 1e-10;
    int maxit = 500;
    int qoi = Q_INTEGRAL;
    double qx = 7.0 / 15.0, qy = 7.0 / 15.0;
    // visit multigrid level 1 twice per cycle when it is a whole level
    // (fewer CG iterations for a few extra launches: worth it where chunks
    // hold many samples, as single levels do, and the coarse levels resolve
    // the coefficient)
    bool twice1 = false;
};

// Batched PCG (double) preconditioned by a geometric multigrid V(2,2) cycle
// in T (level 1 visited twice when SolverCfg::twice1 asks and it is a whole
// level), for S samples of one mesh at a time.  A solve is a small state
// machine so that one host thread can interleave the solves of several
// meshes on several streams: begin() enqueues the set-up, each advance()
// enqueues at most one more iteration and notes (without blocking) which
// enqueued iterations have finished; the solve is done once the count of
// unconverged samples read back after some iteration is zero.
class Solver {
public:
    virtual ~Solver() = default;
    virtual int capacity() const = 0;
    virtual size_t bytes() const = 0;
    virtual int mg_levels() const = 0;
    // k: capacity x kstride values of T (slot s at k + s*kstride); slots
    // [0, S) are solved.  keep_x = false lets a solve whose QoI is linear
    // in u skip the iterate (x() then holds only the Dirichlet lifting).
    virtual hipError_t begin(const void* k, long long kstride, int S, hipStream_t st, bool keep_x) = 0;
    // depth: iterations allowed in flight before their convergence count
    // has been read back (1..4).  graphs: replay iterations from captured
    // HIP graphs (same kernels and arguments).  *progressed: an iteration
    // was enqueued.
    virtual hipError_t advance(hipStream_t st, int depth, bool graphs, bool* done, bool* progressed) = 0;
    // block until the oldest unconfirmed iteration has finished
    virtual hipError_t wait() = 0;
    // bookkeeping after the solve (launch profiler only; host-side, no device wait)
    virtual hipError_t finish(hipStream_t st) = 0;
    // begin + advance to the end + finish
    hipError_t solve(const void* k, long long kstride, int S, hipStream_t st, int depth = 2) {
        hipError_t e = begin(k, kstride, S, st, true);
        bool done = false, prog = false;
        while (e == hipSuccess && !done) {
            e = advance(st, depth, false, &done, &prog);
            if (e == hipSuccess && !done && !prog) e = wait();
        }
        return e == hipSuccess ? finish(st) : e;
    }
    // QoI of the last solve for slots [0, S): q[s], iters[s] (-it if not
    // converged); either may be null.
    virtual hipError_t qoi(const void* k, long long kstride, int S, double* q, int* iters,
                           hipStream_t st) = 0;
    // Nodal solution (double, (m+1)^2 per slot, dense) of a solve begun
    // with keep_x.
    virtual const double* x() const = 0;
    virtual long long xstride() const = 0;
};
// is_double selects T = double (plain path) or float (mixed path).  The
// workspace comes from `alloc` and is zeroed on stream st (by a kernel)
// unless zero = false (the caller zeroes it before every use).
std::unique_ptr<Solver> make_solver(const SolverCfg& cfg, int capacity, bool is_double,
                                    DeviceAllocator* alloc, hipStream_t st, std::string* err, bool zero = true);
// Device bytes make_solver(cfg, capacity, is_double, ...) takes from its
// allocator (host arithmetic only).
size_t solver_bytes(const SolverCfg& cfg, int capacity, bool is_double);
// Zero `bytes` bytes at dst (a multiple of 4, dst 4-byte aligned) with a
// kernel (no memset node when the stream is being captured).
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st);

// y[i] = qf[i] - qc[i] (or qf if qc null) scattered to out slots.
hipError_t launch_finalize(const double* qf, const double* qc, const int* itf, const int* itc,
                           int slot0, int nslots, long long out0, double* y, double* yf, double* yc,
                           int* iters, int* status, hipStream_t st);

// ------------------------------------------------------------- profiler
// Process-wide; times launches with HIP events while enabled.
// Thread-safe (a server's loop may launch while its owner reads).
class Profiler {
public:
    struct Entry {
        std::string name;
        long long launches = 0;
        double ms = 0.0;
        double bytes = 0.0;   // algorithmic bytes summed over launches
    };
    // Events of one launch: passed to hipExtLaunchKernelGGL, which stamps
    // them with the kernel's own start and end (no extra packets in the
    // stream); both null and idx = -1 when the profiler is off.
    struct Slot {
        int idx = -1;
        hipEvent_t a = nullptr, b = nullptr;
    };
    static Profiler& get();
    bool on() const { return on_.load(std::memory_order_relaxed); }
    void enable(bool on);
    // record only launches of kernel `name` (null or empty: every kernel)
    void only(const char* name);
    Slot begin(const char* name = nullptr);
    void end(const Slot& s, const char* name, double bytes_per_sample, int samples);
    void set_samples(int idx, int samples);
    int read(std::vector<Entry>& out);   // synchronises; clears the records

private:
    struct Rec {
        const char* name = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
        double bps = 0.0;
        int samples = 0;
    };
    std::atomic<bool> on_{false};
    std::mutex mu_;
    std::string only_;
    std::vector<Rec> recs_;
    std::vector<hipEvent_t> pool_;
    size_t used_ = 0;
    hipEvent_t event();
};

}  // namespace ces
