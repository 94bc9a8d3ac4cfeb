// ces_sample_noalloc: the level samples of ces_sample (Algorithm 1 step 4
// and the difference of Section 3.4) with every device workspace buffer --
// field DFT intermediate, coefficient slots, solver vectors and multigrid
// levels, per-sample scalars -- carved from one static device array, so
// that a call allocates no memory.  For callers that cannot allocate.
//
// The array is `scratch` below (kScratchBytes per device, held from the
// library's load until the process ends).  Its device address is looked up
// once per device when a context is created (scratch_init); host code uses
// only that address, never the array's name.  Each plan made by
// ces_plan_create whose sample unit fits gets a fixed layout of the array
// (scratch_layout: offsets and the solvers' host state; nothing is written
// to the array then).  A call zeroes the layout's extent with a kernel,
// then runs the field, solve and finalize kernels of ces_sample on the
// caller's stream, chunk by chunk.  All calls on a device share the array:
// calls that overlap on one device (other streams, other threads) race.
#include <algorithm>
#include <map>
#include <mutex>

#include "plan.hpp"

namespace ces {
namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void*> g_scratch;   // device -> address of `scratch` there

void* scratch_address(int device) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_scratch.find(device);
    return it == g_scratch.end() ? nullptr : it->second;
}

// Device bytes of a layout of `units` DFT units; solvers sized for their
// slots (host arithmetic only).
size_t layout_bytes(const ces_plan p, long long units) {
    auto r = [](size_t b) { return (b + 255) / 256 * 256; };
    const int m = p->d.m_fine;
    const bool pair_level = p->d.level_kind == CES_LEVEL_PAIR;
    const long long slots = units * (p->d.field_mode == CES_FIELD_PAIR ? 2 : 1);
    const size_t tb = p->is_double ? 8 : 4;
    size_t b = r((size_t)p->nf * units * (m + 1) * p->n * 2 * tb);
    b += r((size_t)slots * lvl_stride(m) * tb);
    if (pair_level) b += r((size_t)slots * lvl_stride(m / 2) * tb);
    b += 2 * r((size_t)slots * 8) + 2 * r((size_t)slots * 4);
    b += r(solver_bytes(solver_cfg(p, false), (int)slots, p->is_double));
    if (pair_level) b += r(solver_bytes(solver_cfg(p, true), (int)slots, p->is_double));
    return b;
}

template <typename T>
int run_t(ces_plan p, uint64_t seed, uint64_t first, int64_t count, double* y, double* yf, double* yc,
          int32_t* iters, int32_t* status, hipStream_t st) {
    StaticWs& W = *p->sws;
    const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
    const int depth = p->ctx->sched.depth > 0 ? p->ctx->sched.depth : 2;
    auto solve = [&](Solver* S, void* k, long long kss, int n) -> hipError_t {
        hipError_t e = S->begin(k, kss, n, st, false);
        bool done = false, prog = false;
        while (e == hipSuccess && !done) {
            e = S->advance(st, depth, false, &done, &prog);
            if (e == hipSuccess && !done && !prog) e = S->wait();
        }
        return e == hipSuccess ? S->finish(st) : e;
    };
    const uint64_t last = first + (uint64_t)count - 1;
    const uint64_t u_begin = first / per_unit, u_end = last / per_unit + 1;
    // the fewest chunks the layout allows, of equal size
    const uint64_t nch = (u_end - u_begin + (uint64_t)W.units - 1) / (uint64_t)W.units;
    const uint64_t cu = (u_end - u_begin + nch - 1) / nch;
    for (uint64_t u0 = u_begin; u0 < u_end; u0 += cu) {
        const int units = (int)std::min<uint64_t>(cu, u_end - u0);
        const int nslots = units * per_unit;
        CES_HIP(launch_field<T>(make_field_batch<T>(p, W.w, seed, u0, units), st), "field kernels");
        if (p->cpl) CES_HIP(launch_field<T>(make_embedded_batch<T>(p, W.w, seed, u0, units), st), "coarse field kernels");
        CES_HIP(solve(W.sf.get(), W.w.kf, W.w.kf_ss, nslots), "fine solve");
        CES_HIP(W.sf->qoi(W.w.kf, W.w.kf_ss, nslots, W.qf, W.itf, st), "fine qoi");
        if (W.sc) {
            CES_HIP(solve(W.sc.get(), W.w.kc, W.w.kc_ss, nslots), "coarse solve");
            CES_HIP(W.sc->qoi(W.w.kc, W.w.kc_ss, nslots, W.qc, W.itc, st), "coarse qoi");
        }
        const uint64_t s0 = u0 * per_unit;
        const uint64_t lo = std::max(first, s0), hi = std::min(last + 1, s0 + (uint64_t)nslots);
        CES_HIP(launch_finalize(W.qf, W.sc ? W.qc : nullptr, W.itf, W.sc ? W.itc : nullptr, (int)(lo - s0),
                                (int)(hi - lo), (long long)(lo - first), y, yf, yc, iters, status, st),
                "finalize");
    }
    return CES_OK;
}

}  // namespace

int scratch_init(int device) {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_scratch.count(device)) return CES_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch[device] = ptr;
    return CES_OK;
}

int scratch_layout(ces_plan p, hipStream_t st) {
    if (p->sws) return CES_OK;
    void* base = scratch_address(p->ctx->device);
    if (!base) return fail(CES_ERR_DEVICE, "static scratch not set up on this device");
    const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
    // as many units as fit, under the per-chunk caps of the plan's own
    // workspace (65536 samples for m <= 32, 8192 otherwise)
    const long long cap = (p->d.m_fine <= 32 ? 65536 : 8192) / per_unit;
    long long units = std::min<long long>(cap, (long long)(kScratchBytes / (slot_bytes(p) * per_unit)) + 1);
    while (units > 0 && layout_bytes(p, units) > kScratchBytes) --units;
    if (units <= 0) return CES_OK;   // too large: ces_sample_noalloc says so
    const int m = p->d.m_fine;
    const size_t tb = p->is_double ? 8 : 4;
    const long long slots = units * per_unit;
    auto W = std::make_unique<StaticWs>();
    W->device = p->ctx->device;
    W->units = (int)units;
    W->slots = (int)slots;
    W->arena = std::make_unique<ArenaAllocator>(base, kScratchBytes);
    ArenaAllocator& A = *W->arena;
    W->w.kf_ss = (long long)lvl_stride(m);
    W->w.kc_ss = (long long)lvl_stride(m / 2);
    CES_HIP(A.alloc((size_t)p->nf * units * (m + 1) * p->n * 2 * tb, &W->w.work), "static layout");
    CES_HIP(A.alloc((size_t)slots * W->w.kf_ss * tb, &W->w.kf), "static layout");
    if (p->d.level_kind == CES_LEVEL_PAIR) CES_HIP(A.alloc((size_t)slots * W->w.kc_ss * tb, &W->w.kc), "static layout");
    void* v = nullptr;
    CES_HIP(A.alloc((size_t)slots * 8, &v), "static layout");
    W->qf = static_cast<double*>(v);
    CES_HIP(A.alloc((size_t)slots * 8, &v), "static layout");
    W->qc = static_cast<double*>(v);
    CES_HIP(A.alloc((size_t)slots * 4, &v), "static layout");
    W->itf = static_cast<int*>(v);
    CES_HIP(A.alloc((size_t)slots * 4, &v), "static layout");
    W->itc = static_cast<int*>(v);
    std::string err;
    // the solvers only take their offsets here: the array is zeroed by each call
    W->sf = make_solver(solver_cfg(p, false), (int)slots, p->is_double, &A, st, &err, false);
    if (!W->sf) return fail(CES_ERR_DEVICE, err);
    if (p->d.level_kind == CES_LEVEL_PAIR) {
        W->sc = make_solver(solver_cfg(p, true), (int)slots, p->is_double, &A, st, &err, false);
        if (!W->sc) return fail(CES_ERR_DEVICE, err);
    }
    W->bytes = A.used();
    p->sws = std::move(W);
    return CES_OK;
}

}  // namespace ces

using namespace ces;

extern "C" int ces_sample_noalloc(ces_plan p, uint64_t seed, uint64_t first, int64_t count, double* y, double* yf,
                                  double* yc, int32_t* iters, int32_t* status, void* stream) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    if (count < 0) return fail(CES_ERR_ARG, "count < 0");
    if (count == 0) return CES_OK;
    if (!y) return fail(CES_ERR_ARG, "y is NULL");
    if (first + (uint64_t)count < first) return fail(CES_ERR_ARG, "sample range overflows");
    if (p->q_s > 0 && first + (uint64_t)count > (1ull << 63))
        return fail(CES_ERR_ARG, "sample indices of a lattice plan must stay below 2^63");
    if (!p->sws) {
        const int per_unit = p->d.field_mode == CES_FIELD_PAIR ? 2 : 1;
        return fail(CES_ERR_ARG, "one sample unit of this plan needs " + std::to_string(layout_bytes(p, 1)) +
                                     " bytes of workspace (" + std::to_string(per_unit) +
                                     " samples); the static scratch holds " + std::to_string(kScratchBytes) +
                                     " bytes");
    }
    if (p->sws->device != p->ctx->device) return fail(CES_ERR_ARG, "plan layout belongs to another device");
    int z = 0;
    if (!p->busy.compare_exchange_strong(z, 1)) return fail(CES_ERR_BUSY, "plan is in use by another call");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = CES_OK;
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e == hipSuccess) e = launch_zero(scratch_address(p->ctx->device), p->sws->bytes, st);
    if (e != hipSuccess) rc = hip_fail(e, "static scratch");
    if (rc == CES_OK)
        rc = p->is_double ? run_t<double>(p, seed, first, count, y, yf, yc, iters, status, st)
                          : run_t<float>(p, seed, first, count, y, yf, yc, iters, status, st);
    p->busy.store(0);
    return rc;
}
