// C ABI of the library: contexts, plans (Algorithm 1 steps 1-3 and the
// masks of Algorithm 2), the level-sample driver (Algorithm 1 step 4 with
// the level difference of Section 3.4) and the parity hooks.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace ces;


namespace {

constexpr double kPsdTol = 1e-13;

template <typename T>
std::vector<cplx<T>> twiddles(int n) {
    std::vector<cplx<T>> tw(n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < n; ++t) {
        const double a = two_pi * (double)t / (double)n;
        tw[t] = cplx<T>{(T)std::cos(a), (T)std::sin(a)};
    }
    return tw;
}

// Algorithm 2 step 4(b): the tau smallest in the order (Lambda descending,
// index ascending) are dropped.  drop_order receives the first `tmax`
// indices of the reverse order (smallest first).
void smallest_order(const std::vector<double>& lam, int64_t tmax, std::vector<int64_t>& drop_order) {
    const int64_t s = (int64_t)lam.size();
    std::vector<int64_t> idx(s);
    std::iota(idx.begin(), idx.end(), 0);
    auto less = [&](int64_t a, int64_t b) {  // "drops earlier"
        if (lam[a] != lam[b]) return lam[a] < lam[b];
        return a > b;
    };
    if (tmax > 0 && tmax < s) {
        std::nth_element(idx.begin(), idx.begin() + tmax, idx.end(), less);
        std::sort(idx.begin(), idx.begin() + tmax, less);
    } else if (tmax >= s) {
        std::sort(idx.begin(), idx.end(), less);
    }
    drop_order.assign(idx.begin(), idx.begin() + std::min(tmax, s));
    if (tmax < s) drop_order.push_back(*std::min_element(idx.begin() + tmax, idx.end(), less));  // first kept
}

// Scratch of one embedding-size candidate: column, DFT work, raw and
// symmetrised eigenvalues, per-block reductions.
struct SetupBufs {
    DevBuf s, work, raw, tw, blk;
};

// Algorithm 1 steps 2-3(a) at embedding size n = 2(m + J) on the device:
// column, FP64 2-D DFT, orbit symmetrisation into `lam`; host receives the
// extremes, the count of negatives and the largest imaginary part.
int eigen_candidate(const ces_level_desc* d, const CovParams& cp, int J, DeviceAllocator* A, hipStream_t st,
                    SetupBufs& B, DevBuf& lam, double* lmin, double* lmax, int64_t* nneg, double* imag) {
    const int m = d->m_fine, n = 2 * (m + J);
    const size_t nn = (size_t)n * n;
    const FftPlan fp = make_fft_plan(n);
    const int nsym = symmetrise_blocks(n);
    const size_t blk_bytes = (size_t)(n + 2 * nsym) * 8 + (size_t)nsym * 4;
    CES_HIP(B.s.alloc(nn * 8, A), "set-up buffers");
    CES_HIP(B.work.alloc(nn * 16, A), "set-up buffers");
    CES_HIP(B.raw.alloc(nn * 8, A), "set-up buffers");
    CES_HIP(B.tw.alloc((size_t)n * sizeof(cplx<double>), A), "set-up buffers");
    CES_HIP(B.blk.alloc(blk_bytes, A), "set-up buffers");
    CES_HIP(lam.alloc(nn * 8, A), "eigenvalue buffer");
    const auto tw = twiddles<double>(n);
    CES_HIP(hipMemcpyAsync(B.tw.p, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice, st), "twiddles");
    double* imag_blk = B.blk.as<double>();
    double* bmin = imag_blk + n;
    double* bmax = bmin + nsym;
    int* bneg = reinterpret_cast<int*>(bmax + nsym);
    CES_HIP(launch_cov_column(B.s.as<double>(), n, m, J, d->periodization, cp, st), "covariance column");
    int nblk = 0, nb2 = 0;
    CES_HIP(launch_eigen_fft(B.s.as<double>(), n, fp, B.tw.as<cplx<double>>(), B.work.as<cplx<double>>(),
                             B.raw.as<double>(), imag_blk, &nblk, st),
            "eigenvalue DFT");
    CES_HIP(launch_symmetrise(B.raw.as<double>(), lam.as<double>(), n, bmin, bmax, bneg, &nb2, st), "symmetrise");
    std::vector<unsigned char> h(blk_bytes);
    CES_HIP(hipMemcpyAsync(h.data(), B.blk.p, blk_bytes, hipMemcpyDeviceToHost, st), "eigenvalue extremes");
    CES_HIP(hipStreamSynchronize(st), "plan set-up");
    const double* hi = reinterpret_cast<const double*>(h.data());
    const double* hmin = hi + n;
    const double* hmax = hmin + nsym;
    const int* hneg = reinterpret_cast<const int*>(hmax + nsym);
    *imag = *std::max_element(hi, hi + nblk);
    *lmin = *std::min_element(hmin, hmin + nb2);
    *lmax = *std::max_element(hmax, hmax + nb2);
    int64_t c = 0;
    for (int i = 0; i < nb2; ++i) c += hneg[i];
    *nneg = c;
    return CES_OK;
}

}  // namespace

namespace ces {

int plan_create(ces_context ctx, const ces_level_desc* desc, DeviceAllocator* A, hipStream_t st, ces_plan* out,
                bool keep_eigenvalues) {
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc != CES_OK) return rc;
    std::unique_ptr<ces_plan_s> p(new ces_plan_s);
    p->ctx = ctx;
    p->d = *desc;
    p->alloc = A;
    const int m = desc->m_fine;
    CovParams cp;
    cp.kind = desc->cov_kind == CES_COV_SEPEXP ? COV_SEPEXP : COV_MATERN;
    cp.nu = desc->nu;
    cp.lam = desc->lambda;
    cp.sigma2 = desc->sigma2;
    cp.pref = desc->sigma2 * std::pow(2.0, 1.0 - desc->nu) / std::tgamma(desc->nu);
    std::vector<int> cands;
    if (desc->psd_policy == CES_PSD_GROW) {
        for (int J : {0, m / 2, m})
            if (2 * (m + J) <= desc->max_pad_factor * m) cands.push_back(J);
    } else {
        cands.push_back(0);
    }
    bool ok = false;
    int64_t nneg = 0;
    {
        SetupBufs B;
        for (int J : cands) {
            // the Euclidean cutoff needs a plateau radius sqrt(2) < kappa
            if (J > 0 && desc->periodization == CES_PERIOD_EUCLID && !(1.0 + (double)J / m > std::sqrt(2.0))) continue;
            const int n = 2 * (m + J);
            if (make_fft_plan(n).nst < 0) continue;
            double lmin = 0, lmax = 0, imag = 0;
            rc = eigen_candidate(desc, cp, J, A, st, B, p->lam, &lmin, &lmax, &nneg, &imag);
            if (rc != CES_OK) return rc;
            p->n = n;
            p->J = J;
            p->lam_min = lmin;
            p->lam_max = lmax;
            p->imag_max = imag;
            ok = lmin >= -kPsdTol * lmax;
            if (ok || desc->psd_policy == CES_PSD_CLAMP) break;
        }
    }
    if (p->n == 0) return fail(CES_ERR_ARG, "no admissible embedding size");
    if (!ok && desc->psd_policy != CES_PSD_CLAMP)
        return fail(CES_ERR_NOT_PSD, "embedding has negative eigenvalues up to the padding cap (min/max = " +
                                         std::to_string(p->lam_min / p->lam_max) + ")");
    // after acceptance every negative (noise, or CLAMP) becomes zero
    p->n_clamped = nneg;
    const int n = p->n;
    const int64_t s = (int64_t)n * n;
    const bool embed = desc->coupling == CES_COUPLE_EMBED;
    p->tau_f = desc->tau_fine < 0 ? n : desc->tau_fine;
    p->tau_c = desc->tau_coarse < 0 ? n : desc->tau_coarse;
    if (desc->level_kind == CES_LEVEL_SINGLE) p->tau_c = p->tau_f;
    if (embed) {
        // the coarse field comes from the coarse mesh's own embedding: a
        // SINGLE plan of mesh 2h with the coarse drop count
        ces_level_desc cd = *desc;
        cd.m_fine = m / 2;
        cd.level_kind = CES_LEVEL_SINGLE;
        cd.tau_fine = cd.tau_coarse = desc->tau_coarse;
        cd.coupling = CES_COUPLE_RESTRICT;
        ces_plan child = nullptr;
        rc = plan_create(ctx, &cd, A, st, &child, false);
        if (rc != CES_OK) return rc;
        p->cpl.reset(child);
        if (n < 2 * child->n)
            return fail(CES_ERR_ARG, "coupling EMBED needs a fine embedding period at least the coarse one's (fine "
                                     "n = " + std::to_string(n) + ", coarse n = " + std::to_string(child->n) + ")");
        p->tau_c = child->tau_f;
    }
    // drop count of a second fine-embedding field (RESTRICT pairs only)
    const int64_t tau_c2 = embed ? p->tau_f : p->tau_c;
    if (p->tau_f > s || tau_c2 > s) return fail(CES_ERR_ARG, "tau exceeds the number of eigenvalues");
    p->is_double = desc->precision == CES_PREC_FP64;
    p->nf = (desc->level_kind == CES_LEVEL_PAIR && p->tau_f != tau_c2) ? 2 : 1;
    // two DFTs of one xi share a workgroup's LDS: 2 n complex values fit
    // up to n = 4096
    if (p->nf == 2 && n > 4096)
        return fail(CES_ERR_ARG, "a pair level whose fine and coarse drop counts differ needs an embedding of at "
                                 "most 4096 per axis (this one has " + std::to_string(n) + ")");
    p->fp = make_fft_plan(n);
    DevBuf kf_d, kc_d;
    if (p->tau_f > 0 || tau_c2 > 0) {
        // masks: the host orders the clamped eigenvalues
        std::vector<double> lam(s);
        CES_HIP(hipMemcpyAsync(lam.data(), p->lam.p, (size_t)s * 8, hipMemcpyDeviceToHost, st), "eigenvalues");
        CES_HIP(hipStreamSynchronize(st), "plan set-up");
        for (double& v : lam) v = std::max(v, 0.0);
        std::vector<int64_t> order;
        smallest_order(lam, std::max(p->tau_f, tau_c2), order);
        p->keep_f.assign(s, 1);
        p->keep_c.assign(s, 1);
        for (int64_t i = 0; i < p->tau_f; ++i) p->keep_f[order[i]] = 0;
        for (int64_t i = 0; i < tau_c2; ++i) p->keep_c[order[i]] = 0;
        if (tau_c2 > 0 && tau_c2 < s) {
            double kept_min = 1e308;
            for (int64_t i = 0; i < s; ++i)
                if (p->keep_c[i]) kept_min = std::min(kept_min, lam[i]);
            p->gap = (kept_min - lam[order[tau_c2 - 1]]) / std::max(p->lam_max, 1e-300);
        }
        CES_HIP(kf_d.alloc((size_t)s, A), "mask buffers");
        CES_HIP(kc_d.alloc((size_t)s, A), "mask buffers");
        CES_HIP(hipMemcpyAsync(kf_d.p, p->keep_f.data(), (size_t)s, hipMemcpyHostToDevice, st), "masks");
        CES_HIP(hipMemcpyAsync(kc_d.p, p->keep_c.data(), (size_t)s, hipMemcpyHostToDevice, st), "masks");
    }
    if (embed) p->gap = p->cpl->gap;   // the coarse field's mask is the coarse plan's
    const size_t tb = p->is_double ? 8 : 4;
    CES_HIP(p->af.alloc((size_t)s * tb, A), "amplitude buffers");
    if (p->nf == 2) CES_HIP(p->ac.alloc((size_t)s * tb, A), "amplitude buffers");
    const uint8_t* mf = kf_d.as<uint8_t>();
    const uint8_t* mc = kc_d.as<uint8_t>();
    if (p->is_double)
        CES_HIP(launch_amplitudes<double>(p->lam.as<double>(), n, mf, mc, p->af.as<double>(),
                                          p->nf == 2 ? p->ac.as<double>() : nullptr, st),
                "amplitudes");
    else
        CES_HIP(launch_amplitudes<float>(p->lam.as<double>(), n, mf, mc, p->af.as<float>(),
                                         p->nf == 2 ? p->ac.as<float>() : nullptr, st),
                "amplitudes");
    CES_HIP(p->tw.alloc((size_t)n * (p->is_double ? sizeof(cplx<double>) : sizeof(cplx<float>)), A), "twiddles");
    if (p->is_double) {
        const auto tw = twiddles<double>(n);
        CES_HIP(hipMemcpyAsync(p->tw.p, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice, st), "twiddles");
        CES_HIP(hipStreamSynchronize(st), "plan set-up");
    } else {
        const auto tw = twiddles<float>(n);
        CES_HIP(hipMemcpyAsync(p->tw.p, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice, st), "twiddles");
        CES_HIP(hipStreamSynchronize(st), "plan set-up");
    }
    if (!keep_eigenvalues) p->lam.reset();
    *out = p.release();
    return CES_OK;
}

}  // namespace ces

extern "C" {

int ces_profile_enable(int32_t on) {
    Profiler::get().enable(on != 0);
    return CES_OK;
}

int ces_profile_only(const char* name) {
    Profiler::get().only(name);
    return CES_OK;
}

int ces_profile_read(ces_profile_entry* out, int32_t max_entries, int32_t* n_entries) {
    if (max_entries < 0 || (max_entries > 0 && !out)) return fail(CES_ERR_ARG, "profile output buffer");
    std::vector<Profiler::Entry> v;
    if (Profiler::get().read(v) != 0) return fail(CES_ERR_DEVICE, "profile events could not be read");
    const int n = std::min<int>((int)v.size(), max_entries);
    for (int i = 0; i < n; ++i) {
        std::memset(&out[i], 0, sizeof(out[i]));
        std::strncpy(out[i].name, v[i].name.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = v[i].launches;
        out[i].total_ms = v[i].ms;
        out[i].bytes = v[i].bytes;
    }
    if (n_entries) *n_entries = (int32_t)v.size();
    return CES_OK;
}

int ces_context_create(int device, size_t mem_budget_bytes, ces_context* out) {
    if (!out) return fail(CES_ERR_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    CES_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(CES_ERR_ARG, "no such device");
    CES_HIP(hipSetDevice(device), "hipSetDevice");
    size_t fr = 0, tot = 0;
    CES_HIP(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    // the static array of ces_sample_noalloc: its address on this device
    int rc = scratch_init(device);
    if (rc != CES_OK) return rc;
    auto* c = new ces_context_s;
    c->device = device;
    c->budget = mem_budget_bytes ? mem_budget_bytes : (size_t)(0.9 * (double)fr);
    *out = c;
    return CES_OK;
}

int ces_context_destroy(ces_context ctx) {
    delete ctx;
    return CES_OK;
}

int ces_plan_create(ces_context ctx, const ces_level_desc* desc, ces_plan* out) {
    if (!ctx || !out) return fail(CES_ERR_ARG, "context or out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc != CES_OK) return rc;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = nullptr;
    CES_HIP(ctx->pool.stream(0, &st), "set-up stream");
    rc = plan_create(ctx, desc, default_allocator(), st, out);
    if (rc != CES_OK) return rc;
    // offsets of ces_sample_noalloc's workspace in the static array
    rc = scratch_layout(*out, st);
    if (rc != CES_OK) {
        ces_plan_destroy(*out);
        *out = nullptr;
    }
    return rc;
}

int ces_plan_info_get(ces_plan p, ces_plan_info* info) {
    if (!p || !info) return fail(CES_ERR_ARG, "plan or info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->n = p->n;
    info->J = p->J;
    info->lam_min = p->lam_min;
    info->lam_max = p->lam_max;
    info->n_clamped = p->n_clamped;
    info->tau_fine = p->tau_f;
    info->tau_coarse = p->tau_c;
    info->boundary_gap = p->gap;
    int lv = 0;
    for (int mm = p->d.m_fine; mm >= 2; mm /= 2) ++lv;
    info->mg_levels = lv;
    info->n_coarse = p->cpl ? p->cpl->n : p->n;
    info->bytes_per_sample = slot_bytes(p);
    return CES_OK;
}

int ces_plan_destroy(ces_plan p) {
    if (!p) return CES_OK;
    (void)hipSetDevice(p->ctx->device);
    p->ctx->used -= std::min(p->ctx->used.load(), p->ws_bytes);
    delete p;
    return CES_OK;
}

int ces_normals(uint64_t seed, uint64_t q, uint32_t stream, uint64_t first_e, int64_t count, double* out,
                void* hs) {
    if (count < 0) return fail(CES_ERR_ARG, "count < 0");
    if (count > 0 && !out) return fail(CES_ERR_ARG, "out is NULL");
    if (first_e + (uint64_t)count > (1ull << 32)) return fail(CES_ERR_ARG, "element index exceeds 32 bits");
    CES_HIP(launch_normals(seed, q, stream, first_e, count, out, reinterpret_cast<hipStream_t>(hs)), "normals");
    return CES_OK;
}

int ces_plan_eigenvalues(ces_plan p, double* host_out) {
    if (!p || !host_out) return fail(CES_ERR_ARG, "plan or out is NULL");
    if (!p->lam.p) return fail(CES_ERR_ARG, "plan kept no eigenvalues");
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    CES_HIP(hipMemcpy(host_out, p->lam.p, (size_t)p->n * p->n * 8, hipMemcpyDeviceToHost), "download eigenvalues");
    return CES_OK;
}

int ces_plan_mask(ces_plan p, uint8_t* f, uint8_t* c) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    const size_t s = (size_t)p->n * p->n;
    if (f) {
        if (p->keep_f.empty()) std::memset(f, 1, s);
        else std::memcpy(f, p->keep_f.data(), s);
    }
    if (c) {
        // EMBED: the coarse field's mask lives on the coarse embedding
        const ces_plan_s* q = p->cpl ? p->cpl.get() : p;
        const std::vector<uint8_t>& kc = p->cpl ? q->keep_f : q->keep_c;
        const size_t sc = (size_t)q->n * q->n;
        if (kc.empty()) std::memset(c, 1, sc);
        else std::memcpy(c, kc.data(), sc);
    }
    return CES_OK;
}

int ces_field(ces_plan p, uint64_t seed, uint64_t sample, double* zf, double* zc, void* stream) {
    if (!p || !zf) return fail(CES_ERR_ARG, "plan or z_fine is NULL");
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return field_impl(p, seed, sample, zf, zc, st);
}

int ces_solve(ces_plan p, int32_t grid, int64_t count, const double* k, double* u, int32_t* iters, void* stream) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    if (grid != 0 && grid != 1) return fail(CES_ERR_ARG, "grid must be 0 (fine) or 1 (coarse)");
    if (grid == 1 && p->d.level_kind != CES_LEVEL_PAIR) return fail(CES_ERR_ARG, "coarse grid needs a PAIR plan");
    if (count < 0) return fail(CES_ERR_ARG, "count < 0");
    if (count == 0) return CES_OK;
    if (!k || !u) return fail(CES_ERR_ARG, "k or u is NULL");
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return solve_impl(p, grid, count, k, u, iters, st);
}

}  // extern "C"
