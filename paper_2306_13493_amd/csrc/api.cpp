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

namespace ces {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
int hip_fail(hipError_t e, const char* what) {
    return fail(CES_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace ces

namespace {

constexpr double kPsdTol = 1e-13;

// ------------------------------------------------------------ covariance
struct Cov {
    int kind;
    double nu, lam, sigma2;
    // Matern, eq. (matern-cov-function); separable exponential,
    // eq. (p-norm-cov-function) with p = 1.
    double operator()(double t1, double t2) const {
        if (kind == CES_COV_SEPEXP) return sigma2 * std::exp(-(std::fabs(t1) + std::fabs(t2)) / lam);
        const double r = std::sqrt(t1 * t1 + t2 * t2);
        const double x = std::sqrt(2.0 * nu) * r / lam;
        if (x == 0.0) return sigma2;
        if (nu == 0.5) return sigma2 * std::exp(-x);
        if (nu == 1.5) return sigma2 * (1.0 + x) * std::exp(-x);
        if (nu == 2.5) return sigma2 * (1.0 + x + x * x / 3.0) * std::exp(-x);
        if (x > 700.0) return 0.0;
        return sigma2 * std::pow(2.0, 1.0 - nu) / std::tgamma(nu) * std::pow(x, nu) * std::cyl_bessel_k(nu, x);
    }
};

double eta(double x) { return x > 0.0 ? std::exp(-1.0 / x) : 0.0; }

// First column of the embedding (Section 2.1.2 mirroring for J = 0; the
// 2 ell-periodic extension of eq. (periodic-cov-fun) for J > 0), n x n,
// index [j2][j1].  Computed on the quadrant j <= n/2 and mirrored (the
// column is even in each index).
std::vector<double> first_column(const Cov& C, int m, int J, int reading) {
    const int n = 2 * (m + J);
    const double h = 1.0 / m;
    const int nh = n / 2;
    std::vector<double> q((size_t)(nh + 1) * (nh + 1));
    if (J == 0) {
        for (int b = 0; b <= nh; ++b)
            for (int a = 0; a <= nh; ++a) q[(size_t)b * (nh + 1) + a] = C(a * h, b * h);
    } else {
        const double ell = 1.0 + (double)J / m;
        const double lo = reading == CES_PERIOD_INF ? 1.0 : std::sqrt(2.0);
        const double kappa = reading == CES_PERIOD_INF ? 2.0 * ell - 1.0 : 2.0 * ell - std::sqrt(2.0);
        const double wdt = kappa - lo;
        auto phi = [&](double t) {
            const double a = eta((kappa - t) / wdt), b = eta((t - lo) / wdt);
            return a / (a + b);
        };
        for (int b = 0; b <= nh; ++b)
            for (int a = 0; a <= nh; ++a) {
                double acc = 0.0;
                for (int s2 = 0; s2 >= -1; --s2)
                    for (int s1 = 0; s1 >= -1; --s1) {
                        const double y1 = a * h + 2.0 * ell * s1, y2 = b * h + 2.0 * ell * s2;
                        const double t = reading == CES_PERIOD_INF ? std::max(std::fabs(y1), std::fabs(y2))
                                                                   : std::sqrt(y1 * y1 + y2 * y2);
                        if (t >= kappa) continue;
                        acc += C(y1, y2) * phi(t);
                    }
                q[(size_t)b * (nh + 1) + a] = acc;
            }
    }
    std::vector<double> s((size_t)n * n);
    for (int j2 = 0; j2 < n; ++j2) {
        const int b = std::min(j2, n - j2);
        for (int j1 = 0; j1 < n; ++j1) {
            const int a = std::min(j1, n - j1);
            s[(size_t)j2 * n + j1] = q[(size_t)b * (nh + 1) + a];
        }
    }
    return s;
}

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

}  // namespace

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int validate(const ces_level_desc* d) {
    if (!d) return fail(CES_ERR_ARG, "desc is NULL");
    if (d->struct_size != (int32_t)sizeof(ces_level_desc)) return fail(CES_ERR_ARG, "desc.struct_size mismatch");
    if (d->cov_kind != CES_COV_MATERN && d->cov_kind != CES_COV_SEPEXP) return fail(CES_ERR_ARG, "cov_kind");
    if (d->cov_kind == CES_COV_MATERN && !(d->nu > 0.0)) return fail(CES_ERR_ARG, "nu must be > 0");
    if (!(d->lambda > 0.0) || !(d->sigma2 > 0.0)) return fail(CES_ERR_ARG, "lambda and sigma2 must be > 0");
    if (!is_pow2(d->m_fine) || d->m_fine < 4 || d->m_fine > 4096)
        return fail(CES_ERR_ARG, "m_fine must be a power of two in [4, 4096]");
    if (d->level_kind != CES_LEVEL_SINGLE && d->level_kind != CES_LEVEL_PAIR) return fail(CES_ERR_ARG, "level_kind");
    if (d->level_kind == CES_LEVEL_PAIR && d->m_fine < 8) return fail(CES_ERR_ARG, "PAIR levels need m_fine >= 8");
    if (d->psd_policy < 0 || d->psd_policy > 2) return fail(CES_ERR_ARG, "psd_policy");
    if (d->periodization != CES_PERIOD_EUCLID && d->periodization != CES_PERIOD_INF) return fail(CES_ERR_ARG, "periodization");
    if (d->max_pad_factor < 2 || d->max_pad_factor > 4) return fail(CES_ERR_ARG, "max_pad_factor must be in [2, 4]");
    if (d->field_mode != CES_FIELD_PAIR && d->field_mode != CES_FIELD_HARTLEY) return fail(CES_ERR_ARG, "field_mode");
    if (d->precision != CES_PREC_FP64 && d->precision != CES_PREC_MIXED) return fail(CES_ERR_ARG, "precision");
    if (d->bc != CES_BC_DIRICHLET0 && d->bc != CES_BC_FLOWCELL) return fail(CES_ERR_ARG, "bc");
    if (d->qoi < CES_QOI_INTEGRAL || d->qoi > CES_QOI_OUTFLUX) return fail(CES_ERR_ARG, "qoi");
    if (d->qoi == CES_QOI_POINT && !(d->qoi_x >= 0 && d->qoi_x <= 1 && d->qoi_y >= 0 && d->qoi_y <= 1))
        return fail(CES_ERR_ARG, "qoi point outside the unit square");
    if (!(d->cg_rtol > 0.0) || d->cg_max_iter < 1) return fail(CES_ERR_ARG, "cg_rtol / cg_max_iter");
    if (d->tau_fine < -1 || d->tau_coarse < -1) return fail(CES_ERR_ARG, "tau must be >= -1");
    return CES_OK;
}

// Orbit symmetrisation: each index takes the value at its representative
// (min(k1, n-k1), min(k2, n-k2)) with the pair sorted.
void symmetrise(std::vector<double>& lam, int n) {
    std::vector<double> out((size_t)n * n);
    for (int k2 = 0; k2 < n; ++k2)
        for (int k1 = 0; k1 < n; ++k1) {
            const int a = std::min(k1, n - k1), b = std::min(k2, n - k2);
            const int lo = std::min(a, b), hi = std::max(a, b);
            out[(size_t)k2 * n + k1] = lam[(size_t)hi * n + lo];
        }
    lam.swap(out);
}

// Device FP64 DFT of the first column -> eigenvalues on the host.
int eigenvalues(const std::vector<double>& s, int n, std::vector<double>& lam, double* imag_max) {
    FftPlan fp = make_fft_plan(n);
    if (fp.nst < 0) return fail(CES_ERR_ARG, "embedding size not of the form 2^a 3^b");
    auto tw = twiddles<double>(n);
    DevBuf ds, dw, dl, dtw, di;
    CES_HIP(ds.alloc(s.size() * 8), "eigen buffers");
    CES_HIP(dw.alloc(s.size() * 16), "eigen buffers");
    CES_HIP(dl.alloc(s.size() * 8), "eigen buffers");
    CES_HIP(dtw.alloc(tw.size() * sizeof(tw[0])), "eigen buffers");
    CES_HIP(di.alloc((size_t)n * 8), "eigen buffers");
    CES_HIP(hipMemcpy(ds.p, s.data(), s.size() * 8, hipMemcpyHostToDevice), "upload column");
    CES_HIP(hipMemcpy(dtw.p, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice), "upload twiddles");
    int nblk = 0;
    CES_HIP(launch_eigen_fft(ds.as<double>(), n, fp, dtw.as<cplx<double>>(), dw.as<cplx<double>>(), dl.as<double>(),
                             di.as<double>(), &nblk, nullptr),
            "eigen DFT launch");
    lam.resize(s.size());
    std::vector<double> im(nblk);
    CES_HIP(hipMemcpy(lam.data(), dl.p, s.size() * 8, hipMemcpyDeviceToHost), "download eigenvalues");
    CES_HIP(hipMemcpy(im.data(), di.p, (size_t)nblk * 8, hipMemcpyDeviceToHost), "download eigenvalues");
    *imag_max = im.empty() ? 0.0 : *std::max_element(im.begin(), im.end());
    return CES_OK;
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

template <typename T>
int upload_amplitudes(ces_plan p) {
    const int n = p->n;
    const size_t s = (size_t)n * n;
    std::vector<T> a(s), c(s);
    for (size_t i = 0; i < s; ++i) {
        const double base = std::sqrt(std::max(p->lam[i], 0.0)) / n;
        a[i] = (T)(p->keep_f[i] ? base : 0.0);
        c[i] = (T)(p->keep_c[i] ? base : 0.0);
    }
    CES_HIP(p->af.alloc(s * sizeof(T)), "amplitude buffers");
    CES_HIP(hipMemcpy(p->af.p, a.data(), s * sizeof(T), hipMemcpyHostToDevice), "upload amplitudes");
    if (p->nf == 2) {
        CES_HIP(p->ac.alloc(s * sizeof(T)), "amplitude buffers");
        CES_HIP(hipMemcpy(p->ac.p, c.data(), s * sizeof(T), hipMemcpyHostToDevice), "upload amplitudes");
    }
    auto tw = twiddles<T>(n);
    CES_HIP(p->tw.alloc(tw.size() * sizeof(tw[0])), "twiddle buffer");
    CES_HIP(hipMemcpy(p->tw.p, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice), "upload twiddles");
    return CES_OK;
}

}  // namespace

extern "C" {

void ces_level_desc_default(ces_level_desc* d) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    d->struct_size = (int32_t)sizeof(ces_level_desc);
    d->cov_kind = CES_COV_MATERN;
    d->nu = 0.5;
    d->lambda = 0.1;
    d->sigma2 = 1.0;
    d->m_fine = 32;
    d->level_kind = CES_LEVEL_SINGLE;
    d->tau_fine = 0;
    d->tau_coarse = 0;
    d->psd_policy = CES_PSD_GROW;
    d->periodization = CES_PERIOD_EUCLID;
    d->max_pad_factor = 4;
    d->field_mode = CES_FIELD_PAIR;
    d->precision = CES_PREC_MIXED;
    d->bc = CES_BC_DIRICHLET0;
    d->qoi = CES_QOI_INTEGRAL;
    d->qoi_x = 7.0 / 15.0;
    d->qoi_y = 7.0 / 15.0;
    d->f_value = 1.0;
    d->cg_rtol = 1e-10;
    d->cg_max_iter = 500;
    d->stream = 0;
}

const char* ces_last_error(void) { return g_err.c_str(); }

int ces_profile_enable(int32_t on) {
    Profiler::get().enable(on != 0);
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
    int rc = validate(desc);
    if (rc != CES_OK) return rc;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    std::unique_ptr<ces_plan_s> p(new ces_plan_s);
    p->ctx = ctx;
    p->d = *desc;
    const int m = desc->m_fine;
    Cov C{desc->cov_kind, desc->nu, desc->lambda, desc->sigma2};
    std::vector<int> cands;
    if (desc->psd_policy == CES_PSD_GROW) {
        for (int J : {0, m / 2, m})
            if (2 * (m + J) <= desc->max_pad_factor * m) cands.push_back(J);
    } else {
        cands.push_back(0);
    }
    bool ok = false;
    for (int J : cands) {
        if (J > 0 && desc->periodization == CES_PERIOD_EUCLID && !(1.0 + (double)J / m > std::sqrt(2.0))) continue;
        const int n = 2 * (m + J);
        if (make_fft_plan(n).nst < 0) continue;
        std::vector<double> s = first_column(C, m, J, desc->periodization);
        std::vector<double> lam;
        double imag = 0.0;
        rc = eigenvalues(s, n, lam, &imag);
        if (rc != CES_OK) return rc;
        symmetrise(lam, n);
        const double lmin = *std::min_element(lam.begin(), lam.end());
        const double lmax = *std::max_element(lam.begin(), lam.end());
        p->n = n;
        p->J = J;
        p->lam_min = lmin;
        p->lam_max = lmax;
        p->lam.swap(lam);
        ok = lmin >= -kPsdTol * lmax;
        if (ok || desc->psd_policy == CES_PSD_CLAMP) break;
    }
    if (p->n == 0) return fail(CES_ERR_ARG, "no admissible embedding size");
    if (!ok && desc->psd_policy != CES_PSD_CLAMP)
        return fail(CES_ERR_NOT_PSD, "embedding has negative eigenvalues up to the padding cap (min/max = " +
                                         std::to_string(p->lam_min / p->lam_max) + ")");
    for (double& v : p->lam)
        if (v < 0.0) {
            v = 0.0;
            ++p->n_clamped;
        }
    const int n = p->n;
    const int64_t s = (int64_t)n * n;
    p->tau_f = desc->tau_fine < 0 ? n : desc->tau_fine;
    p->tau_c = desc->tau_coarse < 0 ? n : desc->tau_coarse;
    if (desc->level_kind == CES_LEVEL_SINGLE) p->tau_c = p->tau_f;
    if (p->tau_f > s || p->tau_c > s) return fail(CES_ERR_ARG, "tau exceeds the number of eigenvalues");
    std::vector<int64_t> order;
    smallest_order(p->lam, std::max(p->tau_f, p->tau_c), order);
    p->keep_f.assign(s, 1);
    p->keep_c.assign(s, 1);
    for (int64_t i = 0; i < p->tau_f; ++i) p->keep_f[order[i]] = 0;
    for (int64_t i = 0; i < p->tau_c; ++i) p->keep_c[order[i]] = 0;
    if (p->tau_c > 0 && p->tau_c < s) {
        // order[tau_c - 1]: largest dropped; smallest kept is the minimum
        // over kept indices (order holds it only when tau_c is the max tau)
        double kept_min = 1e308;
        for (int64_t i = 0; i < s; ++i)
            if (p->keep_c[i]) kept_min = std::min(kept_min, p->lam[i]);
        p->gap = (kept_min - p->lam[order[p->tau_c - 1]]) / std::max(p->lam_max, 1e-300);
    }
    p->is_double = desc->precision == CES_PREC_FP64;
    p->nf = (desc->level_kind == CES_LEVEL_PAIR && p->tau_f != p->tau_c) ? 2 : 1;
    p->fp = make_fft_plan(n);
    rc = p->is_double ? upload_amplitudes<double>(p.get()) : upload_amplitudes<float>(p.get());
    if (rc != CES_OK) return rc;
    *out = p.release();
    return CES_OK;
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
    std::memcpy(host_out, p->lam.data(), p->lam.size() * 8);
    return CES_OK;
}

int ces_plan_mask(ces_plan p, uint8_t* f, uint8_t* c) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    if (f) std::memcpy(f, p->keep_f.data(), p->keep_f.size());
    if (c) std::memcpy(c, p->keep_c.data(), p->keep_c.size());
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
