// Smoothing-parameter rule and smoothing-error statistic (Section 3.5: the
// number of eigenvalues to drop per level from the balance of
// discretisation and smoothing error, eq. (k-values-p-norm-cov) and eq.
// (tau-values-matern); Section 4.1: the smoothing error Q_h - Q~_h of one
// mesh, both terms computed on the same realisation).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.hpp"

using namespace ces;

namespace {

// fields of two descriptors that must agree for a smoothing comparison
// (everything but the drop counts)
bool same_but_tau(const ces_level_desc& a, const ces_level_desc& b) {
    return a.cov_kind == b.cov_kind && a.nu == b.nu && a.lambda == b.lambda && a.sigma2 == b.sigma2 &&
           a.m_fine == b.m_fine && a.level_kind == b.level_kind && a.psd_policy == b.psd_policy &&
           a.periodization == b.periodization && a.max_pad_factor == b.max_pad_factor &&
           a.field_mode == b.field_mode && a.precision == b.precision && a.bc == b.bc && a.qoi == b.qoi &&
           a.qoi_x == b.qoi_x && a.qoi_y == b.qoi_y && a.f_value == b.f_value && a.cg_rtol == b.cg_rtol &&
           a.cg_max_iter == b.cg_max_iter && a.stream == b.stream;
}

}  // namespace

extern "C" {

int ces_tau_rule(int32_t cov_kind, double nu, int32_t m, int32_t J, double alpha, double cs_over_calpha,
                 int64_t* tau, double* tau_real) {
    if (!tau) return fail(CES_ERR_ARG, "tau is NULL");
    if (m < 1 || J < 0) return fail(CES_ERR_ARG, "m >= 1 and J >= 0 required");
    if (!(alpha > 0.0) || !(cs_over_calpha > 0.0) || !std::isfinite(alpha) || !std::isfinite(cs_over_calpha))
        return fail(CES_ERR_ARG, "alpha and C_s / C_alpha must be positive and finite");
    const double h = 1.0 / m;
    const double s = 4.0 * ((double)m + J) * ((double)m + J);   // embedding size n^2, n = 2 (m + J)
    double t = 0.0;
    if (cov_kind == CES_COV_SEPEXP) {
        // C_alpha h^alpha = C_s tau / (s - tau + 1) solved for tau; with the
        // classical embedding (J = 0) h = 2 / sqrt(s) and this is eq.
        // (k-values-p-norm-cov)
        if (J != 0) return fail(CES_ERR_ARG, "the separable exponential rule assumes no padding (J = 0)");
        t = (s + 1.0) / (cs_over_calpha * std::pow(h, -alpha) + 1.0);
    } else if (cov_kind == CES_COV_MATERN) {
        if (!(nu > 0.0)) return fail(CES_ERR_ARG, "nu must be positive");
        // eq. (tau-values-matern): (s - tau + 1)^(-(1+nu)/2) tau = 2 / (C_s / C_alpha) h^(alpha+1) (1/h + J);
        // the left side increases strictly from 0 (tau = 0) to s (tau = s)
        const double rhs = 2.0 / cs_over_calpha * std::pow(h, alpha + 1.0) * (1.0 / h + J);
        const double p = 0.5 * (1.0 + nu);
        auto g = [&](double x) { return std::pow(s - x + 1.0, -p) * x - rhs; };
        if (g(s) <= 0.0) {
            t = s;
        } else {
            double lo = 0.0, hi = s;   // g(lo) < 0 < g(hi)
            for (int it = 0; it < 200 && hi - lo > 1e-12 * std::max(1.0, hi); ++it) {
                const double mid = 0.5 * (lo + hi);
                (g(mid) < 0.0 ? lo : hi) = mid;
            }
            t = 0.5 * (lo + hi);
        }
    } else {
        return fail(CES_ERR_ARG, "cov_kind");
    }
    t = std::min(std::max(t, 0.0), s);
    if (tau_real) *tau_real = t;
    *tau = (int64_t)std::floor(t + 0.5);
    return CES_OK;
}

int ces_smoothing_error(ces_context ctx, ces_plan full, ces_plan smoothed, uint64_t seed, uint64_t first,
                        int64_t count, void* stream, ces_smoothing_stats* out) {
    if (!ctx || !full || !smoothed || !out) return fail(CES_ERR_ARG, "context, plans or out is NULL");
    if (out->struct_size != (int32_t)sizeof(ces_smoothing_stats))
        return fail(CES_ERR_ARG, "out.struct_size mismatch");
    if (full->ctx != ctx || smoothed->ctx != ctx) return fail(CES_ERR_ARG, "plans of another context");
    if (full == smoothed) return fail(CES_ERR_ARG, "the two plans must differ");
    if (count < 2) return fail(CES_ERR_ARG, "count >= 2 required");
    if (full->d.level_kind != CES_LEVEL_SINGLE || smoothed->d.level_kind != CES_LEVEL_SINGLE)
        return fail(CES_ERR_ARG, "both plans must be SINGLE levels");
    if (!same_but_tau(full->d, smoothed->d))
        return fail(CES_ERR_ARG, "the plans must differ only in their drop counts (same mesh, covariance, "
                                 "field mode, precision, PDE data and stream)");
    if (full->n != smoothed->n) return fail(CES_ERR_ARG, "the plans have different embeddings");
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DevBuf y;
    CES_HIP(y.alloc((size_t)count * 16), "study buffers");
    double* yd = y.as<double>();
    ces_request reqs[2] = {
        ces_request{full, seed, first, count, yd, nullptr, nullptr, nullptr, nullptr},
        ces_request{smoothed, seed, first, count, yd + count, nullptr, nullptr, nullptr, nullptr},
    };
    int rc = ces_sample_batch(ctx, reqs, 2, stream);
    if (rc != CES_OK) return rc;
    std::vector<double> h((size_t)count * 2);
    CES_HIP(hipMemcpyAsync(h.data(), yd, h.size() * 8, hipMemcpyDeviceToHost, st), "results");
    CES_HIP(hipStreamSynchronize(st), "results");
    // statistics in sample order: mean and variance by Welford's recurrence
    double mean = 0.0, m2 = 0.0, sabs = 0.0, sq = 0.0, sqs = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const double q = h[i], qs = h[count + i], d = q - qs;
        const double dm = d - mean;
        mean += dm / (double)(i + 1);
        m2 += dm * (d - mean);
        sabs += std::fabs(d);
        sq += q;
        sqs += qs;
    }
    const int32_t sz = out->struct_size;
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sz;
    out->n = count;
    out->mean = mean;
    out->mean_abs = sabs / (double)count;
    out->var = m2 / (double)(count - 1);
    out->mean_q = sq / (double)count;
    out->mean_q_smoothed = sqs / (double)count;
    return CES_OK;
}

}  // extern "C"
