// Randomised quasi-Monte Carlo for the Hartley sampler (the multilevel QMC
// extension named in Section 5; the real factorisation of Sections
// 2.1.1-2.1.2 is what QMC drives): CBC generating vectors, lattice
// attachment to plans, and the multilevel QMC estimator of Giles and
// Waterhouse (2009) on top of the batch sampler.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "plan.hpp"

using namespace ces;

namespace {

// The CBC criterion's terms are truncated to multiples of 2^-kFracBits and
// added exactly (128-bit), so a candidate's score does not depend on how
// the sum is split over threads.
constexpr int kFracBits = 40;

// B2 table and the weighted factor 1 + gamma B2(a / N), a = 0..N-1
void factor_table(int N, double g, std::vector<double>& f) {
#pragma clang fp contract(off)
    f.resize(N);
    for (int a = 0; a < N; ++a) {
        const double x = (double)a / (double)N;
        const double b2 = x * (x - 1.0) + (1.0 / 6.0);
        f[a] = 1.0 + g * b2;
    }
}

unsigned __int128 score(const std::vector<double>& P, const std::vector<double>& f, uint32_t c, int N) {
#pragma clang fp contract(off)
    unsigned __int128 s = 0;
    const uint32_t mask = (uint32_t)N - 1;
    for (int k = 0; k < N; ++k) {
        const double t = P[k] * f[((uint32_t)k * c) & mask];
        s += (uint64_t)std::floor(std::ldexp(t, kFracBits));
    }
    return s;
}

int threads_for(size_t work) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t by_work = std::max<size_t>(1, work / (1u << 20));
    return (int)std::min<size_t>(std::min<size_t>(hw, 16), by_work);
}

// running per-shift sums of one level (samples added in index order)
struct ShiftSums {
    std::vector<double> s;
    int64_t pts = 0;
    void reset(int R) {
        s.assign(R, 0.0);
        pts = 0;
    }
    // mean of the shift averages and their sample variance (R - 1)
    void stats(double* mu, double* var) const {
        const int R = (int)s.size();
        std::vector<double> m(R);
        double t = 0.0;
        for (int r = 0; r < R; ++r) {
            m[r] = s[r] / (double)pts;
            t += m[r];
        }
        const double mean = t / (double)R;
        double v = 0.0;
        for (int r = 0; r < R; ++r) v += (m[r] - mean) * (m[r] - mean);
        *mu = mean;
        *var = v / (double)(R - 1);
    }
};

double slope(const std::vector<int>& idx, const std::vector<double>& v) {
    const double n = (double)idx.size();
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (size_t k = 0; k < idx.size(); ++k) {
        sx += idx[k];
        sy += v[k];
        sxx += (double)idx[k] * idx[k];
        sxy += idx[k] * v[k];
    }
    const double den = n * sxx - sx * sx;
    return den != 0.0 ? (n * sxy - sx * sy) / den : 0.0;
}

double unknowns(const ces_level_desc& d, int m) {
    const double rows = d.bc == CES_BC_FLOWCELL ? m + 1 : m - 1;
    return (double)(m - 1) * rows;
}

int eigen_order(ces_plan p, int32_t s, std::vector<int64_t>& dims, std::vector<double>& lam_sel) {
    if (!p->lam.p) return fail(CES_ERR_ARG, "plan kept no eigenvalues");
    const int64_t ns = (int64_t)p->n * p->n;
    if (s < 1 || s > ns) return fail(CES_ERR_ARG, "s must be in 1..n^2");
    std::vector<double> lam(ns);
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    CES_HIP(hipMemcpy(lam.data(), p->lam.p, (size_t)ns * 8, hipMemcpyDeviceToHost), "download eigenvalues");
    for (double& v : lam) v = std::max(v, 0.0);
    std::vector<int64_t> idx(ns);
    std::iota(idx.begin(), idx.end(), 0);
    auto before = [&](int64_t a, int64_t b) {
        if (lam[a] != lam[b]) return lam[a] > lam[b];
        return a < b;
    };
    std::partial_sort(idx.begin(), idx.begin() + s, idx.end(), before);
    dims.assign(idx.begin(), idx.begin() + s);
    lam_sel.resize(s);
    for (int32_t j = 0; j < s; ++j) lam_sel[j] = lam[dims[j]];
    return CES_OK;
}

}  // namespace

extern "C" {

int ces_lattice_cbc(int32_t log2_points, int32_t s, const double* gamma, uint32_t* z) {
    if (!gamma || !z) return fail(CES_ERR_ARG, "gamma or z is NULL");
    if (log2_points < 0 || log2_points > 20 || s < 1) return fail(CES_ERR_ARG, "need 0 <= log2_points <= 20, s >= 1");
    double gsum = 0.0;
    for (int32_t j = 0; j < s; ++j) {
        if (!(gamma[j] >= 0.0) || !std::isfinite(gamma[j])) return fail(CES_ERR_ARG, "weights must be finite and >= 0");
        gsum += gamma[j];
    }
    // every term is below exp(sum gamma / 6) < 2^16, so t 2^40 fits 64 bits
    if (gsum > 64.0) return fail(CES_ERR_ARG, "the weights must sum to at most 64");
    const int N = 1 << log2_points;
    std::vector<uint32_t> cand;
    if (N <= 2) cand.push_back(1);
    else
        for (uint32_t c = 1; c <= (uint32_t)N / 2; c += 2) cand.push_back(c);
    std::vector<double> P(N, 1.0), f;
    const int nt = threads_for((size_t)N * cand.size());
    for (int32_t j = 0; j < s; ++j) {
        factor_table(N, gamma[j], f);
        // each thread scores a contiguous block of candidates; blocks are
        // combined in candidate order, so ties go to the smaller z
        std::vector<unsigned __int128> best_s(nt);
        std::vector<size_t> best_i(nt, SIZE_MAX);
        auto work = [&](int t) {
            const size_t lo = cand.size() * t / nt, hi = cand.size() * (t + 1) / nt;
            for (size_t i = lo; i < hi; ++i) {
                const unsigned __int128 v = score(P, f, cand[i], N);
                if (best_i[t] == SIZE_MAX || v < best_s[t]) {
                    best_s[t] = v;
                    best_i[t] = i;
                }
            }
        };
        if (nt == 1) {
            work(0);
        } else {
            std::vector<std::thread> th;
            for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
            for (auto& x : th) x.join();
        }
        size_t bi = SIZE_MAX;
        unsigned __int128 bs = 0;
        for (int t = 0; t < nt; ++t)
            if (best_i[t] != SIZE_MAX && (bi == SIZE_MAX || best_s[t] < bs)) {
                bs = best_s[t];
                bi = best_i[t];
            }
        z[j] = cand[bi];
        {
#pragma clang fp contract(off)
            const uint32_t mask = (uint32_t)N - 1;
            for (int k = 0; k < N; ++k) P[k] = P[k] * f[((uint32_t)k * z[j]) & mask];
        }
    }
    return CES_OK;
}

int ces_plan_lattice_order(ces_plan p, int32_t s, int64_t* dims, double* lam) {
    if (!p || !dims) return fail(CES_ERR_ARG, "plan or dims is NULL");
    std::vector<int64_t> d;
    std::vector<double> l;
    const int rc = eigen_order(p, s, d, l);
    if (rc != CES_OK) return rc;
    std::copy(d.begin(), d.end(), dims);
    if (lam) std::copy(l.begin(), l.end(), lam);
    return CES_OK;
}

int ces_plan_set_lattice(ces_plan p, int32_t s, const uint32_t* z, const int64_t* dims, int32_t shifts) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    int busy = 0;
    if (!p->busy.compare_exchange_strong(busy, 1)) return fail(CES_ERR_BUSY, "plan is in use by another call");
    struct Release {
        ces_plan p;
        ~Release() { p->busy.store(0); }
    } release{p};
    if (s == 0) {
        // earlier sampling on the plan may still read the tables
        CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
        CES_HIP(hipDeviceSynchronize(), "lattice detach");
        p->q_s = 0;
        p->q_shifts = 0;
        p->q_z.reset();
        p->q_rank.reset();
        return CES_OK;
    }
    if (p->d.field_mode != CES_FIELD_HARTLEY) return fail(CES_ERR_ARG, "a lattice needs the HARTLEY field mode");
    const int64_t ns = (int64_t)p->n * p->n;
    if (s < 0 || s > ns) return fail(CES_ERR_ARG, "s must be in 0..n^2");
    if (!z) return fail(CES_ERR_ARG, "z is NULL");
    if (shifts < 2) return fail(CES_ERR_ARG, "shifts must be >= 2");
    std::vector<int64_t> d;
    if (dims) {
        d.assign(dims, dims + s);
    } else {
        std::vector<double> l;
        const int rc = eigen_order(p, s, d, l);
        if (rc != CES_OK) return rc;
    }
    std::vector<int32_t> rank(ns, -1);
    for (int32_t j = 0; j < s; ++j) {
        if (d[j] < 0 || d[j] >= ns) return fail(CES_ERR_ARG, "dims entry out of [0, n^2)");
        if (rank[d[j]] >= 0) return fail(CES_ERR_ARG, "dims entries must be distinct");
        rank[d[j]] = j;
    }
    CES_HIP(hipSetDevice(p->ctx->device), "hipSetDevice");
    DevBuf zb, rb;
    CES_HIP(zb.alloc((size_t)s * 4, p->alloc), "lattice buffers");
    CES_HIP(rb.alloc((size_t)ns * 4, p->alloc), "lattice buffers");
    CES_HIP(hipMemcpy(zb.p, z, (size_t)s * 4, hipMemcpyHostToDevice), "upload lattice");
    CES_HIP(hipMemcpy(rb.p, rank.data(), (size_t)ns * 4, hipMemcpyHostToDevice), "upload lattice");
    // earlier sampling on the plan may still read the old tables
    CES_HIP(hipDeviceSynchronize(), "lattice swap");
    std::swap(p->q_z.p, zb.p);
    std::swap(p->q_z.bytes, zb.bytes);
    std::swap(p->q_z.a, zb.a);
    std::swap(p->q_rank.p, rb.p);
    std::swap(p->q_rank.bytes, rb.bytes);
    std::swap(p->q_rank.a, rb.a);
    p->q_s = s;
    p->q_shifts = shifts;
    return CES_OK;
}

int ces_plan_set_lattice_default(ces_plan p, int32_t s, int32_t log2_points, int32_t shifts) {
    if (!p) return fail(CES_ERR_ARG, "plan is NULL");
    if (p->d.field_mode != CES_FIELD_HARTLEY) return fail(CES_ERR_ARG, "a lattice needs the HARTLEY field mode");
    std::vector<int64_t> d;
    std::vector<double> lam;
    int rc = eigen_order(p, s, d, lam);
    if (rc != CES_OK) return rc;
    double t = 0.0;
    for (double v : lam) t += v;
    std::vector<double> g(s);
    for (int32_t j = 0; j < s; ++j) g[j] = t > 0.0 ? lam[j] / t : 1.0 / (double)s;
    std::vector<uint32_t> z(s);
    if ((rc = ces_lattice_cbc(log2_points, s, g.data(), z.data())) != CES_OK) return rc;
    return ces_plan_set_lattice(p, s, z.data(), d.data(), shifts);
}

void ces_mlqmc_opts_default(ces_mlqmc_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = (int32_t)sizeof(ces_mlqmc_opts);
    o->l_start = 2;
    o->eps = 1e-3;
    o->n_pilot = 1;
    o->theta = 0.5;
    o->alpha = 0.0;
    o->cost_model = 0;
    o->max_rounds = 50;
    o->seed = 0;
}

int ces_mlqmc_run(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                  const ces_mlqmc_opts* o, void* stream, ces_mlmc_result* out) {
    if (!ctx || !levels || !o || !out) return fail(CES_ERR_ARG, "context, levels, opts or out is NULL");
    if (o->struct_size != (int32_t)sizeof(ces_mlqmc_opts)) return fail(CES_ERR_ARG, "opts.struct_size mismatch");
    if (nlevels < 1 || nlevels > CES_MLMC_MAX_LEVELS) return fail(CES_ERR_ARG, "nlevels must be in 1..16");
    if (!(o->eps > 0.0) || !(o->theta > 0.0 && o->theta < 1.0) || o->n_pilot < 1 || o->l_start < 0 ||
        o->max_rounds < 1)
        return fail(CES_ERR_ARG, "eps > 0, 0 < theta < 1, n_pilot >= 1, l_start >= 0, max_rounds >= 1");
    const int R = levels[0] ? levels[0]->q_shifts : 0;
    for (int l = 0; l < nlevels; ++l) {
        for (int f = 0; f < (finest ? 2 : 1); ++f) {
            const ces_plan p = f ? finest[l] : levels[l];
            if (!p || p->ctx != ctx) return fail(CES_ERR_ARG, "level plan missing or of another context");
            const int want = l == 0 ? CES_LEVEL_SINGLE : CES_LEVEL_PAIR;
            if (p->d.level_kind != want) return fail(CES_ERR_ARG, "level 0 must be SINGLE and levels >= 1 PAIR");
            if (p->q_s <= 0 || p->q_shifts != R) return fail(CES_ERR_ARG, "every plan needs a lattice, one shift count");
        }
        if (l > 0 && levels[l]->d.m_fine != 2 * levels[l - 1]->d.m_fine)
            return fail(CES_ERR_ARG, "level l must halve the mesh of level l-1");
    }
    if (int rc = check_level_tags(levels, finest, nlevels); rc != CES_OK) return rc;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::memset(out, 0, sizeof(*out));

    int L = std::min(o->l_start, nlevels - 1);
    std::vector<ShiftSums> S(nlevels);
    for (auto& x : S) x.reset(R);
    std::vector<int64_t> want(nlevels, 0);
    std::vector<double> cost(nlevels, 0.0);
    for (int l = 0; l <= L; ++l) want[l] = o->n_pilot;
    auto plan_of = [&](int l) { return (finest && l == L) ? finest[l] : levels[l]; };
    for (int l = 0; l < nlevels; ++l) {
        const ces_level_desc& d = levels[l]->d;
        cost[l] = unknowns(d, d.m_fine) + (l > 0 ? unknowns(d, d.m_fine / 2) : 0.0);
    }
    DevBuf ydev;
    std::vector<double> yh;
    double alpha = o->alpha, beta = 0.0, gamma = 0.0, bias = 0.0;
    bool converged = false;
    int rounds = 0;
    std::vector<double> mu(nlevels, 0.0), var(nlevels, 0.0);
    while (rounds < o->max_rounds) {
        // the new points of every shift, every level in one batch
        std::vector<ces_request> reqs;
        std::vector<int> lv;
        int64_t total = 0;
        for (int l = 0; l <= L; ++l)
            if (want[l] > S[l].pts) total += (want[l] - S[l].pts) * R;
        if (total > 0) {
            if (ydev.bytes < (size_t)total * 8) CES_HIP(ydev.alloc((size_t)total * 8), "estimator buffers");
            int64_t off = 0;
            for (int l = 0; l <= L; ++l) {
                const int64_t c = (want[l] - S[l].pts) * R;
                if (c <= 0) continue;
                reqs.push_back(ces_request{plan_of(l), o->seed, (uint64_t)(S[l].pts * R), c, ydev.as<double>() + off,
                                           nullptr, nullptr, nullptr, nullptr});
                lv.push_back(l);
                off += c;
            }
            std::vector<double> secs(reqs.size(), 0.0);
            if (o->cost_model == 1) {
                for (size_t i = 0; i < reqs.size(); ++i) {
                    CES_HIP(hipStreamSynchronize(st), "estimator sync");
                    const auto t0 = std::chrono::steady_clock::now();
                    int rc = ces_sample_batch(ctx, &reqs[i], 1, stream);
                    if (rc != CES_OK) return rc;
                    CES_HIP(hipStreamSynchronize(st), "estimator sync");
                    secs[i] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                }
            } else {
                int rc = ces_sample_batch(ctx, reqs.data(), (int32_t)reqs.size(), stream);
                if (rc != CES_OK) return rc;
            }
            yh.resize(total);
            CES_HIP(hipMemcpyAsync(yh.data(), ydev.p, (size_t)total * 8, hipMemcpyDeviceToHost, st), "results");
            CES_HIP(hipStreamSynchronize(st), "results");
            int64_t k = 0;
            for (size_t i = 0; i < reqs.size(); ++i) {
                const int l = lv[i];
                const uint64_t first = reqs[i].first_sample;
                for (int64_t t = 0; t < reqs[i].count; ++t) S[l].s[(first + (uint64_t)t) % (uint64_t)R] += yh[k++];
                S[l].pts = want[l];
                if (o->cost_model == 1) cost[l] = secs[i] / (double)reqs[i].count;
            }
        }
        ++rounds;
        for (int l = 0; l <= L; ++l) S[l].stats(&mu[l], &var[l]);
        // doublings planned with the Monte Carlo rate (V_l halves)
        std::vector<double> proj(L + 1);
        std::vector<int64_t> np(L + 1);
        double tot = 0.0;
        for (int l = 0; l <= L; ++l) {
            proj[l] = var[l] / (double)R;
            np[l] = S[l].pts;
            tot += proj[l];
        }
        while (tot > o->theta * o->eps * o->eps) {
            int ls = 0;
            double br = -1.0;
            for (int l = 0; l <= L; ++l) {
                const double r = proj[l] / (cost[l] * (double)np[l]);
                if (r > br) {
                    br = r;
                    ls = l;
                }
            }
            np[ls] *= 2;
            proj[ls] /= 2.0;
            tot = 0.0;
            for (int l = 0; l <= L; ++l) tot += proj[l];
        }
        bool more = false;
        for (int l = 0; l <= L; ++l) {
            want[l] = np[l];
            more = more || want[l] > S[l].pts;
        }
        std::vector<int> idx;
        std::vector<double> lm, lv2, lc;
        for (int l = 1; l <= L; ++l) {
            idx.push_back(l);
            lm.push_back(std::log2(std::max(std::fabs(mu[l]), 1e-300)));
            lv2.push_back(std::log2(std::max(var[l], 1e-300)));
            lc.push_back(std::log2(cost[l]));
        }
        if (idx.size() >= 2) {
            if (o->alpha <= 0.0) alpha = std::max(0.5, -slope(idx, lm));
            beta = -slope(idx, lv2);
            gamma = slope(idx, lc);
        } else if (o->alpha <= 0.0) {
            alpha = 1.0;
        }
        bias = L >= 1 ? std::fabs(mu[L]) / (std::pow(2.0, alpha) - 1.0) : 0.0;
        if (more) continue;
        if (L >= 1 && bias * bias <= (1.0 - o->theta) * o->eps * o->eps) {
            converged = true;
            break;
        }
        // a level is only added when a round is left to sample it
        if (L + 1 >= nlevels || rounds >= o->max_rounds) break;
        if (finest && finest[L] != levels[L]) {
            S[L].reset(R);
            want[L] = o->n_pilot;
        }
        ++L;
        want[L] = o->n_pilot;
    }
    out->estimate = 0.0;
    out->variance = 0.0;
    for (int l = 0; l <= L; ++l) {
        out->estimate += mu[l];
        out->variance += var[l] / (double)R;
        out->n[l] = S[l].pts * R;
        out->mean[l] = mu[l];
        out->var[l] = var[l];
        out->cost[l] = cost[l];
    }
    out->bias = bias;
    out->alpha = alpha;
    out->beta = beta;
    out->gamma = gamma;
    out->levels = L + 1;
    out->converged = converged ? 1 : 0;
    out->rounds = rounds;
    return CES_OK;
}

}  // extern "C"
