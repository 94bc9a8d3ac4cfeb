// Adaptive MLMC estimator on top of the batch sampler (Section 3.3: the
// estimator eq. (mlmc-estimator) and its smoothed form eq.
// (mlmc-estimator-smoothed), the sample sizes of eq. (optimal-nl); Section
// 4: Richardson extrapolation for the bias and rate fits on a log scale;
// Section 3.5: the coarsest-mesh rules).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace ces;

namespace {

// running mean and variance of one level's Y, samples added in index order
struct Welford {
    int64_t n = 0;
    double mean = 0.0, m2 = 0.0;
    void add(double y) {
        ++n;
        const double d = y - mean;
        mean += d / (double)n;
        m2 += d * (y - mean);
    }
    double var() const { return n > 1 ? m2 / (double)(n - 1) : 0.0; }
};

// least-squares slope of v[i] against i over the given indices
double slope(const std::vector<int>& idx, const std::vector<double>& v) {
    const double n = (double)idx.size();
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (size_t k = 0; k < idx.size(); ++k) {
        const double x = idx[k], y = v[k];
        sx += x;
        sy += y;
        sxx += x * x;
        sxy += x * y;
    }
    const double den = n * sxx - sx * sx;
    return den != 0.0 ? (n * sxy - sx * sy) / den : 0.0;
}

double unknowns(const ces_level_desc& d, int m) {
    const double rows = d.bc == CES_BC_FLOWCELL ? m + 1 : m - 1;
    return (double)(m - 1) * rows;
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    return h;
}

// identifies a run for its checkpoint: the options that shape its rounds
// (not max_rounds, which a resumed call may raise) and every level's plans
uint64_t run_key(const ces_plan* levels, const ces_plan* finest, int nlevels, const ces_mlmc_opts* o) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &nlevels, sizeof(nlevels));
    for (const void* v : {(const void*)&o->eps, (const void*)&o->theta, (const void*)&o->alpha})
        h = fnv1a(h, v, sizeof(double));
    h = fnv1a(h, &o->l_start, sizeof(o->l_start));
    h = fnv1a(h, &o->n_pilot, sizeof(o->n_pilot));
    h = fnv1a(h, &o->cost_model, sizeof(o->cost_model));
    h = fnv1a(h, &o->seed, sizeof(o->seed));
    for (int l = 0; l < nlevels; ++l) {
        h = fnv1a(h, &levels[l]->d, sizeof(ces_level_desc));
        const int fl = finest ? 1 : 0;
        h = fnv1a(h, &fl, sizeof(fl));
        if (finest) h = fnv1a(h, &finest[l]->d, sizeof(ces_level_desc));
    }
    return h;
}

// The estimator between rounds: enough to continue it bit for bit.
struct RunState {
    int L = 0, rounds = 0;
    bool done = false, converged = false;
    std::vector<Welford> W;
    std::vector<int64_t> want, next;
    std::vector<double> cost;
    double alpha = 0.0, beta = 0.0, gamma = 0.0, bias = 0.0, varsum = 0.0;

    void init(int nlevels, const ces_mlmc_opts* o, const ces_plan* levels) {
        L = std::min(o->l_start, nlevels - 1);
        W.assign(nlevels, Welford());
        want.assign(nlevels, 0);
        next.assign(nlevels, 0);
        cost.assign(nlevels, 0.0);
        for (int l = 0; l <= L; ++l) want[l] = o->n_pilot;
        for (int l = 0; l < nlevels; ++l) {
            const ces_level_desc& d = levels[l]->d;
            cost[l] = unknowns(d, d.m_fine) + (l > 0 ? unknowns(d, d.m_fine / 2) : 0.0);
        }
        alpha = o->alpha;
    }

    // after a round's samples: sample sizes, rates, bias, and whether to
    // stop or add a level
    void decide(const ces_mlmc_opts* o, int nlevels, const ces_plan* finest, const ces_plan* levels) {
        // sample sizes, eq. (optimal-nl) with the variance budget theta eps^2
        double acc = 0.0;
        for (int l = 0; l <= L; ++l) acc += std::sqrt(W[l].var() * cost[l]);
        bool more = false;
        for (int l = 0; l <= L; ++l) {
            const double v = W[l].var();
            const int64_t nl = (int64_t)std::ceil(acc * std::sqrt(v / cost[l]) / (o->theta * o->eps * o->eps));
            want[l] = std::max<int64_t>(std::max<int64_t>(nl, 2), W[l].n);
            more = more || want[l] > W[l].n;
        }
        // rates over levels 1..L (log2 of the quantity against l)
        std::vector<int> idx;
        std::vector<double> lm, lv2, lc;
        for (int l = 1; l <= L; ++l) {
            idx.push_back(l);
            lm.push_back(std::log2(std::max(std::fabs(W[l].mean), 1e-300)));
            lv2.push_back(std::log2(std::max(W[l].var(), 1e-300)));
            lc.push_back(std::log2(cost[l]));
        }
        if (idx.size() >= 2) {
            if (o->alpha <= 0.0) alpha = std::max(0.5, -slope(idx, lm));
            beta = -slope(idx, lv2);
            gamma = slope(idx, lc);
        } else if (o->alpha <= 0.0) {
            alpha = 1.0;
        }
        varsum = 0.0;
        for (int l = 0; l <= L; ++l) varsum += W[l].var() / (double)W[l].n;
        // Richardson extrapolation with extrapolant Q_2h (Section 4)
        bias = L >= 1 ? std::fabs(W[L].mean) / (std::pow(2.0, alpha) - 1.0) : 0.0;
        if (more) return;
        if (L >= 1 && bias * bias <= (1.0 - o->theta) * o->eps * o->eps) {
            converged = done = true;
            return;
        }
        // a level is added only when a round is left to sample it, so that
        // every level of the result has samples
        if (L + 1 >= nlevels || rounds >= o->max_rounds) {
            done = true;
            return;
        }
        // add a level; the old finest level changes plan if finest plans differ
        if (finest && finest[L] != levels[L]) {
            W[L] = Welford();
            next[L] = 0;
            want[L] = o->n_pilot;
        }
        ++L;
        want[L] = o->n_pilot;
    }

    void fill(ces_mlmc_result* out) const {
        out->estimate = 0.0;
        for (int l = 0; l <= L; ++l) out->estimate += W[l].mean;
        out->variance = varsum;
        out->bias = bias;
        out->alpha = alpha;
        out->beta = beta;
        out->gamma = gamma;
        out->levels = L + 1;
        out->converged = converged ? 1 : 0;
        out->rounds = rounds;
        for (int l = 0; l <= L; ++l) {
            out->n[l] = W[l].n;
            out->mean[l] = W[l].mean;
            out->var[l] = W[l].var();
            out->cost[l] = cost[l];
        }
    }

    // JSON, doubles with 17 significant digits (they read back exactly);
    // written to path.tmp and renamed over path
    int save(const char* path, uint64_t key) const {
        const std::string tmp = std::string(path) + ".tmp";
        FILE* f = std::fopen(tmp.c_str(), "w");
        if (!f) return fail(CES_ERR_ARG, std::string("cannot write checkpoint ") + tmp);
        std::fprintf(f, "{\n  \"format\": \"cesmlmc-mlmc-checkpoint\", \"version\": 1,\n");
        std::fprintf(f, "  \"key\": \"%016llx\",\n", (unsigned long long)key);
        std::fprintf(f, "  \"nlevels\": %d, \"L\": %d, \"rounds\": %d, \"done\": %d, \"converged\": %d,\n",
                     (int)W.size(), L, rounds, done ? 1 : 0, converged ? 1 : 0);
        std::fprintf(f, "  \"alpha\": %.17g, \"beta\": %.17g, \"gamma\": %.17g, \"bias\": %.17g, \"varsum\": %.17g,\n",
                     alpha, beta, gamma, bias, varsum);
        std::fprintf(f, "  \"levels\": [\n");
        for (size_t l = 0; l < W.size(); ++l)
            std::fprintf(f, "    {\"n\": %lld, \"mean\": %.17g, \"m2\": %.17g, \"want\": %lld, \"next\": %lld, \"cost\": %.17g}%s\n",
                         (long long)W[l].n, W[l].mean, W[l].m2, (long long)want[l], (long long)next[l], cost[l],
                         l + 1 < W.size() ? "," : "");
        std::fprintf(f, "  ]\n}\n");
        const bool ok = std::fflush(f) == 0;
        std::fclose(f);
        if (!ok || std::rename(tmp.c_str(), path) != 0)
            return fail(CES_ERR_ARG, std::string("cannot write checkpoint ") + path);
        return CES_OK;
    }

    // a missing file starts the run afresh
    int load(const char* path, uint64_t key) {
        FILE* f = std::fopen(path, "r");
        if (!f) return CES_OK;
        std::string text;
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
        std::fclose(f);
        size_t pos = 0;
        bool ok = true;
        auto field = [&](const char* name) -> const char* {
            const std::string k = std::string("\"") + name + "\":";
            const size_t at = text.find(k, pos);
            if (at == std::string::npos) {
                ok = false;
                return nullptr;
            }
            pos = at + k.size();
            while (pos < text.size() && (text[pos] == ' ' || text[pos] == '"')) ++pos;
            return text.c_str() + pos;
        };
        auto num = [&](const char* name) -> double {
            const char* p = field(name);
            return p ? std::strtod(p, nullptr) : 0.0;
        };
        auto inum = [&](const char* name) -> long long {
            const char* p = field(name);
            return p ? std::strtoll(p, nullptr, 10) : 0;
        };
        const char* kp = field("key");
        if (!ok || std::strtoull(kp, nullptr, 16) != key)
            return fail(CES_ERR_ARG, std::string("checkpoint ") + path + " belongs to another run");
        const long long nl = inum("nlevels");
        if (!ok || nl != (long long)W.size()) return fail(CES_ERR_ARG, "checkpoint level count differs");
        L = (int)inum("L");
        rounds = (int)inum("rounds");
        done = inum("done") != 0;
        converged = inum("converged") != 0;
        alpha = num("alpha");
        beta = num("beta");
        gamma = num("gamma");
        bias = num("bias");
        varsum = num("varsum");
        for (size_t l = 0; l < W.size(); ++l) {
            W[l].n = inum("n");
            W[l].mean = num("mean");
            W[l].m2 = num("m2");
            want[l] = inum("want");
            next[l] = inum("next");
            cost[l] = num("cost");
        }
        if (!ok || L < 0 || L >= (int)W.size() || rounds < 0)
            return fail(CES_ERR_ARG, std::string("checkpoint ") + path + " is malformed");
        return CES_OK;
    }
};

}  // namespace

int ces::check_level_tags(const ces_plan* levels, const ces_plan* finest, int nlevels) {
    auto tags = [&](int l, uint32_t* t) {
        t[0] = levels[l]->d.stream;
        t[1] = finest ? finest[l]->d.stream : t[0];
    };
    for (int l = 0; l < nlevels; ++l)
        for (int k = l + 1; k < nlevels; ++k) {
            uint32_t a[2], b[2];
            tags(l, a);
            tags(k, b);
            for (uint32_t x : a)
                for (uint32_t y : b)
                    if (x == y)
                        return fail(CES_ERR_ARG, "levels " + std::to_string(l) + " and " + std::to_string(k) +
                                                     " share the level tag (stream) " + std::to_string(x) +
                                                     ": their normals would coincide");
        }
    return CES_OK;
}

extern "C" {

void ces_mlmc_opts_default(ces_mlmc_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = (int32_t)sizeof(ces_mlmc_opts);
    o->eps = 1e-3;
    o->l_start = 2;
    o->n_pilot = 100;
    o->theta = 0.5;
    o->alpha = 0.0;
    o->cost_model = 0;
    o->max_rounds = 50;
    o->seed = 0;
}

int ces_mlmc_coarsest_mesh(const ces_level_desc* d, int32_t* m0) {
    if (!d || !m0) return fail(CES_ERR_ARG, "desc or m0 is NULL");
    const double hmax = d->cov_kind == CES_COV_SEPEXP ? d->lambda : std::sqrt(8.0 * d->nu) * d->lambda;
    int m = 1;
    while (1.0 / m > hmax && m < (1 << 20)) m *= 2;
    *m0 = m;
    return CES_OK;
}

int ces_mlmc_run(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                 const ces_mlmc_opts* o, void* stream, ces_mlmc_result* out) {
    return ces_mlmc_run_checkpointed(ctx, levels, finest, nlevels, o, nullptr, 0, stream, out);
}

int ces_mlmc_run_checkpointed(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                              const ces_mlmc_opts* o, const char* path, int32_t max_new_rounds, void* stream,
                              ces_mlmc_result* out) {
    if (!ctx || !levels || !o || !out) return fail(CES_ERR_ARG, "context, levels, opts or out is NULL");
    if (o->struct_size != (int32_t)sizeof(ces_mlmc_opts)) return fail(CES_ERR_ARG, "opts.struct_size mismatch");
    if (nlevels < 1 || nlevels > CES_MLMC_MAX_LEVELS) return fail(CES_ERR_ARG, "nlevels must be in 1..16");
    if (!(o->eps > 0.0) || !(o->theta > 0.0 && o->theta < 1.0) || o->n_pilot < 2 || o->l_start < 0 ||
        o->max_rounds < 1)
        return fail(CES_ERR_ARG, "eps > 0, 0 < theta < 1, n_pilot >= 2, l_start >= 0, max_rounds >= 1");
    if (max_new_rounds < 0) return fail(CES_ERR_ARG, "max_new_rounds must be >= 0");
    for (int l = 0; l < nlevels; ++l) {
        const ces_plan p = levels[l];
        if (!p || p->ctx != ctx) return fail(CES_ERR_ARG, "level plan missing or of another context");
        if (finest && (!finest[l] || finest[l]->ctx != ctx)) return fail(CES_ERR_ARG, "finest plan missing");
        const int want = l == 0 ? CES_LEVEL_SINGLE : CES_LEVEL_PAIR;
        if (p->d.level_kind != want || (finest && finest[l]->d.level_kind != want))
            return fail(CES_ERR_ARG, "level 0 must be SINGLE and levels >= 1 PAIR");
        if (l > 0 && p->d.m_fine != 2 * levels[l - 1]->d.m_fine)
            return fail(CES_ERR_ARG, "level l must halve the mesh of level l-1");
    }
    if (int rc = check_level_tags(levels, finest, nlevels); rc != CES_OK) return rc;
    CES_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::memset(out, 0, sizeof(*out));

    RunState S;
    S.init(nlevels, o, levels);
    const uint64_t key = run_key(levels, finest, nlevels, o);
    if (path && *path) {
        int rc = S.load(path, key);
        if (rc != CES_OK) return rc;
    }
    int& L = S.L;
    std::vector<Welford>& W = S.W;
    std::vector<int64_t>&want = S.want, &next_index = S.next;
    std::vector<double>& cost = S.cost;
    auto plan_of = [&](int l) { return (finest && l == L) ? finest[l] : levels[l]; };
    DevBuf ydev;
    std::vector<double> yh;
    int new_rounds = 0;
    while (!S.done && S.rounds < o->max_rounds && (max_new_rounds == 0 || new_rounds < max_new_rounds)) {
        // sample what is missing, every level in one batch
        std::vector<ces_request> reqs;
        std::vector<int> lv;
        int64_t total = 0;
        for (int l = 0; l <= L; ++l)
            if (want[l] > W[l].n) total += want[l] - W[l].n;
        if (total > 0) {
            if (ydev.bytes < (size_t)total * 8) CES_HIP(ydev.alloc((size_t)total * 8), "estimator buffers");
            int64_t off = 0;
            for (int l = 0; l <= L; ++l) {
                const int64_t c = want[l] - W[l].n;
                if (c <= 0) continue;
                reqs.push_back(ces_request{plan_of(l), o->seed, (uint64_t)next_index[l], c,
                                           ydev.as<double>() + off, nullptr, nullptr, nullptr, nullptr});
                lv.push_back(l);
                off += c;
            }
            std::vector<double> secs(reqs.size(), 0.0);
            if (o->cost_model == 1) {
                // measured: each level's share of the round timed alone
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
                for (int64_t j = 0; j < reqs[i].count; ++j) W[l].add(yh[k++]);
                next_index[l] += reqs[i].count;
                if (o->cost_model == 1) cost[l] = secs[i] / (double)reqs[i].count;
            }
        }
        ++S.rounds;
        ++new_rounds;
        S.decide(o, nlevels, finest, levels);
        if (path && *path) {
            int rc = S.save(path, key);
            if (rc != CES_OK) return rc;
        }
    }
    S.fill(out);
    return CES_OK;
}

}  // extern "C"
