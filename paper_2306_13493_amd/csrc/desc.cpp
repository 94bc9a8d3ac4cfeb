// Level descriptors (defaults and validation) and error reporting of the
// C ABI: host code only, shared by the plan set-up, the sampler, the
// serving loop and the estimators.
#include <cstring>
#include <string>

#include "plan.hpp"

namespace ces {

namespace {
thread_local std::string g_err;
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// An allocation the device cannot satisfy is CES_ERR_NOMEM (as an
// exhausted budget is); every other runtime error is CES_ERR_DEVICE.
int hip_fail(hipError_t e, const char* what) {
    const int code = e == hipErrorOutOfMemory ? CES_ERR_NOMEM : CES_ERR_DEVICE;
    return fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

int validate_desc(const ces_level_desc* d) {
    if (!d) return fail(CES_ERR_ARG, "desc is NULL");
    if (d->struct_size != (int32_t)sizeof(ces_level_desc)) return fail(CES_ERR_ARG, "desc.struct_size mismatch");
    if (d->cov_kind != CES_COV_MATERN && d->cov_kind != CES_COV_SEPEXP) return fail(CES_ERR_ARG, "cov_kind");
    if (d->cov_kind == CES_COV_MATERN && !(d->nu > 0.0 && d->nu <= 5.0))
        return fail(CES_ERR_ARG, "nu must be in (0, 5]");
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
    if (d->coupling != CES_COUPLE_RESTRICT && d->coupling != CES_COUPLE_EMBED) return fail(CES_ERR_ARG, "coupling");
    if (d->coupling == CES_COUPLE_EMBED && d->level_kind != CES_LEVEL_PAIR)
        return fail(CES_ERR_ARG, "coupling EMBED applies to PAIR levels");
    if (d->mg_cycle < CES_CYCLE_AUTO || d->mg_cycle > CES_CYCLE_W1) return fail(CES_ERR_ARG, "mg_cycle");
    return CES_OK;
}

size_t plan_setup_bytes(const ces_level_desc* d) {
    auto one = [&](int m) {
        const int pad = d->psd_policy == CES_PSD_GROW ? d->max_pad_factor : 2;
        const size_t nn = (size_t)pad * m * pad * m;
        // column, complex DFT work, raw and symmetrised eigenvalues (double),
        // two masks, two amplitude arrays (double at most)
        return nn * (8 + 16 + 8 + 8) + 2 * nn + 2 * nn * 8 + 64 * (size_t)pad * m + 4096;
    };
    size_t b = one(d->m_fine);
    if (d->coupling == CES_COUPLE_EMBED) b += one(d->m_fine / 2);
    return b + b / DevicePool::kReuseSlack + 64 * 256;
}

}  // namespace ces

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

const char* ces_last_error(void) { return ces::g_err.c_str(); }

}  // extern "C"
