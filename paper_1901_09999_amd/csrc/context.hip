// Context creation: configuration checks and the kernel-basis tables.
//
// The basis (Section 2, Eq. 7 with the zero-sum requirement; Section 3.1) is
// evaluated once on the host in FP64 and uploaded:
//   * full taps k_i(u, v) in FP64, used to realise per-patch kernels;
//   * the separable factors of each raw term,
//       raw_i(u, v) = f_{j,p}(u) f_{j,q}(v),  f_{j,e}(t) = t^e exp(-t^2 / 2 sigma_j^2),
//     in FP32 with the per-term normalisation psi_i and a flag z_i saying
//     whether k_0 is subtracted, so that the stamp fit can form
//       k_i (x) I = psi_i [f_{j,p} (x)_x (f_{j,q} (x)_y I)] - z_i (k_0 (x) I)
//     with two 1-D passes instead of a 2-D one.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace psfm {

int check_hip(hipError_t e) {
    (void)e;
    return PSFM_ERR_HIP;
}

int fit_bands(const psfm_context* ctx) { return (2 * ctx->r + 1 + ctx->fit_br - 1) / ctx->fit_br; }

int n_patches(const psfm_context* ctx, int W, int H) {
    const int P = ctx->cfg.patch;
    return ((W + P - 1) / P) * ((H + P - 1) / P);
}

}  // namespace psfm

extern "C" {

void psfm_config_default(psfm_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_gauss = 3;
    cfg->sigma[0] = 0.7;
    cfg->sigma[1] = 1.5;
    cfg->sigma[2] = 3.0;
    cfg->degree[0] = 6;
    cfg->degree[1] = 4;
    cfg->degree[2] = 2;
    cfg->half_width = 10;
    cfg->spatial_order = 0;
    cfg->stamp_half = 20;
    cfg->patch = 64;
    cfg->clip_sigma = 3.0;
    cfg->max_iter = 3;
    cfg->min_stamps = 3;
    cfg->bad_frac = 0.2;
    cfg->precision = PSFM_PREC_FP32;
    cfg->refine = 1;
}

int psfm_create(const psfm_config* cfg, psfm_context** out) {
    if (!cfg || !out) return PSFM_ERR_INVALID_ARG;
    *out = nullptr;
    const psfm_config& c = *cfg;
    if (c.n_gauss < 1 || c.n_gauss > PSFM_MAX_GAUSS) return PSFM_ERR_INVALID_ARG;
    int nb = 0, nf = 0;
    for (int j = 0; j < c.n_gauss; j++) {
        if (!(c.sigma[j] > 0.0) || c.degree[j] < 0 || c.degree[j] > 12) return PSFM_ERR_INVALID_ARG;
        nb += (c.degree[j] + 1) * (c.degree[j] + 2) / 2;
        nf += c.degree[j] + 1;
    }
    if (c.half_width < 1 || c.stamp_half < 1 || c.patch < 1 || c.spatial_order < 0 ||
        c.max_iter < 1 || c.min_stamps < 1 || !(c.clip_sigma > 0.0) || !(c.bad_frac > 0.0) ||
        !(c.bad_frac <= 1.0))
        return PSFM_ERR_INVALID_ARG;
    if (c.half_width > PSFM_HMAX || c.stamp_half > PSFM_RMAX || c.spatial_order > 6 ||
        nb + 2 > PSFM_GRAM_COLS || nf > 32 || c.precision < PSFM_PREC_FP32 ||
        c.precision > PSFM_PREC_FP16 || c.refine < 0 || c.refine > 4)
        return PSFM_ERR_UNSUPPORTED;
    if (c.weight_mode != PSFM_WEIGHT_V2 && c.weight_mode != PSFM_WEIGHT_V1V2)
        return PSFM_ERR_INVALID_ARG;
    if (c.ortho_basis != 0 && c.ortho_basis != 1) return PSFM_ERR_INVALID_ARG;
    if (c.flags & ~PSFM_SYNC) return PSFM_ERR_INVALID_ARG;
    if (c.fit_band_rows != 0 && c.fit_band_rows != PSFM_FIT_BR_SHORT &&
        c.fit_band_rows != PSFM_FIT_BR_MID && c.fit_band_rows != PSFM_FIT_BR_TALL)
        return PSFM_ERR_UNSUPPORTED;

    psfm_context* ctx = new psfm_context();
    ctx->cfg = c;
    ctx->nb = nb;
    ctx->nf = nf;
    ctx->ns = (c.spatial_order + 1) * (c.spatial_order + 2) / 2;
    ctx->N = nb * ctx->ns + 1;
    ctx->L = nb + 1;
    ctx->h = c.half_width;
    ctx->r = c.stamp_half;
    // fit band: 7 rows up to 41-row stamps (r <= 20: three workgroups' LDS per CU
    // at h = 10, which hides the band's latencies better than fewer, taller
    // bands: 7+7+7+7+7+6 rows at r = 20), 11 rows beyond (fewer bands per stamp
    // when the stamps are large: 11+11+11+11+5 at r = 24); a caller (a tuner)
    // may pick any of the three heights instead
    ctx->fit_br = c.fit_band_rows ? c.fit_band_rows
                                  : c.stamp_half <= 20 ? PSFM_FIT_BR_SHORT : PSFM_FIT_BR_TALL;
    ctx->KW = 2 * c.half_width + 1;
    ctx->T = ctx->KW * ctx->KW;
    const int h = ctx->h, KW = ctx->KW, T = ctx->T;

    // host tables
    std::vector<double> kb((size_t)nb * T);
    std::vector<float> fac((size_t)nf * KW);
    std::vector<double> fac64((size_t)nf * KW);
    std::vector<double> psi64(nb);
    std::vector<int> rowf(nb), colf(nb);
    std::vector<float> psi(nb), z(nb);
    // The basis is separable: term (j, p, q) is f_{j,p}(u) f_{j,q}(v) with
    // f_{j,e}(t) = t^e exp(-t^2 / 2 s_j^2).  Its 2-D sum and absolute sum are
    // products of the factors' 1-D sums, which give the normalisation psi_i
    // (unit sum for the even-even terms, unit absolute sum for the others);
    // the even-even terms i >= 1 then have k_0 (unit sum) subtracted, so
    // that every term but k_0 sums to zero.
    std::vector<double> sum1((size_t)nf), abs1((size_t)nf);
    {
        int f = 0;
        for (int j = 0; j < c.n_gauss; j++) {
            const double inv2s2 = 0.5 / (c.sigma[j] * c.sigma[j]);
            for (int e = 0; e <= c.degree[j]; e++, f++) {
                double s1 = 0.0, a1 = 0.0;
                for (int t = -h; t <= h; t++) {
                    double mono = 1.0;
                    for (int k = 0; k < e; k++) mono *= (double)t;
                    const double v = mono * std::exp(-(double)(t * t) * inv2s2);
                    fac64[(size_t)f * KW + (t + h)] = v;
                    fac[(size_t)f * KW + (t + h)] = (float)v;
                    s1 += v;
                    a1 += std::fabs(v);
                }
                sum1[f] = s1;
                abs1[f] = a1;
            }
        }
    }
    {
        int i = 0, f0 = 0;
        for (int j = 0; j < c.n_gauss; j++) {
            for (int d = 0; d <= c.degree[j]; d++)
                for (int p = d; p >= 0; p--, i++) {
                    const int fu = f0 + p, fv = f0 + (d - p);
                    const bool even = (p % 2 == 0) && ((d - p) % 2 == 0);
                    const double nrm = even ? 1.0 / (sum1[fu] * sum1[fv]) : 1.0 / (abs1[fu] * abs1[fv]);
                    const bool zs = even && i > 0;
                    rowf[i] = fu;
                    colf[i] = fv;
                    psi64[i] = nrm;
                    psi[i] = (float)nrm;
                    z[i] = zs ? 1.0f : 0.0f;
                    double* ki = kb.data() + (size_t)i * T;
                    for (int v = 0; v < KW; v++)
                        for (int u = 0; u < KW; u++) {
                            const double sep = nrm * fac64[(size_t)fu * KW + u] * fac64[(size_t)fv * KW + v];
                            ki[v * KW + u] = zs ? sep - kb[v * KW + u] : sep;
                        }
                }
            f0 += c.degree[j] + 1;
        }
    }

    // R: upper Cholesky factor of the basis Gram G_ij = sum_t k_i(t) k_j(t), so
    // that R a holds the coefficients of the kernel in an orthonormal basis of
    // the same span (kernel-image norms become coefficient norms)
    std::vector<double> R((size_t)nb * nb, 0.0);
    ctx->kgram_ok = true;
    {
        std::vector<double> G((size_t)nb * nb);
        for (int a = 0; a < nb; a++)
            for (int b = 0; b <= a; b++) {
                double g = 0.0;
                for (int t = 0; t < T; t++) g += kb[(size_t)a * T + t] * kb[(size_t)b * T + t];
                G[(size_t)a * nb + b] = G[(size_t)b * nb + a] = g;
            }
        for (int j = 0; j < nb && ctx->kgram_ok; j++) {   // G = R^T R, R upper
            double d = G[(size_t)j * nb + j];
            for (int k = 0; k < j; k++) d -= R[(size_t)k * nb + j] * R[(size_t)k * nb + j];
            if (!(d > 1e-12 * G[(size_t)j * nb + j])) {   // terms (nearly) dependent on these taps:
                ctx->kgram_ok = false;                      // no orthonormal map (learned prior only)
                break;
            }
            const double rjj = std::sqrt(d);
            R[(size_t)j * nb + j] = rjj;
            for (int m = j + 1; m < nb; m++) {
                double v = G[(size_t)j * nb + m];
                for (int k = 0; k < j; k++) v -= R[(size_t)k * nb + j] * R[(size_t)k * nb + m];
                R[(size_t)j * nb + m] = v / rjj;
            }
        }
    }

    // penalty weights of the two-kernel form (Eq. 9 without Phi):
    // Q_i = sum_{u,v} (u^2 + v^2)^2 k_i(u, v)^2
    std::vector<double> penq(nb);
    for (int t = 0; t < nb; t++) {
        double q = 0.0;
        for (int v = -h; v <= h; v++)
            for (int u = -h; u <= h; u++) {
                const double rr = (double)(u * u + v * v), k = kb[(size_t)t * T + (v + h) * KW + (u + h)];
                q += rr * rr * k * k;
            }
        penq[t] = q;
    }

    // one device block for all tables
    psfm::Carver layout(nullptr);
    double* d_kb = layout.take<double>(kb.size());
    float* d_fac = layout.take<float>(fac.size());
    int* d_rowf = layout.take<int>(nb);
    int* d_colf = layout.take<int>(nb);
    int* d_rorder = layout.take<int>(nb);
    int* d_rstart = layout.take<int>(nf + 1);
    float* d_psi = layout.take<float>(nb);
    float* d_z = layout.take<float>(nb);
    double* d_fac64 = layout.take<double>(fac64.size());
    double* d_psi64 = layout.take<double>(nb);
    double* d_R = layout.take<double>(R.size());
    double* d_penq = layout.take<double>(nb);
    const size_t bytes = layout.off;
    char* blk = nullptr;
    if (hipMalloc(&blk, bytes) != hipSuccess) {
        delete ctx;
        return PSFM_ERR_HIP;
    }
    auto rebase = [&](auto* p) { return reinterpret_cast<decltype(p)>(blk + reinterpret_cast<size_t>(p)); };
    ctx->dev_block = blk;
    ctx->kb64 = rebase(d_kb);
    ctx->fac = rebase(d_fac);
    ctx->term_rowf = rebase(d_rowf);
    ctx->term_colf = rebase(d_colf);
    ctx->term_rorder = rebase(d_rorder);
    ctx->row_start = rebase(d_rstart);
    ctx->term_psi = rebase(d_psi);
    ctx->term_z = rebase(d_z);
    ctx->fac64 = rebase(d_fac64);
    ctx->psi64 = rebase(d_psi64);
    ctx->kgram_R = rebase(d_R);
    ctx->penq = rebase(d_penq);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(ctx->kb64, kb.data(), kb.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->fac, fac.data(), fac.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->term_rowf, rowf.data(), nb * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->term_colf, colf.data(), nb * sizeof(int), hipMemcpyHostToDevice);
    {
        // the terms grouped by row factor (stable: increasing i within a group)
        std::vector<int> rorder(nb), rstart(nf + 1, 0);
        for (int i = 0; i < nb; i++) rstart[rowf[i] + 1]++;
        for (int f = 0; f < nf; f++) rstart[f + 1] += rstart[f];
        std::vector<int> fill(rstart.begin(), rstart.end() - 1);
        for (int i = 0; i < nb; i++) rorder[fill[rowf[i]]++] = i;
        if (e == hipSuccess)
            e = hipMemcpy(ctx->term_rorder, rorder.data(), nb * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(ctx->row_start, rstart.data(), (nf + 1) * sizeof(int), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(ctx->term_psi, psi.data(), nb * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->term_z, z.data(), nb * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->fac64, fac64.data(), fac64.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->psi64, psi64.data(), nb * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->kgram_R, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->penq, penq.data(), nb * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(blk);
        delete ctx;
        return PSFM_ERR_HIP;
    }
    *out = ctx;
    return PSFM_OK;
}

int psfm_destroy(psfm_context* ctx) {
    if (!ctx) return PSFM_ERR_INVALID_ARG;
    hipError_t e = hipFree(ctx->dev_block);
    delete ctx;
    return e == hipSuccess ? PSFM_OK : PSFM_ERR_HIP;
}

int psfm_n_basis(const psfm_context* ctx) { return ctx ? ctx->nb : -1; }
int psfm_n_spatial(const psfm_context* ctx) { return ctx ? ctx->ns : -1; }
int psfm_n_unknowns(const psfm_context* ctx) { return ctx ? ctx->N : -1; }
int psfm_stamp_dim(const psfm_context* ctx) { return ctx ? ctx->L : -1; }

size_t psfm_workspace_bytes(const psfm_context* ctx, int W, int H, int n_stamps) {
    if (!ctx || W < 1 || H < 1 || n_stamps < 0) return 0;
    size_t b = psfm::fit_workspace(ctx, n_stamps);
    size_t s = psfm::solve_workspace(ctx, n_stamps);
    size_t c = psfm::conv_workspace(ctx, W, H);
    size_t d = psfm::subtract_workspace(ctx, W, H);
    size_t e = psfm::match_workspace(ctx, W, H);
    size_t m = b;
    if (s > m) m = s;
    if (c > m) m = c;
    if (d > m) m = d;
    if (e > m) m = e;
    return psfm::align_up(m, 256) + 256;
}

size_t psfm_dual_workspace_bytes(const psfm_context* ctx, int W, int H, int n_stamps) {
    if (!ctx || W < 1 || H < 1 || n_stamps < 0) return 0;
    size_t f = psfm::dual_fit_workspace(ctx, n_stamps);
    size_t s = psfm::dual_solve_workspace(ctx, n_stamps);
    return psfm::align_up(f > s ? f : s, 256) + 256;
}

int psfm_dual_unknowns(const psfm_context* ctx) { return ctx ? psfm::dual_unknowns(ctx) : -1; }

size_t psfm_stamp_design_floats(const psfm_context* ctx, int n_stamps) {
    if (!ctx || n_stamps < 0 || ctx->cfg.precision == PSFM_PREC_FP32) return 0;
    const size_t npx = (size_t)(2 * ctx->r + 1) * (2 * ctx->r + 1);
    return (size_t)n_stamps * (ctx->nb + 2) * npx;
}

const char* psfm_status_string(int status) {
    switch (status) {
        case PSFM_OK: return "ok";
        case PSFM_ERR_INVALID_ARG: return "invalid argument";
        case PSFM_ERR_SHAPE: return "invalid image or stamp shape";
        case PSFM_ERR_TOO_FEW_STAMPS: return "too few usable stamps";
        case PSFM_ERR_NOT_PD: return "normal matrix not positive definite";
        case PSFM_ERR_HIP: return "HIP runtime error";
        case PSFM_ERR_WORKSPACE: return "workspace missing or too small";
        case PSFM_ERR_UNSUPPORTED: return "configuration not supported by the kernels";
        case PSFM_ERR_NORM_SINGULAR: return "normalisation undetermined by the stamp totals";
        default: return "unknown status";
    }
}

}  // extern "C"
