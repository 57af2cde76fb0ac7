// C ABI of libagis (include/agis.h): context, parameters, update blocks,
// frame rotator and the simple-iteration driver.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "agis_internal.h"

namespace agis {

int set_error(agis_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_check(agis_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return AGIS_OK;
    return set_error(ctx, e == hipErrorOutOfMemory ? AGIS_E_OOM : AGIS_E_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace agis

using namespace agis;

static std::string g_create_error;

// Scratch of agis_chi2_noalloc: the per-block partial sums of chi^2 and
// their total, in a file-scope device array of which each GPU holds its own
// copy until the process ends.  Host code reaches a GPU's copy only through
// the address hipGetSymbolAddress returns with that GPU current (resolved
// once per device by agis_create), never through the array's name.
constexpr int64_t kScratchDoubles = 131072;               // 1 MiB per GPU
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;                // per device ordinal (null: not resolved)

// Address of the current device's copy of scratch (device must be current).
static double* scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_dev[device] = static_cast<double*>(p);
    }
    return g_scratch_dev[device];
}

#define HIPCHK(expr)                                            \
    do {                                                        \
        int rc_ = hip_check(ctx, (expr), #expr);                \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

#define CHECK_CTX()                                                              \
    do {                                                                         \
        if (!ctx) return AGIS_E_INVALID_ARG;                                     \
        ctx->err.clear();                                                        \
        int rc_ = hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice");     \
        if (rc_ != AGIS_OK) return rc_;                                          \
    } while (0)

#define REQUIRE_LOADED()                                                                        \
    do {                                                                                        \
        if (!ctx->loaded) return set_error(ctx, AGIS_E_STATE, "observations not loaded");       \
    } while (0)

template <typename T>
static int dalloc(agis_ctx* ctx, T** p, size_t n, const char* what) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(ctx, AGIS_E_OOM, std::string("device allocation failed: ") + what);
    }
    return AGIS_OK;
}

#define ALLOC(p, n, what)                                       \
    do {                                                        \
        int rc_ = dalloc(ctx, &(p), (size_t)(n), what);         \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

template <typename T>
static void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

static void free_store(agis_ctx* ctx) {
    dfree(ctx->s_t);
    dfree(ctx->s_eta);
    dfree(ctx->s_sig);
    dfree(ctx->s_cell);
    dfree(ctx->s_ell);
    dfree(ctx->src_off);
    dfree(ctx->src_order);
    dfree(ctx->t_t);
    dfree(ctx->t_eta);
    dfree(ctx->t_sig);
    dfree(ctx->t_cellfov);
    dfree(ctx->t_src);
    dfree(ctx->t_perm);
    dfree(ctx->s_from_t);
    dfree(ctx->s_sig_eff);
    dfree(ctx->t_sig_eff);
    ctx->frozen = false;
    for (double** v : {&ctx->geo, &ctx->dgeo, &ctx->geo_sums, &ctx->t_eta0, &ctx->s_eta0, &ctx->geo_wr}) dfree(*v);
    dfree(ctx->t_geo_g);
    dfree(ctx->s_geo_g);
    dfree(ctx->t_geo_mu);
    dfree(ctx->s_geo_mu);
    dfree(ctx->geo_flags);
    dfree(ctx->geo_pos);
    dfree(ctx->geo_off);
    dfree(ctx->geo_mu_g);
    dfree(ctx->geo_coff);
    dfree(ctx->geo_colsum);
    dfree(ctx->geo_dcol);
    dfree(ctx->geo_zpart);
    ctx->geo_ccds = 0;
    ctx->geo_ac_cells = 0;
    ctx->geo_small_days = 0;
    ctx->n_small = 0;
    ctx->n_groups = 0;
    dfree(ctx->iv_off);
    dfree(ctx->iv_cell);
    dfree(ctx->cell_iv);
    dfree(ctx->s);
    dfree(ctx->c);
    dfree(ctx->prep);
    dfree(ctx->s_ref);
    dfree(ctx->ds);
    dfree(ctx->qsrc);
    dfree(ctx->sdef);
    dfree(ctx->svar);
    dfree(ctx->dc);
    dfree(ctx->vs);
    dfree(ctx->src_eps2);
    dfree(ctx->src_D);
    dfree(ctx->rcol);
    ctx->s_classes.clear();
    ctx->s_fallback = 0;
    ctx->eps_cap = 0;
    ctx->eps_fused = false;
    dfree(ctx->lh_anchor_s);
    dfree(ctx->lh_ring_s);
    dfree(ctx->lh_anchor_a);
    dfree(ctx->lh_ring_a);
    dfree(ctx->lh_anchor_c);
    dfree(ctx->lh_ring_c);
    dfree(ctx->asi_part);
    dfree(ctx->asi_out);
    for (int w = 0; w < 2; ++w) {
        dfree(ctx->lf_X[w]);
        dfree(ctx->lf_scale[w]);
        dfree(ctx->lf_Y[w]);
    }
    for (int k = 0; k < 2; ++k) {
        dfree(ctx->bk_s[k]);
        dfree(ctx->bk_a[k]);
        dfree(ctx->bk_c[k]);
        dfree(ctx->bk_e[k]);
    }
    dfree(ctx->chi2_part);
    dfree(ctx->chi2_out);
    for (double** v : {&ctx->cg_r, &ctx->cg_z, &ctx->cg_p, &ctx->cg_ry, &ctx->cg_zy, &ctx->cg_sy, &ctx->cg_part,
                       &ctx->cg_qpart, &ctx->cg_out})
        dfree(*v);
    ctx->cg_k = 0;
    ctx->lh_count = 0;
    ctx->loaded = false;
    ctx->have_ref = false;
    ++ctx->gen;
}

static int copy_in(agis_ctx* ctx, void* dst, const void* src, size_t bytes, int where) {
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    HIPCHK(hipMemcpyAsync(dst, src, bytes, where == AGIS_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                          ctx->stream));
    if (where == AGIS_HOST) HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

static int copy_out(agis_ctx* ctx, void* dst, const void* src, size_t bytes, int where) {
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    HIPCHK(hipMemcpyAsync(dst, src, bytes, where == AGIS_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_version(void) { return AGIS_VERSION; }

extern "C" const char* agis_last_error(const agis_ctx_t* ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

// Segments of Sect. 5.2.2: segment K uses the knot intervals of
// [tau_{x_K - L}, tau_{x_{K+1} + L}) and supplies the updates of
// x_K - 1 <= n <= x_{K+1} - 2 (M = 4); x_K = 3 + K * seg_len.
static void build_segments(agis_ctx* ctx) {
    const int64_t N = ctx->N, K = ctx->K;
    const int64_t S = ctx->cfg.seg_len, L = ctx->cfg.seg_overlap;
    const int64_t nseg = (K + S - 1) / S;
    ctx->h_segs.clear();
    int64_t off = 0;
    for (int64_t s = 0; s < nseg; ++s) {
        const int64_t x0 = 3 + s * S;
        const int64_t x1 = s + 1 < nseg ? x0 + S : N;
        int64_t lo = s == 0 ? 3 : x0 - L;
        int64_t hi = s + 1 < nseg ? x1 + L : N;
        lo = std::max<int64_t>(lo, 3);
        hi = std::min<int64_t>(hi, N);
        SegDesc d;
        d.n_lo = lo - 3;
        d.n_hi = hi - 1;
        d.keep_lo = s == 0 ? 0 : x0 - 1;
        d.keep_hi = s + 1 < nseg ? x1 - 2 : N - 1;
        d.u_off = off;
        off += 4 * (d.n_hi - d.n_lo + 1);
        ctx->h_segs.push_back(d);
    }
    ctx->ufac_rows = off;
}

// Table of the observation model per knot interval l = j + 3: orbital
// longitude at tau_l, and 1/(tau_l+1 - tau_l) when tau_l-2..tau_l+3 are
// exactly equally spaced (the closed-form B-splines then equal the general
// recursion to rounding), else 0.
static std::vector<KnotTab> knot_table(const agis_ctx* ctx) {
    const std::vector<double>& kn = ctx->h_knots;
    std::vector<KnotTab> tab(ctx->K);
    for (int64_t j = 0; j < ctx->K; ++j) {
        const int64_t l = j + 3;
        const double dt = kn[l + 1] - kn[l];
        bool uniform = dt > 0.0;
        for (int64_t i = l - 2; i < l + 3 && uniform; ++i) uniform = (kn[i + 1] - kn[i]) == dt;
        const double L = ctx->cfg.eph_L0 + ctx->cfg.eph_Lrate * kn[l];
        tab[j].sL = std::sin(L);
        tab[j].cL = std::cos(L);
        tab[j].inv_dt = uniform ? 1.0 / dt : 0.0;
        tab[j].tau = kn[l];
    }
    return tab;
}

extern "C" int agis_create(const agis_config_t* cfg, agis_ctx_t** out) {
    g_create_error.clear();
    if (!cfg || !out) {
        g_create_error = "null argument";
        return AGIS_E_INVALID_ARG;
    }
    *out = nullptr;
    if (cfg->n_knots < 8 || !cfg->knots) {
        g_create_error = "need at least 8 knots (order 4, one interval)";
        return AGIS_E_SHAPE;
    }
    for (int64_t i = 1; i < cfg->n_knots; ++i) {
        if (!(cfg->knots[i] >= cfg->knots[i - 1])) {
            g_create_error = "knot sequence must be non-decreasing and finite";
            return AGIS_E_INVALID_ARG;
        }
    }
    if (!(cfg->knots[cfg->n_knots - 4] > cfg->knots[3])) {
        g_create_error = "empty spline interval";
        return AGIS_E_SHAPE;
    }
    if (cfg->seg_len < 1 || cfg->seg_overlap < 0) {
        g_create_error = "seg_len must be >= 1 and seg_overlap >= 0";
        return AGIS_E_INVALID_ARG;
    }
    if (cfg->precision != AGIS_FP64 && cfg->precision != AGIS_MIXED) {
        g_create_error = "precision must be AGIS_FP64 or AGIS_MIXED";
        return AGIS_E_INVALID_ARG;
    }
    if (cfg->robust < 0 || cfg->robust > 2 || (cfg->robust && cfg->eps_bucket < 1) ||
        !(std::isfinite(cfg->eps_a_init) && cfg->eps_a_init >= 0.0)) {
        g_create_error = "robust must be 0, 1 or 2, eps_bucket >= 1 and eps_a_init finite and >= 0";
        return AGIS_E_INVALID_ARG;
    }
    if (!(cfg->year_s > 0) || !(cfg->c_mps > 0) || !(cfg->au_m > 0)) {
        g_create_error = "year_s, c_mps and au_m must be positive";
        return AGIS_E_INVALID_ARG;
    }
    if (!(std::isfinite(cfg->defl) && cfg->defl >= 0.0) || (cfg->ppn && !(cfg->defl > 0.0)) ||
        (cfg->defl > 0.0 && cfg->precision != AGIS_FP64)) {
        g_create_error = "defl must be finite and >= 0, ppn needs defl > 0, and the deflection runs in FP64 only";
        return AGIS_E_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        g_create_error = "no such HIP device";
        return AGIS_E_DEVICE;
    }
    agis_ctx* ctx = new (std::nothrow) agis_ctx();
    if (!ctx) {
        g_create_error = "out of host memory";
        return AGIS_E_OOM;
    }
    ctx->cfg = *cfg;
    ctx->cfg.knots = nullptr;
    ctx->device = cfg->device;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        delete ctx;
        return AGIS_E_DEVICE;
    }
    if (!scratch_address(ctx->device)) {
        g_create_error = "hipGetSymbolAddress of the scratch array failed";
        delete ctx;
        return AGIS_E_DEVICE;
    }
    if (cfg->stream) {
        ctx->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            g_create_error = "hipStreamCreate failed";
            delete ctx;
            return AGIS_E_DEVICE;
        }
        ctx->own_stream = true;
    }
    ctx->n_knots = cfg->n_knots;
    ctx->N = cfg->n_knots - 4;
    ctx->K = ctx->N - 3;
    ctx->h_knots.assign(cfg->knots, cfg->knots + cfg->n_knots);
    DevConsts& k = ctx->k;
    k.gamma_half = 0.5 * cfg->gamma_c;
    k.t_ep = cfg->t_ep;
    k.t_fr = cfg->t_fr;
    k.inv_year = 1.0 / cfg->year_s;
    k.year_s = cfg->year_s;
    k.au_c = cfg->au_m / cfg->c_mps;
    k.lam2 = cfg->lambda_reg * cfg->lambda_reg;
    k.eph_r = cfg->eph_radius_au;
    k.eph_L0 = cfg->eph_L0;
    k.eph_Lrate = cfg->eph_Lrate;
    k.cos_obl = std::cos(cfg->eps_obl);
    k.sin_obl = std::sin(cfg->eps_obl);
    k.cos_half_gamma = std::cos(k.gamma_half);
    k.sin_half_gamma = std::sin(k.gamma_half);
    k.half_gamma_err = (double)((long double)k.gamma_half -
                                std::atan2((long double)k.sin_half_gamma, (long double)k.cos_half_gamma));
    k.ac_cf0 = INT32_MAX;                    // set by agis_load_observations
    k.defl = cfg->defl > 0.0 ? cfg->defl : 0.0;
    build_segments(ctx);
    if (cfg->robust) {
        ctx->n_buckets = (ctx->K + cfg->eps_bucket - 1) / cfg->eps_bucket;
        k.n_buckets = ctx->n_buckets;
    }
    if (const char* e = std::getenv("AGIS_S_GROUP")) ctx->s_group = std::atoi(e);
    if (const char* e = std::getenv("AGIS_SELECT_REG_LIMIT")) ctx->select_reg_limit = std::atoll(e);
    if (const char* e = std::getenv("AGIS_SELECT_REG_MIN_MEAN")) ctx->select_reg_min_mean = std::atoll(e);
    if (const char* e = std::getenv("AGIS_SELECT_PAIR")) ctx->select_pair = std::atoi(e) != 0;
    // robust kernel paths: AGIS_ROBUST_FUSED = 0 (every step through HBM
    // columns), 1 (the excess-noise estimate in one kernel, the S block
    // through HBM columns; the default), 2 (the whole S block per source in
    // LDS), 3 (the S block's rows to HBM columns, then varsigma and the
    // solves per source in LDS), 4 (the S block per source with its rows in
    // registers)
    if (const char* e = std::getenv("AGIS_ROBUST_FUSED")) {
        const int v = std::atoi(e);
        ctx->robust_fused_eps = v >= 1;
        ctx->robust_s_mode = v == 4 ? 3 : (v == 3 ? 1 : (v == 2 ? 2 : 0));
    }
    if (const char* e = std::getenv("AGIS_ROBUST_MAX_CAP")) ctx->robust_max_cap = std::atoll(e);
    if (const char* e = std::getenv("AGIS_SREG_ROWS")) ctx->sreg_rows = std::atoi(e);
    if (const char* e = std::getenv("AGIS_IRLS_CACHE")) ctx->irls_cache = std::atoi(e);
    int rc = AGIS_OK;
    auto fail = [&](int code) {
        g_create_error = ctx->err;
        agis_destroy(ctx);
        return code;
    };
    if ((rc = dalloc(ctx, &ctx->knots, ctx->n_knots, "knots")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->ktab, ctx->K, "knot table")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->a, 4 * ctx->N, "attitude")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->da, 4 * ctx->N, "attitude update")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->gpar, 2, "global parameters")) != AGIS_OK ||
        (rc = dalloc(ctx, &ctx->dgpar, 2, "global update")) != AGIS_OK)
        return fail(rc);
    if (ctx->cfg.ppn && (rc = dalloc(ctx, &ctx->g_iv, 5 * std::max<int64_t>(ctx->K, 1), "global sums")) != AGIS_OK)
        return fail(rc);
    if (hipMemset(ctx->gpar, 0, 2 * sizeof(double)) != hipSuccess ||
        hipMemset(ctx->dgpar, 0, 2 * sizeof(double)) != hipSuccess)
        return fail(set_error(ctx, AGIS_E_DEVICE, "global parameters: clear failed"));
    ctx->k.gpar = ctx->gpar;
    if ((rc = dalloc(ctx, &ctx->iv_sums, (size_t)IV_SUMS * ctx->K, "interval sums")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->iv_cal, (size_t)IV_CAL * ctx->K, "interval calibration sums")) != AGIS_OK)
        return fail(rc);
    if ((rc = dalloc(ctx, &ctx->segs, ctx->h_segs.size(), "segments")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->seg_def, ctx->h_segs.size(), "segment defects")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->ufac, (size_t)16 * ctx->ufac_rows, "band factor")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->yfac, (size_t)ctx->ufac_rows, "band rhs")) != AGIS_OK) return fail(rc);
    ctx->red_len = 1 << 16;
    if ((rc = dalloc(ctx, &ctx->red, ctx->red_len, "reduction scratch")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->eo, 8, "frame parameters")) != AGIS_OK) return fail(rc);
    if ((rc = dalloc(ctx, &ctx->stat, 64, "statistics")) != AGIS_OK) return fail(rc);
    for (int w = 0; w < 2; ++w) {
        const int nw = mlp_num_weights(w);
        if ((rc = dalloc(ctx, &ctx->mlp_w[w], nw, "mlp weights")) != AGIS_OK) return fail(rc);
        if ((rc = dalloc(ctx, &ctx->mlp_wb[w], nw, "mlp weights")) != AGIS_OK) return fail(rc);
        if ((rc = dalloc(ctx, &ctx->mlp_m1[w], nw, "mlp moments")) != AGIS_OK) return fail(rc);
        if ((rc = dalloc(ctx, &ctx->mlp_m2[w], nw, "mlp moments")) != AGIS_OK) return fail(rc);
        if ((rc = dalloc(ctx, &ctx->mlp_g[w], nw + 1, "mlp gradient")) != AGIS_OK) return fail(rc);
        if (hipMemset(ctx->mlp_w[w], 0, nw * sizeof(float)) != hipSuccess ||
            hipMemset(ctx->mlp_wb[w], 0, nw * sizeof(float)) != hipSuccess ||
            hipMemset(ctx->mlp_m1[w], 0, nw * sizeof(float)) != hipSuccess ||
            hipMemset(ctx->mlp_m2[w], 0, nw * sizeof(float)) != hipSuccess) {
            ctx->err = "initial copies failed";
            return fail(AGIS_E_DEVICE);
        }
    }
    if (ctx->n_buckets > 0) {
        // three excess-noise functions (AL, ACP, ACF), n_buckets each
        if ((rc = dalloc(ctx, &ctx->eps_a2, 3 * ctx->n_buckets, "excess attitude noise")) != AGIS_OK) return fail(rc);
        const std::vector<double> e0(3 * ctx->n_buckets, cfg->eps_a_init * cfg->eps_a_init);
        if (hipMemcpy(ctx->eps_a2, e0.data(), e0.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            ctx->err = "initial copies failed";
            return fail(AGIS_E_DEVICE);
        }
    }
    const std::vector<KnotTab> h_ktab = knot_table(ctx);
    if (hipMemcpy(ctx->knots, cfg->knots, ctx->n_knots * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->ktab, h_ktab.data(), h_ktab.size() * sizeof(KnotTab), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->segs, ctx->h_segs.data(), ctx->h_segs.size() * sizeof(SegDesc), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(ctx->da, 0, 4 * ctx->N * sizeof(double)) != hipSuccess ||
        hipMemset(ctx->eo, 0, 8 * sizeof(double)) != hipSuccess) {
        ctx->err = "initial copies failed";
        return fail(AGIS_E_DEVICE);
    }
    for (int e = 0; e < 10; ++e) {
        ctx->tm.valid[e] = false;
        if (hipEventCreate(&ctx->tm.ev[e][0]) != hipSuccess || hipEventCreate(&ctx->tm.ev[e][1]) != hipSuccess) {
            ctx->err = "hipEventCreate failed";
            return fail(AGIS_E_DEVICE);
        }
    }
    *out = ctx;
    return AGIS_OK;
}

extern "C" void agis_destroy(agis_ctx_t* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    free_store(ctx);
    dfree(ctx->knots);
    dfree(ctx->ktab);
    dfree(ctx->a);
    dfree(ctx->da);
    dfree(ctx->gpar);
    dfree(ctx->dgpar);
    dfree(ctx->g_iv);
    dfree(ctx->iv_sums);
    dfree(ctx->iv_cal);
    dfree(ctx->segs);
    dfree(ctx->seg_def);
    dfree(ctx->ufac);
    dfree(ctx->yfac);
    dfree(ctx->red);
    dfree(ctx->eo);
    dfree(ctx->stat);
    dfree(ctx->eps_a2);
    for (int w = 0; w < 2; ++w) {
        dfree(ctx->mlp_w[w]);
        dfree(ctx->mlp_wb[w]);
        dfree(ctx->mlp_m1[w]);
        dfree(ctx->mlp_m2[w]);
        dfree(ctx->mlp_g[w]);
    }
    for (int e = 0; e < 10; ++e) {
        if (ctx->tm.ev[e][0]) (void)hipEventDestroy(ctx->tm.ev[e][0]);
        if (ctx->tm.ev[e][1]) (void)hipEventDestroy(ctx->tm.ev[e][1]);
    }
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

extern "C" int agis_load_observations(agis_ctx_t* ctx, const agis_obs_soa_t* obs, int64_t n_src, int64_t n_cells,
                                      int where) {
    CHECK_CTX();
    ++ctx->xver;
    if (!obs || n_src < 0 || n_cells < 0 || obs->n < 0) return set_error(ctx, AGIS_E_INVALID_ARG, "bad arguments");
    if (obs->n > 0 && (!obs->t || !obs->eta_obs || !obs->sigma || !obs->src || !obs->fov || !obs->cell))
        return set_error(ctx, AGIS_E_INVALID_ARG, "null observation column");
    if (obs->n >= (int64_t)1 << 31) return set_error(ctx, AGIS_E_SHAPE, "at most 2^31 - 1 observations");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    if (n_cells >= (int64_t)1 << 29) return set_error(ctx, AGIS_E_SHAPE, "at most 2^29 - 1 calibration cells");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    free_store(ctx);
    ctx->n_obs = obs->n;
    ctx->n_src = n_src;
    ctx->n_cells = n_cells;
    ALLOC(ctx->s, 5 * n_src, "sources");
    ALLOC(ctx->c, n_cells + 1, "calibration");
    ctx->k.ac_cf0 = (int32_t)(2 * n_cells);
    ALLOC(ctx->prep, n_src, "source prep");
    ALLOC(ctx->ds, 5 * n_src, "source updates");
    ALLOC(ctx->qsrc, n_src, "source chi2");
    ALLOC(ctx->sdef, n_src, "source defects");
    ALLOC(ctx->svar, 5 * n_src, "source variances");
    ALLOC(ctx->dc, n_cells, "calibration updates");
    HIPCHK(hipMemsetAsync(ctx->s, 0, 5 * std::max<int64_t>(n_src, 1) * sizeof(double), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->c, 0, (n_cells + 1) * sizeof(double), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->dc, 0, std::max<int64_t>(n_cells, 1) * sizeof(double), ctx->stream));
    {
        // unit weights for the frame fit until the first S update
        std::vector<double> ones(5 * std::max<int64_t>(n_src, 1), 1.0);
        HIPCHK(hipMemcpyAsync(ctx->svar, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    int rc = build_store(ctx, obs, where);
    if (rc != AGIS_OK) {
        std::string keep = ctx->err;
        free_store(ctx);
        ctx->err = keep;
        return rc;
    }
    {
        // launch order of the sources in the S pass: by decreasing number of
        // observations, so that the sources sharing a wavefront (and its
        // loop trip count) have nearly equal counts (ties by index)
        std::vector<int64_t> h_off(n_src + 1);
        HIPCHK(hipMemcpyAsync(h_off.data(), ctx->src_off, (n_src + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        std::vector<int32_t> order(n_src);
        for (int64_t i = 0; i < n_src; ++i) order[i] = (int32_t)i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            return h_off[x + 1] - h_off[x] > h_off[y + 1] - h_off[y];
        });
        ALLOC(ctx->src_order, std::max<int64_t>(n_src, 1), "source order");
        HIPCHK(hipMemcpyAsync(ctx->src_order, order.data(), n_src * sizeof(int32_t), hipMemcpyHostToDevice,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        bool need_columns = true;
        if (ctx->cfg.robust) {
            int prc = robust_plan(ctx, h_off, order, &need_columns);
            if (prc != AGIS_OK) return prc;
        }
        if (ctx->cfg.robust && need_columns)
            ALLOC(ctx->rcol, 6 * std::max<int64_t>(ctx->n_obs, 1), "robust columns");
    }
    if (ctx->cfg.robust) {
        // the inner iteration's by-source columns (A, h, sigma~^2), also
        // used for R^2 - sigma^2 by the excess-noise estimate
        ALLOC(ctx->vs, 2 * n_src, "source varsigma per kind");
        if (ctx->cfg.robust == 2) {
            ALLOC(ctx->src_eps2, std::max<int64_t>(n_src, 1), "excess source noise");
            ALLOC(ctx->src_D, std::max<int64_t>(n_src, 1), "excess source noise significance");
            HIPCHK(hipMemsetAsync(ctx->src_eps2, 0, std::max<int64_t>(n_src, 1) * sizeof(double), ctx->stream));
            HIPCHK(hipMemsetAsync(ctx->src_D, 0, std::max<int64_t>(n_src, 1) * sizeof(double), ctx->stream));
        }
    }
    launch_prep_sources(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->loaded = true;
    return AGIS_OK;
}

static int check_finite_host(agis_ctx* ctx, const double* x, int64_t n, int where) {
    if (where != AGIS_HOST) return AGIS_OK;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return set_error(ctx, AGIS_E_NUMERIC, "non-finite parameter value");
    return AGIS_OK;
}

extern "C" int agis_set_sources(agis_ctx_t* ctx, int64_t n, const double* s5, int where) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (n != ctx->n_src || (!s5 && n > 0)) return set_error(ctx, AGIS_E_SHAPE, "source count mismatch");
    int rc = check_finite_host(ctx, s5, 5 * n, where);
    if (rc) return rc;
    rc = copy_in(ctx, ctx->s, s5, 5 * n * sizeof(double), where);
    if (rc) return rc;
    launch_prep_sources(ctx);
    HIPCHK(hipGetLastError());
    return AGIS_OK;
}

extern "C" int agis_get_sources(agis_ctx_t* ctx, int64_t n, double* s5, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (n != ctx->n_src || (!s5 && n > 0)) return set_error(ctx, AGIS_E_SHAPE, "source count mismatch");
    return copy_out(ctx, s5, ctx->s, 5 * n * sizeof(double), where);
}

extern "C" int agis_set_attitude(agis_ctx_t* ctx, int64_t n, const double* a4, int where) {
    CHECK_CTX();
    ++ctx->xver;
    if (n != ctx->N || !a4) return set_error(ctx, AGIS_E_SHAPE, "attitude coefficient count must be n_knots - 4");
    int rc = check_finite_host(ctx, a4, 4 * n, where);
    if (rc) return rc;
    return copy_in(ctx, ctx->a, a4, 4 * n * sizeof(double), where);
}

extern "C" int agis_get_attitude(agis_ctx_t* ctx, int64_t n, double* a4, int where) {
    CHECK_CTX();
    if (n != ctx->N || !a4) return set_error(ctx, AGIS_E_SHAPE, "attitude coefficient count must be n_knots - 4");
    return copy_out(ctx, a4, ctx->a, 4 * n * sizeof(double), where);
}

extern "C" int agis_set_calibration(agis_ctx_t* ctx, int64_t n, const double* c, int where) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (ctx->geo_ccds > 0)
        return set_error(ctx, AGIS_E_STATE, "the geometric calibration replaces the cell offsets "
                                            "(agis_set_geo_calibration)");
    if (n != ctx->n_cells || (!c && n > 0)) return set_error(ctx, AGIS_E_SHAPE, "cell count mismatch");
    int rc = check_finite_host(ctx, c, n, where);
    if (rc) return rc;
    return copy_in(ctx, ctx->c, c, n * sizeof(double), where);
}

extern "C" int agis_load_geometry(agis_ctx_t* ctx, int64_t n, const int8_t* ccd, const float* mu, int32_t n_ccd,
                                  const int32_t* ac_cell, int32_t n_ac_cells, int32_t small_days, int where) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    if (n != ctx->n_obs || ((!ccd || !mu) && n > 0)) return set_error(ctx, AGIS_E_SHAPE, "record count mismatch");
    if (n_ccd < 1 || n_ccd > 127) return set_error(ctx, AGIS_E_INVALID_ARG, "n_ccd outside [1, 127]");
    if (n_ac_cells < 0 || (n_ac_cells > 0 && !ac_cell && n > 0))
        return set_error(ctx, AGIS_E_INVALID_ARG, "n_ac_cells < 0, or AC cells counted but not given");
    if (ctx->cfg.robust == 2) return set_error(ctx, AGIS_E_STATE, "the geometric calibration with robust mode 2");
    if (small_days < 0) return set_error(ctx, AGIS_E_INVALID_ARG, "small_days < 0");
    const int rc = load_geometry(ctx, ccd, mu, n_ccd, ac_cell, n_ac_cells, small_days, where);
    ++ctx->gen;                          // the captured iteration gains the geometric kernels
    return rc;
}

extern "C" int agis_set_geo_calibration(agis_ctx_t* ctx, int64_t n, const double* c, int where) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (ctx->geo_ccds <= 0) return set_error(ctx, AGIS_E_STATE, "agis_load_geometry first");
    if (n != 3 * ctx->n_groups + ctx->n_small || (!c && n > 0))
        return set_error(ctx, AGIS_E_SHAPE, "coefficient count mismatch");
    int rc = check_finite_host(ctx, c, n, where);
    if (rc) return rc;
    if ((rc = copy_in(ctx, ctx->geo, c, n * sizeof(double), where))) return rc;
    launch_geo_eta(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_get_geo_calibration(agis_ctx_t* ctx, int64_t n, double* c, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (ctx->geo_ccds <= 0) return set_error(ctx, AGIS_E_STATE, "agis_load_geometry first");
    if (n != 3 * ctx->n_groups + ctx->n_small || (!c && n > 0))
        return set_error(ctx, AGIS_E_SHAPE, "coefficient count mismatch");
    return copy_out(ctx, c, ctx->geo, n * sizeof(double), where);
}

extern "C" int agis_basic_angle(agis_ctx_t* ctx, int64_t n_days, double* out, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    if (ctx->geo_ccds <= 0) return set_error(ctx, AGIS_E_STATE, "agis_load_geometry first");
    if (n_days != ctx->n_cells / 2 || (!out && n_days > 0)) return set_error(ctx, AGIS_E_SHAPE, "day count mismatch");
    if (n_days == 0) return AGIS_OK;
    double* dst = out;
    if (where == AGIS_HOST) HIPCHK(hipMalloc((void**)&dst, n_days * sizeof(double)));
    launch_geo_basic_angle(ctx, dst);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && where == AGIS_HOST)
        e = hipMemcpyAsync(out, dst, n_days * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (where == AGIS_HOST) (void)hipFree(dst);
    return e == hipSuccess ? AGIS_OK : hip_check(ctx, e, "basic angle");
}

extern "C" int agis_get_calibration(agis_ctx_t* ctx, int64_t n, double* c, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (n != ctx->n_cells || (!c && n > 0)) return set_error(ctx, AGIS_E_SHAPE, "cell count mismatch");
    return copy_out(ctx, c, ctx->c, n * sizeof(double), where);
}

// --- timing and statistics helpers -----------------------------------------
enum { T_S = 0, T_AC = 1, T_BAND = 2, T_CAL = 3, T_FRAME = 4, T_EPS = 5, T_ITER = 6 };

static void tstart(agis_ctx* ctx, int e) {
    if (ctx->timing) (void)hipEventRecord(ctx->tm.ev[e][0], ctx->stream);
}
static void tstop(agis_ctx* ctx, int e) {
    if (!ctx->timing) return;
    (void)hipEventRecord(ctx->tm.ev[e][1], ctx->stream);
    ctx->tm.valid[e] = true;
}
static double tget(agis_ctx* ctx, int e) {
    if (!ctx->tm.valid[e]) return 0.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->tm.ev[e][0], ctx->tm.ev[e][1]) != hipSuccess) return 0.0;
    return (double)ms;
}

static int fill_stats(agis_ctx* ctx, agis_block_stats_t* st, const double* x, int64_t n, int w,
                      const double* extra, const int32_t* iextra, int64_t n_obs, int64_t n_units) {
    if (!st) return AGIS_OK;
    launch_stats(ctx, x, n, w, extra, iextra, ctx->stat);
    HIPCHK(hipGetLastError());
    double h[12];
    HIPCHK(hipMemcpyAsync(h, ctx->stat, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memset(st, 0, sizeof(*st));
    for (int e = 0; e < 5; ++e) {
        st->rms_update[e] = h[e];
        st->max_update[e] = h[5 + e];
    }
    st->chi2 = h[10];
    st->defect = (int64_t)std::llround(h[11]);
    st->n_obs = n_obs;
    st->n_units = n_units;
    return AGIS_OK;
}

static int run_source(agis_ctx* ctx) {
    tstart(ctx, T_S);
    if (robust_now(ctx)) launch_source_update_robust(ctx);
    else launch_source_update(ctx);
    HIPCHK(hipGetLastError());
    tstop(ctx, T_S);
    return AGIS_OK;
}

// A/C accumulation pass followed by the requested solves.  The A update is
// applied only after the C solve has read the interval sums, so both blocks
// see the same parameters (S[AC]).  apply = false leaves the updates in da
// and dc; rc (optional) receives the calibration right-hand sides.
static int run_ac(agis_ctx* ctx, bool do_a, bool do_c, bool eps_update = false, bool apply = true,
                  double* rc = nullptr, bool do_g = false) {
    if (eps_update && robust_now(ctx)) {
        tstart(ctx, T_EPS);
        launch_excess_noise(ctx);
        tstop(ctx, T_EPS);
    }
    tstart(ctx, T_AC);
    launch_ac_pass(ctx);
    HIPCHK(hipGetLastError());
    tstop(ctx, T_AC);
    if (do_a) {
        tstart(ctx, T_BAND);
        launch_band_solve(ctx);
        HIPCHK(hipGetLastError());
        tstop(ctx, T_BAND);
    }
    if (do_c) {
        tstart(ctx, T_CAL);
        if (ctx->geo_ccds > 0) launch_geo_solve(ctx);
        else launch_calib_solve(ctx, rc);
        HIPCHK(hipGetLastError());
        tstop(ctx, T_CAL);
    }
    // the global block from the same parameters (S[ACG]; Sect. 5.4)
    do_g = do_g && ctx->cfg.ppn;
    if (do_g) {
        launch_global_solve(ctx);
        HIPCHK(hipGetLastError());
    }
    if (do_a && apply) launch_apply_attitude(ctx);
    if (do_c && apply) {
        if (ctx->geo_ccds > 0) {
            launch_apply_add(ctx, 3 * ctx->n_groups + ctx->n_small, ctx->geo, ctx->dgeo);
            launch_geo_eta(ctx);
        } else {
            launch_apply_calibration(ctx);
        }
    }
    if (do_g && apply) launch_apply_add(ctx, 1, ctx->gpar, ctx->dgpar);
    HIPCHK(hipGetLastError());
    return AGIS_OK;
}

static int stats_s(agis_ctx* ctx, agis_block_stats_t* st) {
    if (!st) return AGIS_OK;
    int rc = fill_stats(ctx, st, ctx->ds, ctx->n_src, 5, ctx->qsrc, ctx->sdef, ctx->n_obs, ctx->n_src);
    if (rc == AGIS_OK) st->ms = tget(ctx, T_S);
    return rc;
}
static int stats_a(agis_ctx* ctx, agis_block_stats_t* st) {
    if (!st) return AGIS_OK;
    int rc = fill_stats(ctx, st, ctx->da, ctx->N, 4, nullptr, nullptr, ctx->n_obs, ctx->N);
    if (rc) return rc;
    // summed rank-defect count over the segments
    agis_block_stats_t tmp;
    rc = fill_stats(ctx, &tmp, nullptr, (int64_t)ctx->h_segs.size(), 0, nullptr, ctx->seg_def, 0, 0);
    if (rc) return rc;
    st->defect = tmp.defect;
    st->ms = tget(ctx, T_AC) + tget(ctx, T_BAND);
    return AGIS_OK;
}
static int stats_c(agis_ctx* ctx, agis_block_stats_t* st) {
    if (!st) return AGIS_OK;
    int rc = ctx->geo_ccds > 0
                 ? fill_stats(ctx, st, ctx->dgeo, ctx->n_groups, 3, nullptr, nullptr, ctx->n_obs, ctx->n_groups)
                 : fill_stats(ctx, st, ctx->dc, ctx->n_cells, 1, nullptr, nullptr, ctx->n_obs, ctx->n_cells);
    if (rc == AGIS_OK) st->ms = tget(ctx, T_CAL);
    return rc;
}

extern "C" int agis_source_update(agis_ctx_t* ctx, agis_block_stats_t* st) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    int rc = run_source(ctx);
    if (rc) return rc;
    rc = stats_s(ctx, st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_attitude_update(agis_ctx_t* ctx, agis_block_stats_t* st) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    int rc = run_ac(ctx, true, false);
    if (rc) return rc;
    rc = stats_a(ctx, st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_calibration_update(agis_ctx_t* ctx, agis_block_stats_t* st) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    int rc = run_ac(ctx, false, true);
    if (rc) return rc;
    rc = stats_c(ctx, st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_global_update(agis_ctx_t* ctx, double dg[2]) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!ctx->cfg.ppn) return set_error(ctx, AGIS_E_STATE, "the global block needs ppn in the configuration");
    if (ctx->K > 0) {
        launch_global_solve(ctx);
        launch_apply_add(ctx, 1, ctx->gpar, ctx->dgpar);
        HIPCHK(hipGetLastError());
    }
    if (dg) HIPCHK(hipMemcpyAsync(dg, ctx->dgpar, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_set_global(agis_ctx_t* ctx, double g0) {
    CHECK_CTX();
    ++ctx->xver;
    if (!std::isfinite(g0)) return set_error(ctx, AGIS_E_INVALID_ARG, "g0 not finite");
    HIPCHK(hipMemcpyAsync(ctx->gpar, &g0, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_get_global(agis_ctx_t* ctx, double out[3]) {
    CHECK_CTX();
    if (!out) return set_error(ctx, AGIS_E_INVALID_ARG, "null output");
    HIPCHK(hipMemcpyAsync(out, ctx->gpar, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(out + 1, ctx->dgpar, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_attitude_calibration_update(agis_ctx_t* ctx, agis_block_stats_t* st_a, agis_block_stats_t* st_c) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    int rc = run_ac(ctx, true, true);
    if (rc) return rc;
    if ((rc = stats_a(ctx, st_a))) return rc;
    if ((rc = stats_c(ctx, st_c))) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_set_frame_reference(agis_ctx_t* ctx, int64_t n, const double* s_ref5, int where) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (n != ctx->n_src) return set_error(ctx, AGIS_E_SHAPE, "reference catalogue size must equal n_src");
    ++ctx->gen;
    if (!s_ref5) {
        ctx->have_ref = false;
        return AGIS_OK;
    }
    int rc = check_finite_host(ctx, s_ref5, 5 * n, where);
    if (rc) return rc;
    if (!ctx->s_ref) ALLOC(ctx->s_ref, 5 * std::max<int64_t>(n, 1), "frame reference");
    rc = copy_in(ctx, ctx->s_ref, s_ref5, 5 * n * sizeof(double), where);
    if (rc) return rc;
    ctx->have_ref = true;
    return AGIS_OK;
}

extern "C" int agis_frame_fit(agis_ctx_t* ctx, double eps_omega[6]) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (!ctx->have_ref) return set_error(ctx, AGIS_E_STATE, "no frame reference set");
    launch_frame_fit(ctx);
    HIPCHK(hipGetLastError());
    if (eps_omega) {
        HIPCHK(hipMemcpyAsync(eps_omega, ctx->eo, 6 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_frame_apply(agis_ctx_t* ctx, const double eps_omega[6]) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!eps_omega) return set_error(ctx, AGIS_E_INVALID_ARG, "null eps_omega");
    for (int e = 0; e < 6; ++e)
        if (!std::isfinite(eps_omega[e])) return set_error(ctx, AGIS_E_NUMERIC, "non-finite frame parameter");
    HIPCHK(hipMemcpyAsync(ctx->eo, eps_omega, 6 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    launch_frame_apply(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

// One S[AC] iteration followed by the frame rotation (Sect. 4.6, 6.1);
// st (may be null) receives the block statistics.
static int iterate_once(agis_ctx* ctx, agis_iter_stats_t* st) {
    tstart(ctx, T_ITER);
    int rc = run_source(ctx);
    if (rc) return rc;
    if (st && (rc = stats_s(ctx, &st->s))) return rc;
    // robust: eps_a from the residuals after the source update (Sect. 5.2.5)
    rc = run_ac(ctx, true, true, true, true, nullptr, true);
    if (rc) return rc;
    if (st && (rc = stats_a(ctx, &st->a))) return rc;
    if (st && (rc = stats_c(ctx, &st->c))) return rc;
    if (ctx->have_ref) {
        tstart(ctx, T_FRAME);
        launch_frame_fit(ctx);
        launch_frame_apply(ctx);
        HIPCHK(hipGetLastError());
        tstop(ctx, T_FRAME);
    }
    tstop(ctx, T_ITER);
    if (st) {
        if (ctx->have_ref) {
            HIPCHK(hipMemcpyAsync(st->eps_omega, ctx->eo, 6 * sizeof(double), hipMemcpyDeviceToHost,
                                  ctx->stream));
        } else {
            std::memset(st->eps_omega, 0, sizeof st->eps_omega);
        }
        HIPCHK(hipStreamSynchronize(ctx->stream));
        st->ms = tget(ctx, T_ITER);
    }
    return AGIS_OK;
}

extern "C" int agis_iterate(agis_ctx_t* ctx, int32_t n_iter, agis_iter_stats_t* per_iter) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (n_iter < 0) return set_error(ctx, AGIS_E_INVALID_ARG, "n_iter < 0");
    for (int32_t it = 0; it < n_iter; ++it) {
        int rc = iterate_once(ctx, per_iter ? per_iter + it : nullptr);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->last_ms[0] = tget(ctx, T_S);
    ctx->last_ms[1] = tget(ctx, T_AC);
    ctx->last_ms[2] = tget(ctx, T_BAND);
    ctx->last_ms[3] = tget(ctx, T_CAL);
    ctx->last_ms[4] = tget(ctx, T_FRAME);
    ctx->last_ms[5] = robust_now(ctx) ? tget(ctx, T_EPS) : 0.0;
    return AGIS_OK;
}

extern "C" int agis_autotune(agis_ctx_t* ctx, int32_t* s_group) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (ctx->n_src > 0) {
        const int64_t ns = ctx->n_src;
        double *bs = nullptr, *bv = nullptr;
        agis::SrcPrep* bp = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = AGIS_OK;
        auto release = [&]() {
            if (bs) (void)hipFree(bs);
            if (bv) (void)hipFree(bv);
            if (bp) (void)hipFree(bp);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        };
        auto restore = [&]() -> hipError_t {
            hipError_t e = hipMemcpyAsync(ctx->s, bs, 5 * ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctx->svar, bv, 5 * ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctx->prep, bp, ns * sizeof(agis::SrcPrep), hipMemcpyDeviceToDevice, ctx->stream);
            return e;
        };
        if ((rc = dalloc(ctx, &bs, 5 * ns, "tuning backup")) || (rc = dalloc(ctx, &bv, 5 * ns, "tuning backup")) ||
            (rc = dalloc(ctx, &bp, ns, "tuning backup"))) {
            release();
            return rc;
        }
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = hipMemcpyAsync(bs, ctx->s, 5 * ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(bv, ctx->svar, 5 * ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(bp, ctx->prep, ns * sizeof(agis::SrcPrep), hipMemcpyDeviceToDevice, ctx->stream);
        // the faster of two source updates, each from the saved state
        auto time_source = [&](float& best_ms) -> bool {
            bool better = false;
            for (int rep = 0; rep < 2 && e == hipSuccess && rc == AGIS_OK; ++rep) {
                e = restore();
                if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
                if (e == hipSuccess) rc = run_source(ctx);
                if (e == hipSuccess && rc == AGIS_OK) e = hipEventRecord(e1, ctx->stream);
                if (e == hipSuccess && rc == AGIS_OK) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess && rc == AGIS_OK) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && rc == AGIS_OK && ms < best_ms) {
                    best_ms = ms;
                    better = true;
                }
            }
            return better;
        };
        // lanes per source
        const int cand[3] = {8, 16, 32};
        int best = ctx->s_group;
        float best_ms = 3.0e38f;
        for (int ci = 0; ci < 3 && e == hipSuccess && rc == AGIS_OK; ++ci) {
            ctx->s_group = cand[ci];
            if (time_source(best_ms)) best = cand[ci];
        }
        ctx->s_group = best;
        // robust mode 1: the path of the S block (HBM columns, the
        // per-source LDS kernels after the rows or for the whole block, or
        // the per-source kernel with the rows in registers), and
        // for the columns the quantile kernel (both order statistics in one
        // set of passes or one after the other); the same numbers up to the
        // order of the sums (the quantiles bit for bit)
        if (ctx->cfg.robust == 1 && ctx->rcol && e == hipSuccess && rc == AGIS_OK) {
            std::vector<int64_t> h_off(ns + 1);
            std::vector<int32_t> order(ns);
            e = hipMemcpyAsync(h_off.data(), ctx->src_off, (ns + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                               ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(order.data(), ctx->src_order, ns * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            struct Path { int mode; bool pair; int cache; };
            const Path paths[7] = {{0, true, 0}, {0, false, 0}, {0, true, 1}, {0, true, 2},
                                   {1, true, 0}, {2, true, 0}, {3, true, 0}};
            Path keep{ctx->robust_s_mode, ctx->select_pair, ctx->irls_cache};
            float path_ms = 3.0e38f;
            for (int pi = 0; pi < 7 && e == hipSuccess && rc == AGIS_OK; ++pi) {
                ctx->robust_s_mode = paths[pi].mode;
                ctx->select_pair = paths[pi].pair;
                ctx->irls_cache = paths[pi].cache;
                bool need = true;
                rc = robust_plan(ctx, h_off, order, &need);
                if (rc == AGIS_OK && time_source(path_ms)) keep = paths[pi];
            }
            ctx->robust_s_mode = keep.mode;
            ctx->select_pair = keep.pair;
            ctx->irls_cache = keep.cache;
            if (rc == AGIS_OK && e == hipSuccess) {
                bool need = true;
                rc = robust_plan(ctx, h_off, order, &need);
            }
        }
        ++ctx->gen;                      // launch shapes changed
        if (e == hipSuccess) e = restore();
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        release();
        if (rc != AGIS_OK) return rc;
        if (e != hipSuccess) return hip_check(ctx, e, "autotuning");
    }
    if (s_group) *s_group = ctx->s_group;
    return AGIS_OK;
}

extern "C" int agis_get_tuning(const agis_ctx_t* ctx, int32_t out[5]) {
    if (!ctx || !out) return AGIS_E_INVALID_ARG;
    out[0] = ctx->s_group;
    out[1] = ctx->robust_s_mode;
    out[2] = ctx->select_pair ? 1 : 0;
    out[3] = ctx->eps_fused ? 1 : 0;
    out[4] = ctx->irls_cache;
    return AGIS_OK;
}

extern "C" int agis_iterate_graph(agis_ctx_t* ctx, int32_t n_iter) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (n_iter < 0) return set_error(ctx, AGIS_E_INVALID_ARG, "n_iter < 0");
    if (!ctx->graph_exec || ctx->graph_gen != ctx->gen) {
        if (ctx->graph_exec) {
            HIPCHK(hipGraphExecDestroy(ctx->graph_exec));
            ctx->graph_exec = nullptr;
        }
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        ctx->timing = false;
        const int rc = iterate_once(ctx, nullptr);
        ctx->timing = true;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
        if (rc != AGIS_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc != AGIS_OK ? rc : hip_check(ctx, ec, "end of graph capture");
        }
        const hipError_t ei = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            ctx->graph_exec = nullptr;
            return hip_check(ctx, ei, "graph instantiation");
        }
        ctx->graph_gen = ctx->gen;
    }
    for (int32_t it = 0; it < n_iter; ++it) HIPCHK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_set_excess_noise(agis_ctx_t* ctx, int64_t n, const double* eps_a2, int where) {
    CHECK_CTX();
    ++ctx->xver;
    if (!ctx->cfg.robust) return set_error(ctx, AGIS_E_STATE, "the context is not robust");
    if (n != 3 * ctx->n_buckets || !eps_a2) return set_error(ctx, AGIS_E_SHAPE, "bucket count mismatch");
    int rc = check_finite_host(ctx, eps_a2, n, where);
    if (rc) return rc;
    return copy_in(ctx, ctx->eps_a2, eps_a2, n * sizeof(double), where);
}

extern "C" int agis_get_source_noise(agis_ctx_t* ctx, int64_t n, double* eps_i2, double* D, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (ctx->cfg.robust != 2) return set_error(ctx, AGIS_E_STATE, "excess source noise needs robust mode 2");
    if (n != ctx->n_src || (n > 0 && (!eps_i2 || !D))) return set_error(ctx, AGIS_E_SHAPE, "source count mismatch");
    int rc = copy_out(ctx, eps_i2, ctx->src_eps2, n * sizeof(double), where);
    if (rc) return rc;
    return copy_out(ctx, D, ctx->src_D, n * sizeof(double), where);
}

extern "C" int agis_get_excess_noise(agis_ctx_t* ctx, int64_t n, double* eps_a2, int where) {
    CHECK_CTX();
    if (!ctx->cfg.robust) return set_error(ctx, AGIS_E_STATE, "the context is not robust");
    if (n != 3 * ctx->n_buckets || !eps_a2) return set_error(ctx, AGIS_E_SHAPE, "bucket count mismatch");
    return copy_out(ctx, eps_a2, ctx->eps_a2, n * sizeof(double), where);
}

extern "C" int agis_excess_noise_update(agis_ctx_t* ctx) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!ctx->cfg.robust) return set_error(ctx, AGIS_E_STATE, "the context is not robust");
    launch_excess_noise(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}


// --------------------------------------------------- learned extrapolation
// The buffers of the iteration schemes, all or none: a failed allocation
// releases what it had allocated.
static void learned_free(agis_ctx* ctx) {
    for (double** v : {&ctx->lh_anchor_s, &ctx->lh_ring_s, &ctx->lh_anchor_a, &ctx->lh_ring_a, &ctx->lh_anchor_c,
                       &ctx->lh_ring_c, &ctx->asi_part, &ctx->asi_out, &ctx->chi2_part, &ctx->chi2_out})
        dfree(*v);
    for (int w = 0; w < 2; ++w) {
        dfree(ctx->lf_X[w]);
        dfree(ctx->lf_scale[w]);
        dfree(ctx->lf_Y[w]);
    }
    for (int k = 0; k < 2; ++k) {
        dfree(ctx->bk_s[k]);
        dfree(ctx->bk_a[k]);
        dfree(ctx->bk_c[k]);
        dfree(ctx->bk_e[k]);
    }
}

static int learned_alloc_all(agis_ctx* ctx) {
    const int64_t ns = std::max<int64_t>(ctx->n_src, 1), na = std::max<int64_t>(ctx->N, 1);
    ALLOC(ctx->lh_anchor_s, 5 * ns, "history anchor");
    ALLOC(ctx->lh_ring_s, 4 * 5 * ns, "update history");
    ALLOC(ctx->lh_anchor_a, 4 * na, "history anchor");
    ALLOC(ctx->lh_ring_a, 4 * 4 * na, "update history");
    const int64_t nc = std::max<int64_t>(ctx->n_cells, 1);
    ALLOC(ctx->lh_anchor_c, nc, "history anchor");
    ALLOC(ctx->lh_ring_c, 4 * nc, "update history");
    ALLOC(ctx->asi_part, 2 * ((ns + 255) / 256), "accelerated iteration sums");
    ALLOC(ctx->asi_out, 2, "accelerated iteration sums");
    for (int w = 0; w < 2; ++w) {
        const int64_t n = w == 0 ? ns : na;
        ALLOC(ctx->lf_X[w], n * mlp_num_inputs(w), "features");
        ALLOC(ctx->lf_scale[w], n, "feature scales");
        ALLOC(ctx->lf_Y[w], n * mlp_num_outputs(w), "mlp outputs");
    }
    for (int k = 0; k < 2; ++k) {
        ALLOC(ctx->bk_s[k], 5 * ns, "candidate backup");
        ALLOC(ctx->bk_a[k], 4 * na, "candidate backup");
        ALLOC(ctx->bk_c[k], std::max<int64_t>(ctx->n_cells, 1), "candidate backup");
        ALLOC(ctx->bk_e[k], std::max<int64_t>(3 * ctx->n_buckets, 1), "candidate backup");
    }
    ALLOC(ctx->chi2_part, std::max<int64_t>((ctx->K + 63) / 64, 1), "chi2 partials");
    ALLOC(ctx->chi2_out, 2, "chi2");
    return AGIS_OK;
}

static int learned_alloc(agis_ctx* ctx) {
    if (ctx->chi2_out) return AGIS_OK;           // allocated last: the whole set is there
    learned_free(ctx);
    const int rc = learned_alloc_all(ctx);
    if (rc != AGIS_OK) learned_free(ctx);
    return rc;
}

static int check_which(agis_ctx* ctx, int32_t which) {
    if (which != 0 && which != 1) return set_error(ctx, AGIS_E_INVALID_ARG, "which must be 0 (sources) or 1 (knots)");
    return AGIS_OK;
}

extern "C" int agis_learned_reset(agis_ctx_t* ctx) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (ctx->geo_ccds > 0)
        return set_error(ctx, AGIS_E_STATE, "recorded updates and extrapolation: not with the geometric calibration");
    if (ctx->k.defl > 0.0)
        return set_error(ctx, AGIS_E_STATE, "recorded updates and extrapolation: not with the light deflection");
    int rc = learned_alloc(ctx);
    if (rc) return rc;
    launch_hist_anchor(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->lh_count = 0;
    return AGIS_OK;
}

extern "C" int agis_learned_record(agis_ctx_t* ctx) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (!ctx->lh_ring_s) return set_error(ctx, AGIS_E_STATE, "agis_learned_reset first");
    launch_hist_record(ctx, ctx->lh_count % 4);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ++ctx->lh_count;
    return AGIS_OK;
}

extern "C" int agis_learned_features(agis_ctx_t* ctx, int32_t which, int64_t n, float* X, float* scale, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (ctx->lh_count < 4) return set_error(ctx, AGIS_E_STATE, "fewer than four recorded updates");
    const int64_t nu = which == 0 ? ctx->n_src : ctx->N;
    if (n != nu || !X || !scale) return set_error(ctx, AGIS_E_SHAPE, "unit count mismatch");
    launch_features(ctx, which, ctx->lf_X[which], ctx->lf_scale[which]);
    HIPCHK(hipGetLastError());
    rc = copy_out(ctx, X, ctx->lf_X[which], n * mlp_num_inputs(which) * sizeof(float), where);
    if (rc) return rc;
    return copy_out(ctx, scale, ctx->lf_scale[which], n * sizeof(float), where);
}

extern "C" int agis_mlp_init(agis_ctx_t* ctx, int32_t which, uint64_t seed) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    const int F = mlp_num_inputs(which), O = mlp_num_outputs(which), H = 64;
    const int nw = mlp_num_weights(which);
    std::vector<float> w(nw, 0.0f);
    // uniform +-sqrt(6 / (fan_in + fan_out)) weights from a SplitMix64
    // stream, zero biases
    uint64_t st = seed;
    auto next = [&]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int rows, int cols) {
        const double a = std::sqrt(6.0 / (rows + cols));
        for (int e = 0; e < rows * cols; ++e) w[off + e] = (float)((2.0 * next() - 1.0) * a);
    };
    fill(0, H, F);
    fill(H * F + H, H, H);
    fill(H * F + H + H * H + H, O, H);
    HIPCHK(hipMemcpy(ctx->mlp_w[which], w.data(), nw * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(ctx->mlp_m1[which], 0, nw * sizeof(float)));
    HIPCHK(hipMemset(ctx->mlp_m2[which], 0, nw * sizeof(float)));
    ctx->mlp_t[which] = 0;
    launch_round_weights(ctx, which);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_mlp_load(agis_ctx_t* ctx, int32_t which, int64_t n, const float* w, int where) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n != mlp_num_weights(which) || !w) return set_error(ctx, AGIS_E_SHAPE, "weight count mismatch");
    rc = copy_in(ctx, ctx->mlp_w[which], w, n * sizeof(float), where);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(ctx->mlp_m1[which], 0, n * sizeof(float), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->mlp_m2[which], 0, n * sizeof(float), ctx->stream));
    ctx->mlp_t[which] = 0;
    launch_round_weights(ctx, which);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_mlp_get_weights(agis_ctx_t* ctx, int32_t which, int64_t n, float* w, int where) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n != mlp_num_weights(which) || !w) return set_error(ctx, AGIS_E_SHAPE, "weight count mismatch");
    return copy_out(ctx, w, ctx->mlp_w[which], n * sizeof(float), where);
}

// device copies of caller arrays (host) or the caller's device pointers
struct DevIn {
    std::vector<void*> own;
    ~DevIn() {
        for (void* p : own) (void)hipFree(p);
    }
};

static int dev_input(agis_ctx* ctx, DevIn& keep, const float* src, int64_t n, int where, const float** out) {
    if (where == AGIS_DEVICE) {
        *out = src;
        return AGIS_OK;
    }
    float* d = nullptr;
    int rc = dalloc(ctx, &d, (size_t)std::max<int64_t>(n, 1), "staging");
    if (rc) return rc;
    keep.own.push_back(d);
    HIPCHK(hipMemcpyAsync(d, src, n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    *out = d;
    return AGIS_OK;
}

extern "C" int agis_mlp_forward(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, float* Y, int where) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!X || !Y))) return set_error(ctx, AGIS_E_INVALID_ARG, "bad arrays");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    DevIn keep;
    const float* dX = nullptr;
    if ((rc = dev_input(ctx, keep, X, n * mlp_num_inputs(which), where, &dX))) return rc;
    float* dY = Y;
    if (where == AGIS_HOST) {
        if ((rc = dalloc(ctx, &dY, (size_t)std::max<int64_t>(n * mlp_num_outputs(which), 1), "staging"))) return rc;
        keep.own.push_back(dY);
    }
    launch_mlp_forward(ctx, which, n, dX, dY);
    HIPCHK(hipGetLastError());
    if (where == AGIS_HOST)
        HIPCHK(hipMemcpyAsync(Y, dY, n * mlp_num_outputs(which) * sizeof(float), hipMemcpyDeviceToHost,
                              ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_mlp_gradient(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T,
                                 float* grad, float* loss, int where) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n <= 0 || !X || !T || !grad || !loss) return set_error(ctx, AGIS_E_INVALID_ARG, "bad arrays");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    DevIn keep;
    const float *dX = nullptr, *dT = nullptr;
    if ((rc = dev_input(ctx, keep, X, n * mlp_num_inputs(which), where, &dX))) return rc;
    if ((rc = dev_input(ctx, keep, T, n * mlp_num_targets(which), where, &dT))) return rc;
    const int nw = mlp_num_weights(which);
    float* part = nullptr;
    if ((rc = dalloc(ctx, &part, (size_t)((n + 127) / 128) * (nw + 1), "gradient partials"))) return rc;
    keep.own.push_back(part);
    launch_mlp_grad(ctx, which, n, nullptr, dX, dT, part);
    HIPCHK(hipGetLastError());
    std::vector<float> g(nw + 1);
    HIPCHK(hipMemcpyAsync(g.data(), ctx->mlp_g[which], (nw + 1) * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (where == AGIS_HOST) {
        std::memcpy(grad, g.data(), nw * sizeof(float));
    } else {
        HIPCHK(hipMemcpy(grad, ctx->mlp_g[which], nw * sizeof(float), hipMemcpyDeviceToDevice));
    }
    *loss = g[nw];
    return AGIS_OK;
}

extern "C" int agis_mlp_train_step(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T,
                                   int where, float lr, float* loss) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n <= 0 || !X || !T || !(lr > 0.0f)) return set_error(ctx, AGIS_E_INVALID_ARG, "bad training arguments");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    DevIn keep;
    const float *dX = nullptr, *dT = nullptr;
    if ((rc = dev_input(ctx, keep, X, n * mlp_num_inputs(which), where, &dX))) return rc;
    if ((rc = dev_input(ctx, keep, T, n * mlp_num_targets(which), where, &dT))) return rc;
    const int nw = mlp_num_weights(which);
    float* part = nullptr;
    if ((rc = dalloc(ctx, &part, (size_t)((n + 127) / 128) * (nw + 1), "gradient partials"))) return rc;
    keep.own.push_back(part);
    // the whole batch, in its own order (no index list)
    launch_mlp_grad(ctx, which, n, nullptr, dX, dT, part);
    ++ctx->mlp_t[which];
    launch_adam(ctx, which, lr, ctx->mlp_t[which]);
    HIPCHK(hipGetLastError());
    if (loss) HIPCHK(hipMemcpyAsync(loss, ctx->mlp_g[which] + nw, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_mlp_train(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T, int where,
                              int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss_out) {
    CHECK_CTX();
    int rc = check_which(ctx, which);
    if (rc) return rc;
    if (n <= 0 || !X || !T || steps < 0 || batch < 1 || !(lr > 0.0f))
        return set_error(ctx, AGIS_E_INVALID_ARG, "bad training arguments");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    DevIn keep;
    const float *dX = nullptr, *dT = nullptr;
    if ((rc = dev_input(ctx, keep, X, n * mlp_num_inputs(which), where, &dX))) return rc;
    if ((rc = dev_input(ctx, keep, T, n * mlp_num_targets(which), where, &dT))) return rc;
    const int nw = mlp_num_weights(which);
    float* part = nullptr;
    int64_t* idx = nullptr;
    if ((rc = dalloc(ctx, &part, (size_t)((batch + 127) / 128) * (nw + 1), "gradient partials"))) return rc;
    keep.own.push_back(part);
    if ((rc = dalloc(ctx, &idx, (size_t)batch, "minibatch"))) return rc;
    keep.own.push_back(idx);
    for (int32_t it = 0; it < steps; ++it) {
        launch_batch_idx(ctx, batch, n, seed, (uint64_t)(ctx->mlp_t[which] + 1), idx);
        launch_mlp_grad(ctx, which, batch, idx, dX, dT, part);
        ++ctx->mlp_t[which];
        launch_adam(ctx, which, lr, ctx->mlp_t[which]);
        if (loss_out)
            HIPCHK(hipMemcpyAsync(loss_out + it, ctx->mlp_g[which] + nw, sizeof(float), hipMemcpyDeviceToHost,
                                  ctx->stream));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_chi2(agis_ctx_t* ctx, double* q) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (!q) return set_error(ctx, AGIS_E_INVALID_ARG, "null q");
    int rc = learned_alloc(ctx);
    if (rc) return rc;
    launch_chi2(ctx, ctx->chi2_part, ctx->chi2_out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(q, ctx->chi2_out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

extern "C" int agis_chi2_noalloc(agis_ctx_t* ctx, double* q, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (!q) return set_error(ctx, AGIS_E_INVALID_ARG, "null q");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    const int64_t nb = (ctx->K + 63) / 64;              // partial sums (K >= 1)
    if (nb + 1 > kScratchDoubles)
        return set_error(ctx, AGIS_E_SHAPE, "agis_chi2_noalloc: more than " +
                                                std::to_string((kScratchDoubles - 1) * 64) + " knot intervals");
    double* sp = scratch_address(ctx->device);
    if (!sp) return set_error(ctx, AGIS_E_DEVICE, "scratch array not resolved on this device");
    // every partial and the total are written before they are read: nothing
    // has to start at zero
    launch_chi2(ctx, sp, sp + nb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(q, sp + nb, sizeof(double),
                          where == AGIS_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

// Iteration state (sources, attitude, calibration and, when robust, the
// excess attitude noise) to and from backup slot k.
static void save_state(agis_ctx* ctx, int k) {
    launch_copy(ctx, 5 * ctx->n_src, ctx->s, ctx->bk_s[k]);
    launch_copy(ctx, 4 * ctx->N, ctx->a, ctx->bk_a[k]);
    launch_copy(ctx, ctx->n_cells, ctx->c, ctx->bk_c[k]);
    if (ctx->cfg.robust) launch_copy(ctx, 3 * ctx->n_buckets, ctx->eps_a2, ctx->bk_e[k]);
}

static void restore_state(agis_ctx* ctx, int k) {
    launch_copy(ctx, 5 * ctx->n_src, ctx->bk_s[k], ctx->s);
    launch_copy(ctx, 4 * ctx->N, ctx->bk_a[k], ctx->a);
    launch_copy(ctx, ctx->n_cells, ctx->bk_c[k], ctx->c);
    if (ctx->cfg.robust) launch_copy(ctx, 3 * ctx->n_buckets, ctx->bk_e[k], ctx->eps_a2);
    launch_prep_sources(ctx);
}

// x <- x + sum_k c_k u_k, c = MLP(features), for sources and attitude
// coefficients.
static void apply_candidate(agis_ctx* ctx) {
    for (int w = 0; w < 2; ++w) {
        launch_features(ctx, w, ctx->lf_X[w], ctx->lf_scale[w]);
        launch_mlp_forward(ctx, w, w == 0 ? ctx->n_src : ctx->N, ctx->lf_X[w], ctx->lf_Y[w]);
    }
    launch_apply_candidate(ctx, ctx->lf_Y[0], ctx->lf_Y[1]);
    launch_prep_sources(ctx);
}

extern "C" int agis_learned_apply(agis_ctx_t* ctx) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!ctx->lh_ring_s || ctx->lh_count < 4) return set_error(ctx, AGIS_E_STATE, "fewer than four recorded updates");
    apply_candidate(ctx);
    launch_hist_anchor(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->lh_count = 0;
    return AGIS_OK;
}

extern "C" int agis_asi_step(agis_ctx_t* ctx, int32_t stride, double lambda_max, double* lambda, double* factor) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (stride < 1 || !(lambda_max >= 0.0 && lambda_max < 1.0))
        return set_error(ctx, AGIS_E_INVALID_ARG, "stride >= 1 and 0 <= lambda_max < 1");
    if (!ctx->lh_ring_s || ctx->lh_count < 2) return set_error(ctx, AGIS_E_STATE, "fewer than two recorded updates");
    launch_asi_sums(ctx, stride, ctx->asi_part, ctx->asi_out);
    HIPCHK(hipGetLastError());
    double sums[2];
    HIPCHK(hipMemcpyAsync(sums, ctx->asi_out, sizeof sums, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // least-squares ratio of the newest to the previous parallax updates
    double lam = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
    if (!std::isfinite(lam) || lam < 0.0) lam = 0.0;
    lam = std::min(lam, lambda_max);
    const double f = lam / (1.0 - lam);
    if (f > 0.0) {
        launch_asi_apply(ctx, f);
        launch_prep_sources(ctx);
        launch_hist_anchor(ctx);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->lh_count = 0;
    }
    if (lambda) *lambda = lam;
    if (factor) *factor = f;
    return AGIS_OK;
}

// The gated learned step (two iterations); the history holds four records.
static int learned_step(agis_ctx* ctx, double* q_plain, double* q_cand, int32_t* accepted) {
    // plain: x0 -> x1 by one iteration
    save_state(ctx, 0);
    int rc = iterate_once(ctx, nullptr);
    if (rc) return rc;
    launch_chi2(ctx, ctx->chi2_part, ctx->chi2_out);
    save_state(ctx, 1);
    // candidate: x0 + s y, then one iteration
    restore_state(ctx, 0);
    apply_candidate(ctx);
    if ((rc = iterate_once(ctx, nullptr))) return rc;
    launch_chi2(ctx, ctx->chi2_part, ctx->chi2_out + 1);
    HIPCHK(hipGetLastError());
    double q[2];
    HIPCHK(hipMemcpyAsync(q, ctx->chi2_out, sizeof q, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const bool acc = std::isfinite(q[1]) && q[1] < q[0];
    if (acc) {
        // the trajectory restarts from the candidate: new history
        launch_hist_anchor(ctx);
        ctx->lh_count = 0;
    } else {
        // the plain trajectory goes on from x1 (the history keeps its
        // anchor, so the next record spans one iteration more)
        restore_state(ctx, 1);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (q_plain) *q_plain = q[0];
    if (q_cand) *q_cand = q[1];
    if (accepted) *accepted = acc ? 1 : 0;
    return AGIS_OK;
}

extern "C" int agis_learned_step(agis_ctx_t* ctx, double* q_plain, double* q_cand, int32_t* accepted) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!ctx->lh_ring_s || ctx->lh_count < 4) return set_error(ctx, AGIS_E_STATE, "fewer than four recorded updates");
    return learned_step(ctx, q_plain, q_cand, accepted);
}

extern "C" int agis_iterate_learned(agis_ctx_t* ctx, int32_t n_blocks, int32_t m, agis_learned_stats_t* per_block) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (n_blocks < 0 || m < 1) return set_error(ctx, AGIS_E_INVALID_ARG, "n_blocks >= 0 and m >= 1");
    int rc;
    if (!ctx->lh_ring_s) {
        // no history yet: it starts here
        if ((rc = learned_alloc(ctx))) return rc;
        launch_hist_anchor(ctx);
        HIPCHK(hipGetLastError());
        ctx->lh_count = 0;
    }
    for (int32_t b = 0; b < n_blocks; ++b) {
        agis_learned_stats_t st = {m, 0, 0, 0.0, 0.0};
        for (int32_t it = 0; it < m; ++it)
            if ((rc = iterate_once(ctx, nullptr))) return rc;
        launch_hist_record(ctx, ctx->lh_count % 4);
        HIPCHK(hipGetLastError());
        ++ctx->lh_count;
        if (ctx->lh_count >= 4) {
            if ((rc = learned_step(ctx, &st.q_plain, &st.q_cand, &st.accepted))) return rc;
            st.gated = 1;
            st.iterations += 2;
        }
        if (per_block) per_block[b] = st;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

// --- conjugate gradients (Sect. 4.7) ----------------------------------------
// Preconditioned CG (Polak-Ribiere) for the normal equations linearised at
// the current state.  K is the block-Jacobi form of the S, A and C blocks
// (all three at one point); r and z are evaluated at every iterate, and
// p'N p comes from one pass over the observations.

// Each buffer is allocated once; after a failed allocation a later call
// completes the set.
static int cg_alloc(agis_ctx* ctx) {
    const int64_t n = std::max<int64_t>(cg_size(ctx), 1);
    for (double** v : {&ctx->cg_r, &ctx->cg_z, &ctx->cg_p, &ctx->cg_ry, &ctx->cg_zy})
        if (!*v) ALLOC(*v, n, "cg vectors");
    if (!ctx->cg_sy) ALLOC(ctx->cg_sy, 5 * std::max<int64_t>(ctx->n_src, 1), "cg state");
    if (!ctx->cg_part) ALLOC(ctx->cg_part, 2 * 1024, "cg partial sums");
    if (!ctx->cg_qpart) ALLOC(ctx->cg_qpart, std::max<int64_t>(cg_quad_blocks(ctx), 1), "cg partial sums");
    if (!ctx->cg_out) ALLOC(ctx->cg_out, 2, "cg sums");
    return AGIS_OK;
}

// r and z at the current state, which is left as it was: the S pass writes
// its right-hand sides into r and its update into ds, then the sources are
// put back; the A/C pass and the A and C solves run at the same point and
// their updates stay in da and dc.
static int cg_evaluate(agis_ctx* ctx, double* r, double* z) {
    const int64_t ns = ctx->n_src;
    launch_copy(ctx, 5 * ns, ctx->s, ctx->cg_sy);
    ctx->rhs_s_out = r;
    int rc = run_source(ctx);
    ctx->rhs_s_out = nullptr;
    if (rc) return rc;
    launch_copy(ctx, 5 * ns, ctx->cg_sy, ctx->s);
    launch_prep_sources(ctx);
    if ((rc = run_ac(ctx, true, true, false, false, r + 5 * ns + 4 * ctx->N))) return rc;
    launch_cg_gather(ctx, r, z);
    HIPCHK(hipGetLastError());
    return AGIS_OK;
}

static int cg_read(agis_ctx* ctx, double h[2]) {
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h, ctx->cg_out, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AGIS_OK;
}

static int cg_step(agis_ctx* ctx, int32_t restart, agis_cg_stats_t* st) {
    const int64_t n = cg_size(ctx);
    double h[2];
    int rc;
    agis_cg_stats_t out = {0.0, 0.0, 0.0, 0, 0, 0.0};
    tstart(ctx, T_ITER);
    if (ctx->cg_k == 0 || ctx->cg_ver != ctx->xver) {
        // a cycle starts at x: frame rotator, then r, z and p = z
        if (ctx->have_ref) {
            tstart(ctx, T_FRAME);
            launch_frame_fit(ctx);
            launch_frame_apply(ctx);
            HIPCHK(hipGetLastError());
            tstop(ctx, T_FRAME);
        }
        if ((rc = cg_evaluate(ctx, ctx->cg_r, ctx->cg_z))) return rc;
        launch_copy(ctx, n, ctx->cg_z, ctx->cg_p);
        launch_cg_dot(ctx, ctx->cg_r, ctx->cg_z, nullptr, ctx->cg_out);
        if ((rc = cg_read(ctx, h))) return rc;
        ctx->cg_rho = h[0];
        ctx->cg_k = 1;
        out.cycle_start = 1;
    } else {
        launch_cg_quad(ctx, ctx->cg_p, ctx->cg_qpart, ctx->cg_out);
        if ((rc = cg_read(ctx, h))) return rc;
        const double pnp = h[0];
        if (!(std::isfinite(pnp) && pnp > 0.0)) {
            // no descent along p: stay at x, start a new cycle next
            ctx->cg_k = 0;
            out.breakdown = 1;
        } else {
            const double alpha = ctx->cg_rho / pnp;
            launch_cg_step_state(ctx, ctx->cg_p, alpha);
            launch_prep_sources(ctx);
            if ((rc = cg_evaluate(ctx, ctx->cg_ry, ctx->cg_zy))) return rc;
            launch_cg_dot2(ctx, ctx->cg_ry, ctx->cg_zy, ctx->cg_z, ctx->cg_out);   // r'z, r'z_old
            if ((rc = cg_read(ctx, h))) return rc;
            double beta = ctx->cg_rho != 0.0 ? (h[0] - h[1]) / ctx->cg_rho : 0.0;
            beta = std::max(beta, 0.0);
            std::swap(ctx->cg_r, ctx->cg_ry);
            std::swap(ctx->cg_z, ctx->cg_zy);
            launch_cg_direction(ctx, beta);
            HIPCHK(hipGetLastError());
            ctx->cg_rho = h[0];
            ctx->cg_k = ctx->cg_k < restart ? ctx->cg_k + 1 : 0;
            out.alpha = alpha;
            out.beta = beta;
        }
    }
    tstop(ctx, T_ITER);
    ctx->cg_ver = ctx->xver;
    if (st) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        out.rho = ctx->cg_rho;
        out.ms = tget(ctx, T_ITER);
        *st = out;
    }
    return AGIS_OK;
}

extern "C" int agis_cg_iterate(agis_ctx_t* ctx, int32_t n_eval, int32_t restart, agis_cg_stats_t* per_eval) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (n_eval < 0 || restart < 1) return set_error(ctx, AGIS_E_INVALID_ARG, "n_eval >= 0 and restart >= 1");
    if (ctx->geo_ccds > 0)
        return set_error(ctx, AGIS_E_STATE, "conjugate gradients: not with the geometric calibration");
    if (ctx->k.defl > 0.0) return set_error(ctx, AGIS_E_STATE, "conjugate gradients: not with the light deflection");
    if (robust_now(ctx))
        return set_error(ctx, AGIS_E_STATE,
                         "conjugate gradients need fixed observation weights (robust mode: freeze them first)");
    int rc = cg_alloc(ctx);
    if (rc) return rc;
    for (int32_t e = 0; e < n_eval; ++e)
        if ((rc = cg_step(ctx, restart, per_eval ? per_eval + e : nullptr))) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->last_ms[0] = tget(ctx, T_S);
    ctx->last_ms[1] = tget(ctx, T_AC);
    ctx->last_ms[2] = tget(ctx, T_BAND);
    ctx->last_ms[3] = tget(ctx, T_CAL);
    ctx->last_ms[4] = tget(ctx, T_FRAME);
    return AGIS_OK;
}

// Frozen robust weights (the switch of the hybrid scheme, Sect. 4.7): the
// weights of the A/C pass at the current parameters become fixed, and every
// block runs the plain weighted least squares with them until thawed.
extern "C" int agis_freeze_weights(agis_ctx_t* ctx, int32_t freeze) {
    CHECK_CTX();
    ++ctx->xver;
    REQUIRE_LOADED();
    if (!ctx->cfg.robust) return set_error(ctx, AGIS_E_STATE, "the context is not robust");
    if (ctx->k.defl > 0.0) return set_error(ctx, AGIS_E_STATE, "frozen weights: not with the light deflection");
    if (!freeze) {
        if (ctx->frozen) {
            ctx->frozen = false;
            ++ctx->gen;
        }
        return AGIS_OK;
    }
    if (!ctx->t_sig_eff) ALLOC(ctx->t_sig_eff, std::max<int64_t>(ctx->n_obs, 1), "frozen sigma");
    if (!ctx->s_sig_eff) ALLOC(ctx->s_sig_eff, std::max<int64_t>(ctx->n_obs, 1), "frozen sigma");
    launch_freeze_sigma(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->frozen = true;
    ++ctx->gen;
    return AGIS_OK;
}

extern "C" int agis_residuals(agis_ctx_t* ctx, double* R, int where) {
    CHECK_CTX();
    REQUIRE_LOADED();
    if (!R && ctx->n_obs > 0) return set_error(ctx, AGIS_E_INVALID_ARG, "null R");
    if (where != AGIS_HOST && where != AGIS_DEVICE) return set_error(ctx, AGIS_E_INVALID_ARG, "bad 'where'");
    double* dR = R;
    if (where == AGIS_HOST) ALLOC(dR, ctx->n_obs, "residuals");
    launch_residuals(ctx, dR);
    int rc = hip_check(ctx, hipGetLastError(), "residual kernel");
    if (rc == AGIS_OK && where == AGIS_HOST)
        rc = hip_check(ctx, hipMemcpyAsync(R, dR, ctx->n_obs * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
                       "copy residuals");
    if (rc == AGIS_OK) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
    if (where == AGIS_HOST) (void)hipFree(dR);
    return rc;
}

extern "C" int agis_problem_size(const agis_ctx_t* ctx, int64_t* n_obs, int64_t* n_src, int64_t* n_att,
                                 int64_t* n_cells, int64_t* n_segments) {
    if (!ctx) return AGIS_E_INVALID_ARG;
    if (n_obs) *n_obs = ctx->n_obs;
    if (n_src) *n_src = ctx->n_src;
    if (n_att) *n_att = ctx->N;
    if (n_cells) *n_cells = ctx->n_cells;
    if (n_segments) *n_segments = (int64_t)ctx->h_segs.size();
    return AGIS_OK;
}

extern "C" int agis_kernel_times(const agis_ctx_t* ctx, double ms[6]) {
    if (!ctx || !ms) return AGIS_E_INVALID_ARG;
    for (int e = 0; e < 6; ++e) ms[e] = ctx->last_ms[e];
    return AGIS_OK;
}
