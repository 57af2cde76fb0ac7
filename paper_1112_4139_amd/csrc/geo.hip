// Large-scale geometric calibration (Sect. 3.4, eq:etazeta, the large-scale
// terms): per calibration cell (day and field of view) and CCD three
// coefficients of the shifted Legendre polynomials L*_0..2 in the
// across-scan pixel coordinate mu, x = (mu - 13.5) / 1966, in place of one
// offset per cell; optionally the across-scan term, three coefficients per
// AC cell (field of view and long interval) and CCD.
//
// The term enters the residual additively (eq:resAL, eq:resAC): R = eta_obs
// + sum_r c_r L*_r(x) - eta (zeta across scan).  The stored observed angles
// of both orders therefore carry it -- eta = eta_obs + term, refreshed
// whenever the coefficients change -- and every pass reads them unchanged,
// with the per-cell offsets held at zero.  The C block (Sect. 5.3, eq:normC with
// eq:pdC: dR/dc_r = L*_r(x)) is block-diagonal in groups of three
// coefficients (a cell and a CCD).  The records with a group are given a
// second order at load, by group and time within a group (a stable radix
// sort of the group indices); the A/C pass writes each record's W and W R
// at its place in that order, so that one block per group sums W L_r L_s and
// W R L_r over a contiguous range in a fixed order; one thread per
// constraint set then solves the set's 3x3 systems (the small modified
// Cholesky) and applies eq:calCon for its constraint, eq:cc1 (the AL
// constant terms of a day's two cells and all CCDs sum to zero) or eq:cc3
// (the AC constant terms of an AC cell's CCDs sum to zero): their mean is
// removed.
#include <hipcub/hipcub.hpp>

#include "agis_internal.h"
#include "model.h"

namespace agis {
namespace {

template <typename T>
int dalloc(agis_ctx* ctx, T** p, size_t n, const char* what) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(ctx, AGIS_E_OOM, std::string("device allocation failed: ") + what);
    }
    return AGIS_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

__device__ __forceinline__ double shifted_legendre(int r, double x) {
    return r == 0 ? 1.0 : (r == 1 ? 2.0 * x - 1.0 : 6.0 * x * x - 6.0 * x + 1.0);
}

__device__ __forceinline__ double geo_x(float mu) { return ((double)mu - 13.5) / 1966.0; }

// Group index and pixel coordinate of every record in time order from the
// input columns (t_perm: time index -> input index): an along-scan record's
// cell and CCD; with ac_cell an across-scan record's AC cell and CCD after
// the n_cells n_ccd AL groups; -1 for an across-scan record without it.
// Flags: 1 a CCD index out of range, 2 a coordinate not in [13.5, 1979.5],
// 4 an AC cell out of range.
__global__ void k_geo_index(int64_t n, const int32_t* __restrict__ t_perm, const int32_t* __restrict__ t_cellfov,
                            int32_t n_cells, const int8_t* __restrict__ ccd_in, const float* __restrict__ mu_in,
                            const int32_t* __restrict__ ac_cell_in, int32_t n_ac_cells, int32_t n_ccd,
                            int32_t* __restrict__ g_out, float* __restrict__ mu_out, int* __restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = t_perm[i];
        const int32_t cell = t_cellfov[i] >> 1;
        const float mu = mu_in[j];
        int32_t g = -1;
        int32_t base = -1;                       // the record's cell among the groups' cells
        if (cell < n_cells) {
            base = cell;
        } else if (ac_cell_in) {
            const int32_t ac = ac_cell_in[j];
            if (ac < 0 || ac >= n_ac_cells) atomicOr(flags, 4);
            else base = n_cells + ac;
        }
        if (base >= 0 || (cell >= n_cells && ac_cell_in)) {
            const int c = ccd_in[j];
            if (c < 0 || c >= n_ccd) atomicOr(flags, 1);
            else if (base >= 0) g = base * n_ccd + c;
            if (!(mu >= 13.5f && mu <= 1979.5f)) atomicOr(flags, 2);
        }
        g_out[i] = g;
        mu_out[i] = mu;
    }
}

template <typename T>
__global__ void k_geo_gather(int64_t n, const int32_t* __restrict__ from, const T* __restrict__ src,
                             T* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[from[i]];
}

// eta = eta_obs + sum_r c_r L*_r(x) of the record's group (nothing across
// scan), the sum taken from r = 0 up.
__global__ void k_geo_eta(int64_t n, const double* __restrict__ eta0, const int32_t* __restrict__ g,
                          const float* __restrict__ mu, const double* __restrict__ geo, double* __restrict__ eta) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t gi = g[i];
        double v = 0.0;
        if (gi >= 0) {
            const double x = geo_x(mu[i]);
            const double* c = geo + 3 * (int64_t)gi;
            v = c[0] * shifted_legendre(0, x);
            v += c[1] * shifted_legendre(1, x);
            v += c[2] * shifted_legendre(2, x);
        }
        eta[i] = eta0[i] + v;
    }
}

// Sort keys of the group order: the group, or n_groups without one (last).
__global__ void k_geo_keys(int64_t n, const int32_t* __restrict__ g, int32_t n_groups, uint32_t* __restrict__ key,
                           int32_t* __restrict__ idx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = g[i] >= 0 ? (uint32_t)g[i] : (uint32_t)n_groups;
        idx[i] = (int32_t)i;
    }
}

// From the sorted keys and time indices: each time-order record's place in
// the group order (-1 for a record without a group) and the group order's
// coordinates.
__global__ void k_geo_order(int64_t n, const uint32_t* __restrict__ key, const int32_t* __restrict__ idx,
                            uint32_t n_groups, const float* __restrict__ t_mu, int32_t* __restrict__ pos,
                            float* __restrict__ mu_g) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = idx[k];
        const bool in = key[k] < n_groups;
        pos[i] = in ? (int32_t)k : -1;
        if (in) mu_g[k] = t_mu[i];
    }
}

// off[g] = the first place of group g in the sorted keys (g = 0..n_groups).
__global__ void k_geo_offsets(int64_t n, const uint32_t* __restrict__ key, int64_t n_groups,
                              int64_t* __restrict__ off) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g <= n_groups;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)key[mid] < g) lo = mid + 1;
            else hi = mid;
        }
        off[g] = lo;
    }
}

constexpr int GEO_NT = 256;

// Normal equations of one group (block): its contiguous range of the group
// order, each thread summing its strided records, then a fixed-order block
// sum.  out: [group][9] = N00 N01 N02 N11 N12 N22 b0 b1 b2 with
// N = sum W L L', b = -sum W R L.
__global__ __launch_bounds__(GEO_NT) void k_geo_sums(int64_t n_groups, const int64_t* __restrict__ off,
                                                     const float* __restrict__ mu, const double* __restrict__ wr,
                                                     double* __restrict__ out) {
    __shared__ double red[(GEO_NT / 64) * 9];
    const int64_t gi = blockIdx.x;
    if (gi >= n_groups) return;
    const int64_t l0 = off[gi], l1 = off[gi + 1];
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t l = l0 + threadIdx.x; l < l1; l += GEO_NT) {
        const double W = wr[2 * l], WR = wr[2 * l + 1];
        const double x = geo_x(mu[l]);
        double L[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) L[r] = shifted_legendre(r, x);
        s[0] += L[0] * W * L[0];
        s[1] += L[0] * W * L[1];
        s[2] += L[0] * W * L[2];
        s[3] += L[1] * W * L[1];
        s[4] += L[1] * W * L[2];
        s[5] += L[2] * W * L[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) s[6 + r] -= L[r] * WR;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double v = wave_sum(s[e]);
        if (lane == 0) red[wv * 9 + e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < GEO_NT / 64; ++w) t += red[w * 9 + threadIdx.x];
        out[9 * gi + threadIdx.x] = t;
    }
}

// One thread per constraint set of per_set consecutive groups from group
// first: their 3x3 solves, then eq:calCon for its constraint (the set's
// mean constant term removed).  AL: a day's 2 n_ccd groups (eq:cc1); AC: an
// AC cell's n_ccd groups (eq:cc3).
__global__ void k_geo_solve(int64_t n_sets, int64_t first, int32_t per_set, const double* __restrict__ sums,
                            double* __restrict__ dgeo) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_sets;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g0 = first + j * per_set, per_day = per_set;
        double mean = 0.0;
        for (int64_t k = 0; k < per_day; ++k) {
            const double* s = sums + 9 * (g0 + k);
            double U[9] = {s[0], s[1], s[2], s[1], s[3], s[4], s[2], s[4], s[5]};
            double x[3] = {s[6], s[7], s[8]};
            small_chol_solve<3>(U, x);
            double* d = dgeo + 3 * (g0 + k);
            d[0] = x[0];
            d[1] = x[1];
            d[2] = x[2];
            mean += x[0];
        }
        mean /= (double)per_day;
        for (int64_t k = 0; k < per_day; ++k) dgeo[3 * (g0 + k)] -= mean;
    }
}

inline unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

#define HIPCHK(expr)                                            \
    do {                                                        \
        int rc_ = hip_check(ctx, (expr), #expr);                \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

#define ALLOC(p, n, what)                                       \
    do {                                                        \
        int rc_ = dalloc(ctx, &(p), (size_t)(n), what);         \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

void launch_geo_eta(agis_ctx* ctx) {
    if (ctx->geo_ccds <= 0 || ctx->n_obs == 0) return;
    k_geo_eta<<<grid_for(ctx->n_obs), 256, 0, ctx->stream>>>(ctx->n_obs, ctx->t_eta0, ctx->t_geo_g, ctx->t_geo_mu,
                                                             ctx->geo, ctx->t_eta);
    k_geo_eta<<<grid_for(ctx->n_obs), 256, 0, ctx->stream>>>(ctx->n_obs, ctx->s_eta0, ctx->s_geo_g, ctx->s_geo_mu,
                                                             ctx->geo, ctx->s_eta);
}

void launch_geo_solve(agis_ctx* ctx) {
    if (ctx->geo_ccds <= 0 || ctx->n_groups == 0) return;
    k_geo_sums<<<(unsigned)ctx->n_groups, GEO_NT, 0, ctx->stream>>>(ctx->n_groups, ctx->geo_off, ctx->geo_mu_g,
                                                                    ctx->geo_wr, ctx->geo_sums);
    const int64_t n_days = ctx->n_cells / 2;
    k_geo_solve<<<grid_for(n_days), 256, 0, ctx->stream>>>(n_days, 0, 2 * ctx->geo_ccds, ctx->geo_sums, ctx->dgeo);
    if (ctx->geo_ac_cells > 0)
        k_geo_solve<<<grid_for(ctx->geo_ac_cells), 256, 0, ctx->stream>>>(
            ctx->geo_ac_cells, ctx->n_cells * ctx->geo_ccds, ctx->geo_ccds, ctx->geo_sums, ctx->dgeo);
}

// The group order of the along-scan records (time order within a group):
// geo_pos, geo_mu_g and geo_off from the time-order groups t_geo_g.
static int build_group_order(agis_ctx* ctx) {
    const int64_t n = ctx->n_obs, ng = ctx->n_groups;
    hipStream_t st = ctx->stream;
    uint32_t *k_in = nullptr, *k_out = nullptr;
    int32_t *v_in = nullptr, *v_out = nullptr;
    uint8_t* temp = nullptr;
    auto done = [&](int rc) {
        dfree(k_in);
        dfree(k_out);
        dfree(v_in);
        dfree(v_out);
        dfree(temp);
        return rc;
    };
    int rc;
    if ((rc = dalloc(ctx, &k_in, (size_t)n, "group order keys")) || (rc = dalloc(ctx, &k_out, (size_t)n, "group order keys")) ||
        (rc = dalloc(ctx, &v_in, (size_t)n, "group order")) || (rc = dalloc(ctx, &v_out, (size_t)n, "group order")))
        return done(rc);
    const int end_bit = 32 - __builtin_clz((unsigned)ng);       // keys 0..ng
    size_t tb = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k_in, k_out, v_in, v_out, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return done(hip_check(ctx, e, "group order sort"));
    if ((rc = dalloc(ctx, &temp, tb, "group order sort"))) return done(rc);
    k_geo_keys<<<grid_for(n), 256, 0, st>>>(n, ctx->t_geo_g, (int32_t)ng, k_in, v_in);
    e = hipcub::DeviceRadixSort::SortPairs(temp, tb, k_in, k_out, v_in, v_out, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return done(hip_check(ctx, e, "group order sort"));
    k_geo_order<<<grid_for(n), 256, 0, st>>>(n, k_out, v_out, (uint32_t)ng, ctx->t_geo_mu, ctx->geo_pos,
                                             ctx->geo_mu_g);
    k_geo_offsets<<<grid_for(ng + 1), 256, 0, st>>>(n, k_out, ng, ctx->geo_off);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);       // before the temporaries go
    return done(e == hipSuccess ? AGIS_OK : hip_check(ctx, e, "group order"));
}

int load_geometry(agis_ctx* ctx, const int8_t* ccd, const float* mu, int32_t n_ccd, const int32_t* ac_cell,
                  int32_t n_ac_cells, int where) {
    const int64_t n = ctx->n_obs;
    hipStream_t st = ctx->stream;
    const int8_t* ccd_d = ccd;
    const float* mu_d = mu;
    const int32_t* ac_d = n_ac_cells > 0 ? ac_cell : nullptr;
    int8_t* ccd_tmp = nullptr;
    float* mu_tmp = nullptr;
    int32_t* ac_tmp = nullptr;
    auto release = [&]() {
        if (ccd_tmp) (void)hipFree(ccd_tmp);
        if (mu_tmp) (void)hipFree(mu_tmp);
        if (ac_tmp) (void)hipFree(ac_tmp);
    };
    if (where == AGIS_HOST && n > 0) {
        int rc = dalloc(ctx, &ccd_tmp, (size_t)n, "geometry ccd");
        if (rc == AGIS_OK) rc = dalloc(ctx, &mu_tmp, (size_t)n, "geometry mu");
        if (rc == AGIS_OK && ac_d) rc = dalloc(ctx, &ac_tmp, (size_t)n, "geometry AC cells");
        if (rc != AGIS_OK) {
            release();
            return rc;
        }
        hipError_t e = hipMemcpyAsync(ccd_tmp, ccd, n * sizeof(int8_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(mu_tmp, mu, n * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && ac_d) e = hipMemcpyAsync(ac_tmp, ac_cell, n * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            release();
            return hip_check(ctx, e, "geometry upload");
        }
        ccd_d = ccd_tmp;
        mu_d = mu_tmp;
        if (ac_d) ac_d = ac_tmp;
    }
    const int32_t n_ac = ac_d ? n_ac_cells : 0;
    const int64_t ng = (ctx->n_cells + n_ac) * n_ccd;
    if (ng >= INT32_MAX || n > INT32_MAX) {
        release();
        return set_error(ctx, AGIS_E_INVALID_ARG, "agis_load_geometry: more than 2^31 - 1 records or groups");
    }
    auto fail = [&](int rc) {
        release();
        return rc;
    };
    int rc = AGIS_OK;
#define GALLOC(p, cnt, what)                                                 \
    if (!(p) && (rc = dalloc(ctx, &(p), (size_t)std::max<int64_t>(cnt, 1), what)) != AGIS_OK) return fail(rc)
    GALLOC(ctx->t_geo_g, n, "geometry groups");
    GALLOC(ctx->s_geo_g, n, "geometry groups");
    GALLOC(ctx->t_geo_mu, n, "geometry mu");
    GALLOC(ctx->s_geo_mu, n, "geometry mu");
    GALLOC(ctx->t_eta0, n, "observed eta");
    GALLOC(ctx->s_eta0, n, "observed eta");
    GALLOC(ctx->geo_wr, 2 * n, "geometry weights");
    GALLOC(ctx->geo_pos, n, "group order");
    GALLOC(ctx->geo_mu_g, n, "group order mu");
    GALLOC(ctx->geo_flags, 1, "geometry flags");
#undef GALLOC
    if (ctx->geo_ccds != n_ccd || ctx->geo_ac_cells != n_ac || !ctx->geo) {
        if (ctx->geo) {
            dfree(ctx->geo);
            dfree(ctx->dgeo);
            dfree(ctx->geo_sums);
            dfree(ctx->geo_off);
        }
        if ((rc = dalloc(ctx, &ctx->geo, (size_t)std::max<int64_t>(3 * ng, 1), "geometric calibration")) ||
            (rc = dalloc(ctx, &ctx->dgeo, (size_t)std::max<int64_t>(3 * ng, 1), "geometric update")) ||
            (rc = dalloc(ctx, &ctx->geo_sums, (size_t)std::max<int64_t>(9 * ng, 1), "geometric sums")) ||
            (rc = dalloc(ctx, &ctx->geo_off, (size_t)(ng + 1), "group offsets")))
            return fail(rc);
    }
    hipError_t e = hipMemsetAsync(ctx->geo_flags, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->geo, 0, std::max<int64_t>(3 * ng, 1) * sizeof(double), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->dgeo, 0, std::max<int64_t>(3 * ng, 1) * sizeof(double), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->geo_off, 0, (ng + 1) * sizeof(int64_t), st);
    if (e != hipSuccess) return fail(hip_check(ctx, e, "geometry clear"));
    if (n > 0) {
        k_geo_index<<<grid_for(n), 256, 0, st>>>(n, ctx->t_perm, ctx->t_cellfov, (int32_t)ctx->n_cells, ccd_d, mu_d,
                                                  ac_d, n_ac, n_ccd, ctx->t_geo_g, ctx->t_geo_mu, ctx->geo_flags);
        k_geo_gather<int32_t><<<grid_for(n), 256, 0, st>>>(n, ctx->s_from_t, ctx->t_geo_g, ctx->s_geo_g);
        k_geo_gather<float><<<grid_for(n), 256, 0, st>>>(n, ctx->s_from_t, ctx->t_geo_mu, ctx->s_geo_mu);
    }
    e = hipGetLastError();
    int flags = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, ctx->geo_flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess) return hip_check(ctx, e, "geometry load");
    if (flags) {
        // the group columns now hold the rejected input: back to the cell
        // offsets (held at zero) and the observed angles as loaded
        if (ctx->geo_ccds > 0 && n > 0) {
            HIPCHK(hipMemcpyAsync(ctx->t_eta, ctx->t_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(ctx->s_eta, ctx->s_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        ctx->geo_ccds = 0;
        ctx->geo_ac_cells = 0;
        ctx->n_groups = 0;
        std::string m = "agis_load_geometry:";
        if (flags & 1) m += " ccd index outside [0, n_ccd);";
        if (flags & 2) m += " across-scan pixel coordinate outside [13.5, 1979.5];";
        if (flags & 4) m += " AC calibration cell outside [0, n_ac_cells);";
        return set_error(ctx, AGIS_E_INVALID_ARG, m);
    }
    // the observed angles as loaded (the first load of the geometry keeps
    // them; a later one keeps the copies it already holds)
    if (ctx->geo_ccds == 0 && n > 0) {
        HIPCHK(hipMemcpyAsync(ctx->t_eta0, ctx->t_eta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->s_eta0, ctx->s_eta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    ctx->geo_ccds = n_ccd;
    ctx->geo_ac_cells = n_ac;
    ctx->n_groups = ng;
    if (n > 0 && (rc = build_group_order(ctx)) != AGIS_OK) {
        // back to the cell offsets and the observed angles as loaded
        (void)hipMemcpyAsync(ctx->t_eta, ctx->t_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(ctx->s_eta, ctx->s_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        (void)hipStreamSynchronize(st);
        ctx->geo_ccds = 0;
        ctx->geo_ac_cells = 0;
        ctx->n_groups = 0;
        return rc;
    }
    // the per-cell offsets are replaced by the geometric terms
    HIPCHK(hipMemsetAsync(ctx->c, 0, (ctx->n_cells + 1) * sizeof(double), st));
    launch_geo_eta(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return AGIS_OK;
}

#undef HIPCHK
#undef ALLOC

}  // namespace agis
