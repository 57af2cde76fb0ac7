// Robust weighting (Sect. 5.1.2 and 5.2.5).
//
//   k_s_rows<G>     S block, pass 0: G lanes per source evaluate the model at
//                   the current parameters and store, per observation (by-source
//                   order), the design row -dR/ds (5), h = R and
//                   sigma~^2 = sigma^2 + eps_a^2(t) as seven columns in HBM.
//   k_s_sigma       one wavefront per source: half the intersextile range of
//                   its h (exact order statistics by radix selection).
//   k_s_irls<G>     the inner iteration from the stored columns: initial
//                   downweights w(h / varsigma), four solves with the weights
//                   re-derived from R = h - A d after each of the first three,
//                   then the shared per-source tail (variances, Q_i, update).
//   k_ac_resid      one wavefront per knot interval: R^2 - sigma^2 of every
//                   observation at the current parameters (by-time order).
//   k_bucket_eps    one wavefront per bucket of eps_bucket knot intervals:
//                   eps_a^2 = max(0, 68th percentile of R^2 - sigma^2) (eq e09).
//
// Quantiles are the type-7 interpolation between two exact order statistics;
// each order statistic is found by eight 8-bit radix-selection passes over an
// order-preserving integer image of the doubles, with the digit histogram in
// LDS (integer counts: the result does not depend on the order of the adds).
#include "agis_internal.h"
#include "source_block.h"

namespace agis {

namespace {

// Unsigned integer image of a double with the same order (finite values).
__device__ __forceinline__ uint64_t order_key(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double key_value(uint64_t k) {
    const uint64_t u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __builtin_bit_cast(double, u);
}

// k-th smallest (0-based, k < n) of v[0..n) by the whole 64-thread block.
__device__ double block_select(const double* __restrict__ v, int64_t n, int64_t k, uint32_t* hist) {
    const int lane = threadIdx.x;
    uint64_t prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = lane; b < 256; b += 64) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = lane; i < n; i += 64) {
            const uint64_t kk = order_key(v[i]);
            if ((kk & mask) == prefix) atomicAdd(&hist[(kk >> shift) & 255u], 1u);
        }
        __syncthreads();
        // lane owns digits 4 lane .. 4 lane + 3
        const uint32_t c0 = hist[4 * lane], c1 = hist[4 * lane + 1], c2 = hist[4 * lane + 2];
        const uint32_t c3 = hist[4 * lane + 3];
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t inc = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        const uint32_t exc = inc - tot;
        const bool mine = (int64_t)exc <= k && k < (int64_t)inc;
        int digit = 0;
        uint32_t below = exc;
        if (mine) {
            const uint32_t r = (uint32_t)(k - (int64_t)exc);
            if (r < c0) {
                digit = 0;
            } else if (r < c0 + c1) {
                digit = 1;
                below += c0;
            } else if (r < c0 + c1 + c2) {
                digit = 2;
                below += c0 + c1;
            } else {
                digit = 3;
                below += c0 + c1 + c2;
            }
            digit += 4 * lane;
        }
        const uint64_t bal = __ballot(mine);
        const int src = __ffsll((unsigned long long)bal) - 1;
        digit = __shfl(digit, src, 64);
        below = __shfl(below, src, 64);
        prefix |= (uint64_t)digit << shift;
        mask |= 0xFFull << shift;
        k -= (int64_t)below;
        __syncthreads();
    }
    return key_value(prefix);
}

// p-quantile by linear interpolation between the order statistics at
// (n - 1) p (type 7); 0 for n = 0.
__device__ double block_quantile7(const double* __restrict__ v, int64_t n, double p, uint32_t* hist) {
    if (n <= 0) return 0.0;
    const double h = (double)(n - 1) * p;
    const int64_t j = (int64_t)floor(h);
    const double xj = block_select(v, n, j, hist);
    if (j + 1 >= n) return xj;
    const double xj1 = block_select(v, n, j + 1, hist);
    return xj + (h - (double)j) * (xj1 - xj);
}

// ------------------------------------------------------------- S, pass 0
template <int G>
__global__ __launch_bounds__(256, 2) void k_s_rows(DevConsts k, int64_t n_src, const int64_t* __restrict__ off,
                                                   const double* __restrict__ ot, const double* __restrict__ oeta,
                                                   const float* __restrict__ osig, const int32_t* __restrict__ ocell,
                                                   const int32_t* __restrict__ oell,
                                                   const double* __restrict__ knots,
                                                   const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                   const double* __restrict__ c, const double* __restrict__ s,
                                                   const double* __restrict__ eps_a2, int eps_bucket,
                                                   double* __restrict__ col, int64_t n_obs) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int64_t i = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    if (i >= n_src) return;
    const double* si = s + 5 * i;
    const double alpha = si[0], delta = si[1], plx = si[2], pma = si[3], pmd = si[4];
    double sa, ca, sd, cd;
    sincos(alpha, &sa, &ca);
    sincos(delta, &sd, &cd);
    const double p[3] = {-sa, ca, 0.0};
    const double q[3] = {-sd * ca, -sd * sa, cd};
    const double r[3] = {cd * ca, cd * sa, sd};
    double mu[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) mu[cc] = p[cc] * pma + q[cc] * pmd;
    const int64_t l1 = off[i + 1];
    for (int64_t l = off[i] + gl; l < l1; l += G) {
        const int32_t ell = oell[l];
        const double sg = (double)osig[l];
        ObsEval o;
        observe(k, ot[l], oeta[l], c[ocell[l] >> 1], r, mu, plx, a + 4 * (ell - 3), knots + (ell - 2),
                ktab[ell - 3], o);
        double A[5];
        source_partials(o, p, q, r, A);
#pragma unroll
        for (int e = 0; e < 5; ++e) col[e * n_obs + l] = A[e];
        col[5 * n_obs + l] = o.R;
        col[6 * n_obs + l] = sg * sg + eps_a2[(ell - 3) / eps_bucket];
    }
}

// ------------------------------------------------ S, initial downweights
__global__ __launch_bounds__(64) void k_s_sigma(int64_t n_src, const int64_t* __restrict__ off,
                                                const double* __restrict__ h, double* __restrict__ vs) {
    __shared__ uint32_t hist[256];
    const int64_t i = blockIdx.x;
    if (i >= n_src) return;
    const int64_t l0 = off[i], n = off[i + 1] - l0;
    const double q5 = block_quantile7(h + l0, n, 5.0 / 6.0, hist);
    const double q1 = block_quantile7(h + l0, n, 1.0 / 6.0, hist);
    if (threadIdx.x == 0) vs[i] = 0.5 * (q5 - q1);
}

// ------------------------------------------------- S, inner iteration
constexpr int INNER_SOLVES = 4;

template <int G>
__global__ __launch_bounds__(256) void k_s_irls(int64_t n_src, const int64_t* __restrict__ off,
                                                const double* __restrict__ col, int64_t n_obs,
                                                const double* __restrict__ vs, double* __restrict__ s,
                                                SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                double* __restrict__ svar) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int leader = (threadIdx.x & 63) & ~(G - 1);
    const int64_t i = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = i < n_src;
    const int64_t l0 = valid ? off[i] : 0, l1 = valid ? off[i + 1] : 0;
    const double vsi = valid ? vs[i] : 0.0;
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double acc[21];
    for (int it = 0; it < INNER_SOLVES; ++it) {
#pragma unroll
        for (int e = 0; e < 21; ++e) acc[e] = 0.0;
        for (int64_t l = l0 + gl; l < l1; l += G) {
            double A[5];
#pragma unroll
            for (int e = 0; e < 5; ++e) A[e] = col[e * n_obs + l];
            const double h = col[5 * n_obs + l], s2 = col[6 * n_obs + l];
            double wl;
            if (it == 0) {
                wl = vsi > 0.0 ? down_weight(h / vsi) : 1.0;
            } else {
                double R = h;
#pragma unroll
                for (int e = 0; e < 5; ++e) R -= A[e] * d[e];
                wl = down_weight(R / sqrt(s2));
            }
            const double W = wl / s2;
            int e = 0;
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) {
                const double wa = A[rr] * W;
#pragma unroll
                for (int cc = rr; cc < 5; ++cc) acc[e++] += wa * A[cc];
            }
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) acc[15 + rr] += A[rr] * W * h;
            acc[20] += W * h * h;
        }
#pragma unroll
        for (int e = 0; e < 21; ++e) acc[e] = group_sum<G>(acc[e]);
        if (it + 1 < INNER_SOLVES) {
            // the group's leader solves; every lane of the group takes d
            double x[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (gl == 0) {
                double U[25];
                int e = 0;
                for (int rr = 0; rr < 5; ++rr)
                    for (int cc = rr; cc < 5; ++cc) U[rr * 5 + cc] = acc[e++];
                for (int rr = 0; rr < 5; ++rr) x[rr] = acc[15 + rr];
                small_chol_factor<5>(U);
                small_chol_subst<5>(U, x);
            }
#pragma unroll
            for (int e = 0; e < 5; ++e) d[e] = __shfl(x[e], leader, 64);
        }
    }
    if (!valid || gl != 0) return;
    const double* si = s + 5 * i;
    const double alpha = si[0], delta = si[1], plx = si[2], pma = si[3], pmd = si[4];
    source_finish(acc, i, alpha, delta, plx, pma, pmd, cos(delta), s, prep, ds, qsrc, sdef, svar);
}

// ------------------------------------------------ excess attitude noise
__global__ __launch_bounds__(64) void k_ac_resid(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                 const double* __restrict__ ot, const double* __restrict__ oeta,
                                                 const float* __restrict__ osig,
                                                 const int32_t* __restrict__ ocellfov,
                                                 const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                                 const double* __restrict__ knots,
                                                 const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                 const double* __restrict__ c, double* __restrict__ v) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    if (j >= K) return;
    double a4[16], kn[6];
    for (int e = 0; e < 16; ++e) a4[e] = a[4 * j + e];
    for (int e = 0; e < 6; ++e) kn[e] = knots[j + 1 + e];
    const KnotTab kt = ktab[j];
    for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
        const SrcPrep sp = prep[osrc[l]];
        ObsEval o;
        observe(k, ot[l], oeta[l], c[ocellfov[l] >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o);
        const double sg = (double)osig[l];
        v[l] = o.R * o.R - sg * sg;
    }
}

__global__ __launch_bounds__(64) void k_bucket_eps(int64_t n_buckets, int64_t K, int eps_bucket,
                                                   const int64_t* __restrict__ iv_off, const double* __restrict__ v,
                                                   double* __restrict__ eps_a2) {
    __shared__ uint32_t hist[256];
    const int64_t b = blockIdx.x;
    if (b >= n_buckets) return;
    const int64_t j0 = b * eps_bucket;
    const int64_t j1 = j0 + eps_bucket < K ? j0 + eps_bucket : K;
    const int64_t l0 = iv_off[j0], n = iv_off[j1] - l0;
    const double q = block_quantile7(v + l0, n, 0.68, hist);
    if (threadIdx.x == 0) eps_a2[b] = q > 0.0 ? q : 0.0;
}

inline unsigned groups_grid(int64_t n_items, int items_per_block) {
    return (unsigned)((n_items + items_per_block - 1) / items_per_block);
}

}  // namespace

#define AGIS_ROWS_LAUNCH(G)                                                                                      \
    k_s_rows<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                                      \
        ctx->k, ctx->n_src, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots,   \
        ctx->ktab, ctx->a, ctx->c, ctx->s, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->rcol, ctx->n_obs)
#define AGIS_IRLS_LAUNCH(G)                                                                                      \
    k_s_irls<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                                      \
        ctx->n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc, ctx->sdef, \
        ctx->svar)

void launch_source_update_robust(agis_ctx* ctx) {
    if (ctx->n_src == 0) return;
    switch (ctx->s_group) {
        case 8: AGIS_ROWS_LAUNCH(8); break;
        case 16: AGIS_ROWS_LAUNCH(16); break;
        case 32: AGIS_ROWS_LAUNCH(32); break;
        default: AGIS_ROWS_LAUNCH(64); break;
    }
    k_s_sigma<<<(unsigned)ctx->n_src, 64, 0, ctx->stream>>>(ctx->n_src, ctx->src_off, ctx->rcol + 5 * ctx->n_obs,
                                                             ctx->vs);
    switch (ctx->s_group) {
        case 8: AGIS_IRLS_LAUNCH(8); break;
        case 16: AGIS_IRLS_LAUNCH(16); break;
        case 32: AGIS_IRLS_LAUNCH(32); break;
        default: AGIS_IRLS_LAUNCH(64); break;
    }
}

void launch_excess_noise(agis_ctx* ctx) {
    if (ctx->K == 0 || ctx->n_buckets == 0) return;
    k_ac_resid<<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig,
                                                         ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots, ctx->ktab,
                                                         ctx->a, ctx->c, ctx->rcol);
    k_bucket_eps<<<(unsigned)ctx->n_buckets, 64, 0, ctx->stream>>>(ctx->n_buckets, ctx->K, ctx->cfg.eps_bucket,
                                                                   ctx->iv_off, ctx->rcol, ctx->eps_a2);
}

}  // namespace agis
