// Global block (Sect. 5.4, eq:normG) for g = (g0, g1): g0 the PPN parameter
// of eq:gammaPPN (gamma = 1 + g0, entering the model through the Sun's light
// deflection) and g1 the pseudo-parameter of a global parallax shift, solved
// with g0 and never applied (it takes up the parallax-like part of the
// residuals that would otherwise pull g0).
//
// One wavefront per knot interval evaluates the model of the interval's
// records at the current parameters with the A/C weights (robust or plain)
// and sums the five entries of the 2x2 system (N00, N01, N11, b0, b1) in a
// fixed order; one block then adds the intervals' sums in interval order and
// solves the system with the small modified Cholesky (C1-C3): the update of
// g0 and the value of g1.
#include "agis_internal.h"
#include "model.h"
#include "source_block.h"

namespace agis {
namespace {

constexpr int G_NT = 256;

template <typename SigT>
__global__ __launch_bounds__(64) void k_g_pass(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                               const double* __restrict__ ot, const double* __restrict__ oeta,
                                               const SigT* __restrict__ osig, const int32_t* __restrict__ ocellfov,
                                               const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                               const double* __restrict__ knots, const KnotTab* __restrict__ ktab,
                                               const double* __restrict__ a, const double* __restrict__ c,
                                               const double* __restrict__ eps_a2, int eps_bucket, int robust,
                                               double* __restrict__ out) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    if (j >= K) return;
    double a4[16], kn[6];
    for (int e = 0; e < 16; ++e) a4[e] = a[4 * j + e];
    for (int e = 0; e < 6; ++e) kn[e] = knots[j + 1 + e];
    const KnotTab kt = ktab[j];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
        const SrcPrep sp = prep[osrc[l]];
        const int32_t cf = ocellfov[l];
        const bool ac = cf >= k.ac_cf0;
        ObsEval o;
        observe<true>(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o, ac);
        const double sg = (double)osig[l];
        double W;
        if (robust) {
            // the A/C weight (eq:W): sigma~^2 of the record's component and
            // bucket, plus eps_i^2 in robust mode 2
            const double s2 = sg * sg + eps_a2[eps_slot(k, cf, j, eps_bucket)] + (robust == 2 ? sp.pad : 0.0);
            W = down_weight(o.R / sqrt(s2)) / s2;
        } else {
            W = rcp_nr(sg * sg);
        }
        double ag, ap;
        global_partials(o, sp.r, ag, ap, ac);
        s[0] += ag * W * ag;
        s[1] += ag * W * ap;
        s[2] += ap * W * ap;
        s[3] += ag * W * o.R;
        s[4] += ap * W * o.R;
    }
#pragma unroll
    for (int e = 0; e < 5; ++e) {
        const double v = wave_sum(s[e]);
        if (lane == 0) out[5 * j + e] = v;
    }
}

// The intervals' sums added in interval order (each thread a strided run,
// then the threads in order), the 2x2 system solved: dg = (d g0, g1).
__global__ __launch_bounds__(G_NT) void k_g_solve(int64_t K, const double* __restrict__ in, double* __restrict__ dg) {
    __shared__ double red[G_NT][5];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = threadIdx.x; j < K; j += G_NT)
#pragma unroll
        for (int e = 0; e < 5; ++e) s[e] += in[5 * j + e];
#pragma unroll
    for (int e = 0; e < 5; ++e) red[threadIdx.x][e] = s[e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < G_NT; ++i)
#pragma unroll
        for (int e = 0; e < 5; ++e) t[e] += red[i][e];
    double U[4] = {t[0], t[1], t[1], t[2]};
    double x[2] = {t[3], t[4]};
    small_chol_solve<2>(U, x);
    dg[0] = x[0];
    dg[1] = x[1];
}

}  // namespace

void launch_global_solve(agis_ctx* ctx) {
    if (ctx->K == 0 || !ctx->cfg.ppn) return;
    const bool frozen = ctx->frozen;
#define AGIS_G_ARGS(SIG)                                                                                           \
    ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, SIG, ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots,      \
        ctx->ktab, ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, frozen ? 0 : robust_now(ctx), ctx->g_iv
    if (frozen)
        k_g_pass<double><<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(AGIS_G_ARGS(ctx->t_sig_eff));
    else
        k_g_pass<float><<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(AGIS_G_ARGS(ctx->t_sig));
#undef AGIS_G_ARGS
    k_g_solve<<<1, G_NT, 0, ctx->stream>>>(ctx->K, ctx->g_iv, ctx->dgpar);
}

}  // namespace agis
