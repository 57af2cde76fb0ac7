// Kernels of the C block, the frame rotator, residuals and statistics (the
// source update, the A/C accumulation pass and the band solve are in hot.hip).
//
//   k_calib_solve    per constraint pair: eq:normC solve and eq:calCon
//   frame rotator    eq:cond-mu3 normal equations (two-stage reduction),
//                    6x6 solve, rigorous source transform, eq:fr-q4
//
// No global atomics: every reduction has a fixed order, so results are
// bitwise reproducible run to run.
#include "agis_internal.h"

namespace agis {

namespace {

constexpr int WAVE = 64;

// pair index of (n, m), 0 <= n <= m <= 3, and entry index of (r, c), r <= c
__device__ __forceinline__ int tri4(int n, int m) { return n * 4 - (n * (n - 1)) / 2 + (m - n); }

// ---------------------------------------------------------------- sources
// pad carries the source's excess noise eps_i^2 (robust mode 2; else 0)
__global__ __launch_bounds__(256) void k_prep_sources(int64_t n_src, const double* __restrict__ s,
                                                      const double* __restrict__ src_eps2,
                                                      SrcPrep* __restrict__ prep) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_src;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double* si = s + 5 * i;
        double sa, ca, sd, cd;
        sincos(si[0], &sa, &ca);
        sincos(si[1], &sd, &cd);
        SrcPrep o;
        const double p[3] = {-sa, ca, 0.0};
        const double q[3] = {-sd * ca, -sd * sa, cd};
        o.r[0] = cd * ca;
        o.r[1] = cd * sa;
        o.r[2] = sd;
        for (int c = 0; c < 3; ++c) o.mu[c] = p[c] * si[3] + q[c] * si[4];
        o.plx = si[2];
        o.pad = src_eps2 ? src_eps2[i] : 0.0;
        prep[i] = o;
    }
}

__global__ void k_apply_add(int64_t n, double* __restrict__ x, const double* __restrict__ dx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += dx[i];
}

// ------------------------------------------------------ calibration solve
// One block per constraint pair (cells 2j, 2j+1): eq:normC with Phi = 1
// (a 1x1 system per cell, Algorithms C1-C3), then eq:calCon.  rc
// (optional) receives each cell's right-hand side -sum W R.
__global__ __launch_bounds__(256) void k_calib_solve(int64_t n_cells, const int32_t* __restrict__ cell_iv,
                                                     const int32_t* __restrict__ iv_cell,
                                                     const double* __restrict__ iv_cal, double* __restrict__ c,
                                                     double* __restrict__ dc, double* __restrict__ rc) {
    __shared__ double red[256][2];
    __shared__ double dt[2];
    const int64_t pair = blockIdx.x;
    for (int h = 0; h < 2; ++h) {
        const int64_t cell = 2 * pair + h;
        double sw = 0.0, swr = 0.0;
        if (cell < n_cells) {
            const int32_t lo = cell_iv[2 * cell], hi = cell_iv[2 * cell + 1];
            for (int32_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
                for (int f = 0; f < 2; ++f) {
                    if (iv_cell[2 * j + f] == (int32_t)cell) {
                        sw += iv_cal[(int64_t)j * IV_CAL + 2 * f];
                        swr += iv_cal[(int64_t)j * IV_CAL + 2 * f + 1];
                    }
                }
            }
        }
        red[threadIdx.x][0] = sw;
        red[threadIdx.x][1] = swr;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[threadIdx.x][0] += red[threadIdx.x + s][0];
                red[threadIdx.x][1] += red[threadIdx.x + s][1];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double U = red[0][0];
            double x = -red[0][1];
            if (rc && cell < n_cells) rc[cell] = x;
            double Um[1] = {U}, xm[1] = {x};
            small_chol_solve<1>(Um, xm);
            dt[h] = (cell < n_cells) ? xm[0] : 0.0;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t c0 = 2 * pair, c1 = 2 * pair + 1;
        if (c1 < n_cells) {
            const double z = (dt[0] + dt[1]) / 2.0;
            const double d0 = dt[0] - z, d1 = dt[1] - z;
            dc[c0] = d0;
            dc[c1] = d1;
        } else if (c0 < n_cells) {
            dc[c0] = dt[0];
        }
    }
}

// ---------------------------------------------------------- frame rotator
constexpr int FR_BLOCKS = 512;
constexpr int FR_VALS = 27;   // 21 upper entries of the 6x6 matrix + 6 rhs

// Weighted by the inverse variances of the last S update (eq:cond-mu3 rows
// for mu_a*, mu_d, alpha*, delta); zero or non-finite variance: zero weight.
__global__ __launch_bounds__(256) void k_frame_fit_partial(DevConsts k, int64_t n_src, const double* __restrict__ s,
                                                           const double* __restrict__ sref,
                                                           const double* __restrict__ svar,
                                                           double* __restrict__ part) {
    __shared__ double red[256];
    double acc[FR_VALS];
#pragma unroll
    for (int e = 0; e < FR_VALS; ++e) acc[e] = 0.0;
    const double tau = (k.t_ep - k.t_fr) / k.year_s;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_src;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double* x = s + 5 * i;
        const double* h = sref + 5 * i;
        double sa, ca, sd, cd, sah, cah, sdh, cdh;
        sincos(x[0], &sa, &ca);
        sincos(x[1], &sd, &cd);
        sincos(h[0], &sah, &cah);
        sincos(h[1], &sdh, &cdh);
        const double pt[3] = {-sa, ca, 0.0};
        const double qt[3] = {-sd * ca, -sd * sa, cd};
        const double dr[3] = {cd * ca - cdh * cah, cd * sa - cdh * sah, sd - sdh};
        double rows[4][6], rhs[4];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            rows[0][m] = 0.0;
            rows[0][3 + m] = qt[m];
            rows[1][m] = 0.0;
            rows[1][3 + m] = -pt[m];
            rows[2][m] = qt[m];
            rows[2][3 + m] = tau * qt[m];
            rows[3][m] = -pt[m];
            rows[3][3 + m] = -tau * pt[m];
        }
        rhs[0] = x[3] - h[3];
        rhs[1] = x[4] - h[4];
        rhs[2] = dot3(pt, dr);
        rhs[3] = dot3(qt, dr);
        const double* vi = svar + 5 * i;
        const double vv[4] = {vi[3], vi[4], vi[0], vi[1]};
#pragma unroll
        for (int eq = 0; eq < 4; ++eq) {
            const double wt = (vv[eq] > 0.0 && isfinite(vv[eq])) ? 1.0 / vv[eq] : 0.0;
            int e = 0;
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const double rw = rows[eq][r] * wt;
#pragma unroll
                for (int cc = r; cc < 6; ++cc) acc[e++] += rw * rows[eq][cc];
            }
#pragma unroll
            for (int r = 0; r < 6; ++r) acc[21 + r] += rows[eq][r] * wt * rhs[eq];
        }
    }
    for (int e = 0; e < FR_VALS; ++e) {
        red[threadIdx.x] = acc[e];
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * FR_VALS + e] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_frame_fit_final(const double* __restrict__ part, double* __restrict__ eo) {
    __shared__ double tot[FR_VALS];
    const int lane = threadIdx.x;
    for (int e = 0; e < FR_VALS; ++e) {
        double v = 0.0;
        for (int b = lane; b < FR_BLOCKS; b += 64) v += part[b * FR_VALS + e];
        v = wave_sum(v);
        if (lane == 0) tot[e] = v;
    }
    __syncthreads();
    if (lane == 0) {
        double U[36], x[6];
        int e = 0;
        for (int r = 0; r < 6; ++r)
            for (int cc = r; cc < 6; ++cc) U[r * 6 + cc] = tot[e++];
        for (int r = 0; r < 6; ++r) x[r] = tot[21 + r];
        small_chol_solve<6>(U, x);
        for (int r = 0; r < 6; ++r) eo[r] = x[r];
    }
}

// f(t) = Q[(t - t_fr) omega] Q(eps) (eq:fr1)
__device__ __forceinline__ void frame_quat(const DevConsts& k, const double* eo, double t, double f[4]) {
    const double dt = (t - k.t_fr) / k.year_s;
    const double wv[3] = {dt * eo[3], dt * eo[4], dt * eo[5]};
    double qw[4], qe[4];
    qrot(wv, qw);
    qrot(eo, qe);
    qmul(qw, qe, f);
}

// Rigorous transformation of the astrometric parameters (Sect. 6.1.2,
// steps 1-5) and of the source data used by the time-ordered pass.
__global__ __launch_bounds__(256) void k_frame_apply_sources(DevConsts k, int64_t n_src, const double* __restrict__ eo,
                                                             double* __restrict__ s, SrcPrep* __restrict__ prep) {
    double f[4], A[9];
    frame_quat(k, eo, k.t_ep, f);
    quat2mat(f, A);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_src;
         i += (int64_t)gridDim.x * blockDim.x) {
        double* x = s + 5 * i;
        double sa, ca, sd, cd;
        sincos(x[0], &sa, &ca);
        sincos(x[1], &sd, &cd);
        const double pt[3] = {-sa, ca, 0.0};
        const double qt[3] = {-sd * ca, -sd * sa, cd};
        const double rt[3] = {cd * ca, cd * sa, sd};
        const double wxr[3] = {eo[4] * rt[2] - eo[5] * rt[1], eo[5] * rt[0] - eo[3] * rt[2],
                               eo[3] * rt[1] - eo[4] * rt[0]};
        double mut[3];
        for (int m = 0; m < 3; ++m) mut[m] = pt[m] * x[3] + qt[m] * x[4] - wxr[m];
        double rC[3], muC[3];
        for (int m = 0; m < 3; ++m) {
            rC[m] = A[3 * m] * rt[0] + A[3 * m + 1] * rt[1] + A[3 * m + 2] * rt[2];
            muC[m] = A[3 * m] * mut[0] + A[3 * m + 1] * mut[1] + A[3 * m + 2] * mut[2];
        }
        const double alpha = atan2(rC[1], rC[0]);
        const double delta = atan2(rC[2], sqrt(rC[0] * rC[0] + rC[1] * rC[1]));
        double sa2, ca2, sd2, cd2;
        sincos(alpha, &sa2, &ca2);
        sincos(delta, &sd2, &cd2);
        const double p[3] = {-sa2, ca2, 0.0};
        const double q[3] = {-sd2 * ca2, -sd2 * sa2, cd2};
        const double pma = dot3(p, muC), pmd = dot3(q, muC);
        x[0] = alpha;
        x[1] = delta;
        x[3] = pma;
        x[4] = pmd;
        SrcPrep o;
        o.r[0] = cd2 * ca2;
        o.r[1] = cd2 * sa2;
        o.r[2] = sd2;
        for (int m = 0; m < 3; ++m) o.mu[m] = p[m] * pma + q[m] * pmd;
        o.plx = x[2];
        o.pad = prep[i].pad;                  // the source's eps_i^2 stays
        prep[i] = o;
    }
}

// eq:fr-q4 with the support mid-time eq:RF4.
__global__ __launch_bounds__(256) void k_frame_apply_attitude(DevConsts k, int64_t N, const double* __restrict__ eo,
                                                              const double* __restrict__ knots, double* __restrict__ a) {
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const double tbar = 0.5 * (knots[n] + knots[n + 4]);
        double f[4];
        frame_quat(k, eo, tbar, f);
        const double fi[4] = {-f[0], -f[1], -f[2], f[3]};
        double* an = a + 4 * n;
        const double cur[4] = {an[0], an[1], an[2], an[3]};
        double r[4];
        qmul(fi, cur, r);
        an[0] = r[0];
        an[1] = r[1];
        an[2] = r[2];
        an[3] = r[3];
    }
}

// ------------------------------------------------------------ residuals
template <bool DEFL>
__global__ __launch_bounds__(256) void k_residuals(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                   const double* __restrict__ ot, const double* __restrict__ oeta,
                                                   const int32_t* __restrict__ ocellfov,
                                                   const int32_t* __restrict__ osrc,
                                                   const int32_t* __restrict__ operm, const SrcPrep* __restrict__ prep,
                                                   const double* __restrict__ knots,
                                                   const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                   const double* __restrict__ c, double* __restrict__ R) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    if (j >= K) return;
    double a4[16], kn[6];
    for (int e = 0; e < 16; ++e) a4[e] = a[4 * j + e];
    for (int e = 0; e < 6; ++e) kn[e] = knots[j + 1 + e];
    const KnotTab kt = ktab[j];
    for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += WAVE) {
        const SrcPrep sp = prep[osrc[l]];
        const int32_t cf = ocellfov[l];
        ObsEval o;
        observe<DEFL>(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o, cf >= k.ac_cf0);
        R[operm[l]] = o.R;
    }
}

// ----------------------------------------------------------- statistics
constexpr int ST_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_stats_partial(const double* __restrict__ x, int64_t n, int w,
                                                       const double* __restrict__ extra,
                                                       const int32_t* __restrict__ iextra, double* __restrict__ part) {
    __shared__ double red[256];
    double ss[5] = {0, 0, 0, 0, 0}, mx[5] = {0, 0, 0, 0, 0}, ex = 0.0, iex = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int cc = 0; cc < w && cc < 5; ++cc) {
            const double v = x[i * w + cc];
            ss[cc] += v * v;
            mx[cc] = fmax(mx[cc], fabs(v));
        }
        if (extra) ex += extra[i];
        if (iextra) iex += (double)iextra[i];
    }
    for (int e = 0; e < 12; ++e) {
        double v = e < 5 ? ss[e] : (e < 10 ? mx[e - 5] : (e == 10 ? ex : iex));
        red[threadIdx.x] = v;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) {
                if (e >= 5 && e < 10) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
                else red[threadIdx.x] += red[threadIdx.x + st];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * 12 + e] = red[0];
        __syncthreads();
    }
}

__global__ void k_stats_final(const double* __restrict__ part, int64_t n, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double v[12] = {0};
    for (int b = 0; b < ST_BLOCKS; ++b)
        for (int e = 0; e < 12; ++e) {
            const double x = part[b * 12 + e];
            if (e >= 5 && e < 10) v[e] = fmax(v[e], x);
            else v[e] += x;
        }
    for (int e = 0; e < 5; ++e) out[e] = n > 0 ? sqrt(v[e] / (double)n) : 0.0;
    for (int e = 5; e < 12; ++e) out[e] = v[e];
}

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

inline int waves_grid(int64_t n_items, int waves_per_block) {
    return (int)((n_items + waves_per_block - 1) / waves_per_block);
}

}  // namespace

void launch_prep_sources(agis_ctx* ctx) {
    k_prep_sources<<<grid_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->n_src, ctx->s, ctx->src_eps2, ctx->prep);
}




void launch_apply_add(agis_ctx* ctx, int64_t n, double* x, const double* dx) {
    if (n > 0) k_apply_add<<<grid_for(n), 256, 0, ctx->stream>>>(n, x, dx);
}

void launch_apply_attitude(agis_ctx* ctx) {
    k_apply_add<<<grid_for(4 * ctx->N), 256, 0, ctx->stream>>>(4 * ctx->N, ctx->a, ctx->da);
}

void launch_calib_solve(agis_ctx* ctx, double* rc) {
    const int64_t pairs = (ctx->n_cells + 1) / 2;
    if (pairs == 0) return;
    k_calib_solve<<<(unsigned)pairs, 256, 0, ctx->stream>>>(ctx->n_cells, ctx->cell_iv, ctx->iv_cell, ctx->iv_cal,
                                                           ctx->c, ctx->dc, rc);
}

void launch_apply_calibration(agis_ctx* ctx) {
    k_apply_add<<<grid_for(ctx->n_cells), 256, 0, ctx->stream>>>(ctx->n_cells, ctx->c, ctx->dc);
}

void launch_frame_fit(agis_ctx* ctx) {
    k_frame_fit_partial<<<FR_BLOCKS, 256, 0, ctx->stream>>>(ctx->k, ctx->n_src, ctx->s, ctx->s_ref, ctx->svar,
                                                            ctx->red);
    k_frame_fit_final<<<1, 64, 0, ctx->stream>>>(ctx->red, ctx->eo);
}

void launch_frame_apply(agis_ctx* ctx) {
    k_frame_apply_sources<<<grid_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->k, ctx->n_src, ctx->eo, ctx->s,
                                                                         ctx->prep);
    k_frame_apply_attitude<<<grid_for(ctx->N), 256, 0, ctx->stream>>>(ctx->k, ctx->N, ctx->eo, ctx->knots, ctx->a);
}

void launch_residuals(agis_ctx* ctx, double* R) {
    if (ctx->K == 0) return;
    (ctx->k.defl > 0.0 ? k_residuals<true> : k_residuals<false>)<<<waves_grid(ctx->K, 4), 256, 0, ctx->stream>>>(
                                                                 ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta,
                                                                 ctx->t_cellfov, ctx->t_src, ctx->t_perm, ctx->prep,
                                                                 ctx->knots, ctx->ktab, ctx->a, ctx->c, R);
}

void launch_stats(agis_ctx* ctx, const double* x, int64_t n, int w, const double* extra, const int32_t* iextra,
                  double* out) {
    k_stats_partial<<<ST_BLOCKS, 256, 0, ctx->stream>>>(x, n, w, extra, iextra, ctx->red);
    k_stats_final<<<1, 64, 0, ctx->stream>>>(ctx->red, n, out);
}

}  // namespace agis
