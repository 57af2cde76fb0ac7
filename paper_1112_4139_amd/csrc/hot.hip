// The three kernels that carry the iteration's cost.
//
//   k_source_update<G>  S block (Sect. 5.1).  G lanes per source stream the
//                       source's observations (by-source store), evaluate the
//                       model and the design row (Sect. 5.1.3) and accumulate
//                       the 15 + 5 sums of eq:normS in registers; a butterfly
//                       over the G lanes reduces them; one lane per source
//                       runs Algorithms C1-C3 on the 5x5 system and applies
//                       the update.
//   k_ac_pass<G>        A/C accumulation (Sect. 5.2.1, 5.2.4, 5.3).  G lanes per
//                       knot interval stream the time-ordered store at
//                       (s^(k+1), a^(k), c^(k)); per interval they produce the
//                       10 block pairs x 10 unique entries of eq:normAmod, its
//                       16 right-hand-side entries and the per-fov calibration
//                       sums of eq:normC.
//   k_band_solve        A solve (Sect. 5.2.2, App. C): one wavefront per segment;
//                       right-looking modified band Cholesky (Algorithm C1 with
//                       C2 folded in as an extra column) over a sliding window
//                       of 16 unknowns in LDS, with the per-interval sums
//                       prefetched into an LDS ring one coefficient block
//                       ahead; then C3 with the factor rows prefetched 16 rows
//                       ahead; the segment keeps its selected coefficients.
//
// Each lane walks its item's observations with stride G and loads the next
// observation's columns while the current one is evaluated.  No global
// atomics; all sums have a fixed order.
#include "agis_internal.h"

namespace agis {

namespace {

// pair index of (n, m), 0 <= n <= m <= 3 (also the entry index of (r, c))
__host__ __device__ __forceinline__ int tri4(int n, int m) { return n * 4 - (n * (n - 1)) / 2 + (m - n); }

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// ------------------------------------------------------------------ S block
template <int G>
__global__ __launch_bounds__(256) void k_source_update(DevConsts k, int64_t n_src, const int64_t* __restrict__ off,
                                                       const double* __restrict__ ot, const double* __restrict__ oeta,
                                                       const float* __restrict__ osig,
                                                       const int32_t* __restrict__ ocell,
                                                       const int32_t* __restrict__ oell,
                                                       const double* __restrict__ knots, const double* __restrict__ a,
                                                       const double* __restrict__ c, double* __restrict__ s,
                                                       SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                       double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                       double* __restrict__ svar) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int64_t i = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = i < n_src;
    double alpha = 0.0, delta = 0.0, plx = 0.0, pma = 0.0, pmd = 0.0;
    int64_t l0 = 0, l1 = 0;
    if (valid) {
        const double* si = s + 5 * i;
        alpha = si[0];
        delta = si[1];
        plx = si[2];
        pma = si[3];
        pmd = si[4];
        l0 = off[i];
        l1 = off[i + 1];
    }
    double sa, ca, sd, cd;
    sincos(alpha, &sa, &ca);
    sincos(delta, &sd, &cd);
    const double p[3] = {-sa, ca, 0.0};
    const double q[3] = {-sd * ca, -sd * sa, cd};
    const double r[3] = {cd * ca, cd * sa, sd};
    double mu[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) mu[cc] = p[cc] * pma + q[cc] * pmd;

    double acc[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) acc[e] = 0.0;
    int64_t l = l0 + gl;
    // current and next observation columns (software prefetch)
    double t_c = 0.0, e_c = 0.0;
    float s_c = 1.0f;
    int32_t c_c = 0, ell_c = 3;
    if (l < l1) {
        t_c = ot[l];
        e_c = oeta[l];
        s_c = osig[l];
        c_c = ocell[l];
        ell_c = oell[l];
    }
    for (; l < l1; l += G) {
        const int64_t ln = l + G;
        double t_n = 0.0, e_n = 0.0;
        float s_n = 1.0f;
        int32_t c_n = 0, ell_n = 3;
        if (ln < l1) {
            t_n = ot[ln];
            e_n = oeta[ln];
            s_n = osig[ln];
            c_n = ocell[ln];
            ell_n = oell[ln];
        }
        ObsEval o;
        observe(k, t_c, e_c, c[c_c >> 1], r, mu, plx, a + 4 * (ell_c - 3), knots + (ell_c - 2), o);
        double A[5];
        source_partials(o, p, q, r, A);
        const double sg = (double)s_c;
        const double W = 1.0 / (sg * sg);
        int e = 0;
#pragma unroll
        for (int rr = 0; rr < 5; ++rr) {
            const double wa = W * A[rr];
#pragma unroll
            for (int cc = rr; cc < 5; ++cc) acc[e++] += wa * A[cc];
        }
#pragma unroll
        for (int rr = 0; rr < 5; ++rr) acc[15 + rr] += W * A[rr] * o.R;
        acc[20] += W * o.R * o.R;
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        c_c = c_n;
        ell_c = ell_n;
    }
#pragma unroll
    for (int e = 0; e < 21; ++e) acc[e] = group_sum<G>(acc[e]);
    if (!valid || gl != 0) return;
    double U[25], N[25], x[5];
    int e = 0;
    for (int rr = 0; rr < 5; ++rr)
        for (int cc = rr; cc < 5; ++cc) {
            U[rr * 5 + cc] = acc[e];
            N[rr * 5 + cc] = acc[e];
            N[cc * 5 + rr] = acc[e];
            ++e;
        }
    for (int rr = 0; rr < 5; ++rr) x[rr] = acc[15 + rr];
    const int d = small_chol_factor<5>(U);
    small_chol_subst<5>(U, x);
    // diagonal of the inverse normal matrix, the first-order variances of
    // the five parameters (Sect. 5.1.1): C2 and C3 on the unit vectors
#pragma unroll
    for (int kk = 0; kk < 5; ++kk) {
        double ev[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        ev[kk] = 1.0;
        small_chol_subst<5>(U, ev);
        svar[5 * i + kk] = d > 0 ? 0.0 : ev[kk];
    }
    // Q_i = h'Wh - 2 d'b + d'N d (eq:Qi)
    double dNd = 0.0, db = 0.0;
    for (int rr = 0; rr < 5; ++rr) {
        double t = 0.0;
        for (int cc = 0; cc < 5; ++cc) t += N[rr * 5 + cc] * x[cc];
        dNd += x[rr] * t;
        db += x[rr] * acc[15 + rr];
    }
    qsrc[i] = acc[20] - 2.0 * db + dNd;
    sdef[i] = d;
    for (int rr = 0; rr < 5; ++rr) ds[5 * i + rr] = x[rr];
    const double na = alpha + x[0] / cd, nd = delta + x[1];
    const double npl = plx + x[2], npa = pma + x[3], npd = pmd + x[4];
    double* si = s + 5 * i;
    si[0] = na;
    si[1] = nd;
    si[2] = npl;
    si[3] = npa;
    si[4] = npd;
    double sa2, ca2, sd2, cd2;
    sincos(na, &sa2, &ca2);
    sincos(nd, &sd2, &cd2);
    SrcPrep pr;
    const double p2[3] = {-sa2, ca2, 0.0};
    const double q2[3] = {-sd2 * ca2, -sd2 * sa2, cd2};
    pr.r[0] = cd2 * ca2;
    pr.r[1] = cd2 * sa2;
    pr.r[2] = sd2;
    for (int cc = 0; cc < 3; ++cc) pr.mu[cc] = p2[cc] * npa + q2[cc] * npd;
    pr.plx = npl;
    pr.pad = 0.0;
    prep[i] = pr;
}

// ------------------------------------------------------------- A/C pass
template <int G>
__global__ __launch_bounds__(256) void k_ac_pass(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                 const double* __restrict__ ot, const double* __restrict__ oeta,
                                                 const float* __restrict__ osig,
                                                 const int32_t* __restrict__ ocellfov,
                                                 const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                                 const double* __restrict__ knots, const double* __restrict__ a,
                                                 const double* __restrict__ c, double* __restrict__ iv_sums,
                                                 double* __restrict__ iv_cal) {
    constexpr int GPB = 256 / G;
    __shared__ double sh_a[GPB][16];
    __shared__ double sh_k[GPB][6];
    const int gl = threadIdx.x % G;
    const int gi = threadIdx.x / G;
    const int64_t j = (int64_t)blockIdx.x * GPB + gi;
    const bool valid = j < K;
    for (int e = gl; e < 22; e += G) {
        double v = 0.0;
        if (valid) v = e < 16 ? a[4 * j + e] : knots[j + 1 + (e - 16)];
        if (e < 16) sh_a[gi][e] = v;
        else sh_k[gi][e - 16] = v;
    }
    __syncthreads();
    double accP[IV_PAIRS * 10];
    double accR[16];
    double accC[IV_CAL];
#pragma unroll
    for (int e = 0; e < IV_PAIRS * 10; ++e) accP[e] = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) accR[e] = 0.0;
#pragma unroll
    for (int e = 0; e < IV_CAL; ++e) accC[e] = 0.0;
    const double lam2 = k.lam2;
    const int64_t l0 = valid ? iv_off[j] : 0, l1 = valid ? iv_off[j + 1] : 0;
    int64_t l = l0 + gl;
    double t_c = 0.0, e_c = 0.0;
    float s_c = 1.0f;
    int32_t cf_c = 0;
    SrcPrep sp_c = {};
    if (l < l1) {
        t_c = ot[l];
        e_c = oeta[l];
        s_c = osig[l];
        cf_c = ocellfov[l];
        sp_c = prep[osrc[l]];
    }
    for (; l < l1; l += G) {
        const int64_t ln = l + G;
        double t_n = 0.0, e_n = 0.0;
        float s_n = 1.0f;
        int32_t cf_n = 0, src_n = 0;
        if (ln < l1) {
            t_n = ot[ln];
            e_n = oeta[ln];
            s_n = osig[ln];
            cf_n = ocellfov[ln];
            src_n = osrc[ln];
        }
        ObsEval o;
        observe(k, t_c, e_c, c[cf_c >> 1], sp_c.r, sp_c.mu, sp_c.plx, sh_a[gi], sh_k[gi], o);
        SrcPrep sp_n = {};
        if (ln < l1) sp_n = prep[src_n];
        double g[4];
        attitude_partial(o, g);
        const double sg = (double)s_c;
        const double W = 1.0 / (sg * sg);
        double M[10], rv[4];
        int e = 0;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int cc = rr; cc < 4; ++cc)
                M[e++] = W * (g[rr] * g[cc] + 4.0 * lam2 * o.qraw[rr] * o.qraw[cc]);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) rv[rr] = -W * (g[rr] * o.R - 2.0 * lam2 * o.qraw[rr] * o.D);
        int pp = 0;
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int m = n; m < 4; ++m) {
                const double bb = o.B[n] * o.B[m];
#pragma unroll
                for (int ee = 0; ee < 10; ++ee) accP[pp * 10 + ee] += bb * M[ee];
                ++pp;
            }
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) accR[n * 4 + rr] += o.B[n] * rv[rr];
        const int f = cf_c & 1;
        accC[2 * f] += W;
        accC[2 * f + 1] += W * o.R;
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        cf_c = cf_n;
        sp_c = sp_n;
    }
    double* out = iv_sums + j * IV_SUMS;
#pragma unroll
    for (int e = 0; e < IV_PAIRS * 10; ++e) {
        const double v = group_sum<G>(accP[e]);
        if (valid && gl == (e % G)) out[e] = v;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double v = group_sum<G>(accR[e]);
        if (valid && gl == ((100 + e) % G)) out[100 + e] = v;
    }
#pragma unroll
    for (int e = 0; e < IV_CAL; ++e) {
        const double v = group_sum<G>(accC[e]);
        if (valid && gl == (e % G)) iv_cal[j * IV_CAL + e] = v;
    }
}

// ------------------------------------------------------------ band solve
constexpr int RING = 8;                 // intervals held in LDS
constexpr int RING_W = IV_SUMS;         // doubles per interval

// Entry (i, kk) (segment-relative scalar indices, i <= kk <= i + 15) of the
// segment's band matrix from the ring of per-interval sums.
__device__ __forceinline__ double ring_entry(const double (*ring)[RING_W], int64_t nb, int64_t i, int64_t kk) {
    const int64_t bi = i >> 2, bk = kk >> 2;
    const int r = (int)(i & 3), cc = (int)(kk & 3);
    const int e = r < cc ? tri4(r, cc) : tri4(cc, r);
    const int64_t jlo = bk - 3 > 0 ? bk - 3 : 0;
    const int64_t jhi = bi < nb - 4 ? bi : nb - 4;
    double s = 0.0;
    for (int64_t j = jlo; j <= jhi; ++j) s += ring[j & (RING - 1)][tri4((int)(bi - j), (int)(bk - j)) * 10 + e];
    return s;
}

__device__ __forceinline__ double ring_rhs(const double (*ring)[RING_W], int64_t nb, int64_t i) {
    const int64_t bi = i >> 2;
    const int r = (int)(i & 3);
    const int64_t jlo = bi - 3 > 0 ? bi - 3 : 0;
    const int64_t jhi = bi < nb - 4 ? bi : nb - 4;
    double s = 0.0;
    for (int64_t j = jlo; j <= jhi; ++j) s += ring[j & (RING - 1)][100 + (bi - j) * 4 + r];
    return s;
}

constexpr int PF = (RING_W + 63) / 64;  // doubles per lane to fetch one interval

__global__ __launch_bounds__(64) void k_band_solve(int64_t nseg, const SegDesc* __restrict__ segs,
                                                   const double* __restrict__ iv_sums, double* __restrict__ ufac,
                                                   double* __restrict__ yfac, double* __restrict__ da,
                                                   int32_t* __restrict__ seg_def) {
    __shared__ double ring[RING][RING_W];
    __shared__ double Wn[16][17];      // window: row slot i & 15, column slot kk & 15, column 16 = rhs
    __shared__ double Ur[17];
    __shared__ double X[16];
    __shared__ double Ub[2][16][17];   // back substitution: factor rows (+ y) of two 16-row chunks
    const int lane = threadIdx.x;
    const int64_t sgi = blockIdx.x;
    if (sgi >= nseg) return;
    const SegDesc d = segs[sgi];
    const int64_t nb = d.n_hi - d.n_lo + 1;
    const int64_t nu = 4 * nb;
    const int64_t n_iv = nb - 3;       // intervals of the segment
    const double* sums = iv_sums + d.n_lo * IV_SUMS;
    double* U = ufac + d.u_off * 16;
    double* Y = yfac + d.u_off;
    // intervals 0..4 into the ring
    for (int jj = 0; jj < 5 && jj < n_iv; ++jj)
        for (int e = lane; e < RING_W; e += 64) ring[jj][e] = sums[(int64_t)jj * IV_SUMS + e];
    __syncthreads();
    for (int idx = lane; idx < 16 * 17; idx += 64) {
        const int row = idx / 17, col = idx % 17;
        double v = 0.0;
        if (row < nu) {
            if (col == 16) v = ring_rhs(ring, nb, row);
            else if (col >= row && col < nu) v = ring_entry(ring, nb, row, col);
        }
        Wn[row][col] = v;
    }
    __syncthreads();
    int defect = 0;
    double pf[PF];
    for (int64_t i = 0; i < nu; ++i) {
        const int64_t b = i >> 2;
        const bool block_start = (i & 3) == 0;
        const int64_t jpf = b + 5;     // interval to prefetch during this block
        if (block_start && jpf < n_iv) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int e = lane + 64 * u;
                pf[u] = e < RING_W ? sums[jpf * IV_SUMS + e] : 0.0;
            }
        }
        const int si = (int)(i & 15);
        const double piv = Wn[si][si];
        const bool ok = piv > 0.0;
        const double uu = ok ? sqrt(piv) : 0.0;
        const double inv = ok ? 1.0 / uu : 0.0;
        if (!ok) ++defect;
        if (lane < 16) {
            const int64_t kk = i + lane;
            double v = 0.0;
            if (kk < nu) v = lane == 0 ? uu : Wn[si][kk & 15] * inv;
            U[i * 16 + lane] = v;
            Ur[lane] = v;
        } else if (lane == 16) {
            const double y = Wn[si][16] * inv;
            Y[i] = y;
            Ur[16] = y;
        }
        __syncthreads();
        // trailing update: 120 pairs (dj, dk), 1 <= dj <= dk <= 15, then 15
        // right-hand-side items
        for (int w = lane; w < 135; w += 64) {
            if (w < 120) {
                int dj = 1, rem = w;
                while (rem >= 16 - dj) {
                    rem -= 16 - dj;
                    ++dj;
                }
                const int dk = dj + rem;
                const int64_t jj = i + dj, kk = i + dk;
                if (kk < nu) Wn[jj & 15][kk & 15] -= Ur[dj] * Ur[dk];
            } else {
                const int dj = w - 119;
                const int64_t jj = i + dj;
                if (jj < nu) Wn[jj & 15][16] -= Ur[dj] * Ur[16];
            }
        }
        __syncthreads();
        const int64_t kn = i + 16;     // column entering the window
        if (kn < nu) {
            if (lane < 16) {
                const int64_t jj = kn - 15 + lane;
                Wn[jj & 15][kn & 15] = ring_entry(ring, nb, jj, kn);
            } else if (lane == 16) {
                Wn[kn & 15][16] = ring_rhs(ring, nb, kn);
            }
        }
        if ((i & 3) == 3 && jpf < n_iv) {
            // end of block b: the prefetched interval b + 5 enters the ring
            // (its slot held interval b - 3, no longer referenced)
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int e = lane + 64 * u;
                if (e < RING_W) ring[jpf & (RING - 1)][e] = pf[u];
            }
        }
        __syncthreads();
    }
    // back substitution (Algorithm C3), factor rows fetched a chunk ahead
    if (lane < 16) X[lane] = 0.0;
    const int64_t nchunk = (nu + 15) / 16;
    auto load_chunk = [&](int64_t ch, double* regs) {
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int idx = lane + 64 * u;          // 0 .. 16*17-1 used
            double v = 0.0;
            if (idx < 16 * 17) {
                const int row = idx / 17, col = idx % 17;
                const int64_t i = ch * 16 + row;
                if (i < nu) v = col < 16 ? U[i * 16 + col] : Y[i];
            }
            regs[u] = v;
        }
    };
    auto store_chunk = [&](int buf, const double* regs) {
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int idx = lane + 64 * u;
            if (idx < 16 * 17) Ub[buf][idx / 17][idx % 17] = regs[u];
        }
    };
    double cur[5], nxt[5];
    load_chunk(nchunk - 1, cur);
    store_chunk((nchunk - 1) & 1, cur);
    __syncthreads();
    for (int64_t ch = nchunk - 1; ch >= 0; --ch) {
        if (ch > 0) load_chunk(ch - 1, nxt);
        const int buf = (int)(ch & 1);
        const int64_t i_hi = (ch * 16 + 15 < nu - 1) ? ch * 16 + 15 : nu - 1;
        for (int64_t i = i_hi; i >= ch * 16; --i) {
            const int row = (int)(i - ch * 16);
            double v = 0.0;
            if (lane >= 1 && lane < 16) {
                const int64_t kk = i + lane;
                if (kk < nu) v = Ub[buf][row][lane] * X[kk & 15];
            }
            v = group_sum<16>(v);
            if (lane == 0) {
                const double uii = Ub[buf][row][0];
                const double xi = uii > 0.0 ? (Ub[buf][row][16] - v) / uii : 0.0;
                X[i & 15] = xi;
                const int64_t n = d.n_lo + (i >> 2);
                if (n >= d.keep_lo && n <= d.keep_hi) da[4 * n + (i & 3)] = xi;
            }
            __syncthreads();
        }
        if (ch > 0) store_chunk((ch - 1) & 1, nxt);
        __syncthreads();
    }
    if (lane == 0) seg_def[sgi] = defect;
}

inline int groups_grid(int64_t n_items, int items_per_block) {
    return (int)((n_items + items_per_block - 1) / items_per_block);
}

}  // namespace

#define AGIS_S_LAUNCH(G)                                                                                       \
    k_source_update<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                             \
        ctx->k, ctx->n_src, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots, \
        ctx->a, ctx->c, ctx->s, ctx->prep, ctx->ds, ctx->qsrc, ctx->sdef, ctx->svar)

void launch_source_update(agis_ctx* ctx) {
    if (ctx->n_src == 0) return;
    switch (ctx->s_group) {
        case 8: AGIS_S_LAUNCH(8); break;
        case 16: AGIS_S_LAUNCH(16); break;
        case 32: AGIS_S_LAUNCH(32); break;
        default: AGIS_S_LAUNCH(64); break;
    }
}

#define AGIS_AC_LAUNCH(G)                                                                                     \
    k_ac_pass<G><<<groups_grid(ctx->K, 256 / G), 256, 0, ctx->stream>>>(                                       \
        ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig, ctx->t_cellfov, ctx->t_src, ctx->prep, \
        ctx->knots, ctx->a, ctx->c, ctx->iv_sums, ctx->iv_cal)

void launch_ac_pass(agis_ctx* ctx) {
    if (ctx->K == 0) return;
    switch (ctx->ac_group) {
        case 4: AGIS_AC_LAUNCH(4); break;
        case 8: AGIS_AC_LAUNCH(8); break;
        case 16: AGIS_AC_LAUNCH(16); break;
        case 32: AGIS_AC_LAUNCH(32); break;
        default: AGIS_AC_LAUNCH(64); break;
    }
}

void launch_band_solve(agis_ctx* ctx) {
    const int64_t nseg = (int64_t)ctx->h_segs.size();
    if (nseg == 0) return;
    k_band_solve<<<(unsigned)nseg, 64, 0, ctx->stream>>>(nseg, ctx->segs, ctx->iv_sums, ctx->ufac, ctx->yfac, ctx->da,
                                                        ctx->seg_def);
}

}  // namespace agis
