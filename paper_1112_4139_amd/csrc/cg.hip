// Kernels of the conjugate-gradient scheme (Sect. 4.7).  The vectors span
// all unknowns: sources [n_src][5] (d alpha*, d delta, d parallax,
// d mu_alpha*, d mu_delta), attitude coefficients [N][4], calibration
// [n_cells].  r is the right-hand side b - N x of the three normal-equation
// blocks, z = K^-1 r the three block updates at the same point, p the
// search direction; k_cg_quad forms p'N p from the observations.
// Reductions use a fixed grid and a fixed summation order, so every result
// is reproducible bit for bit.
#include "agis_internal.h"
#include "model.h"

namespace agis {

constexpr int CG_BLOCKS = 1024;
constexpr int CG_THREADS = 256;

int64_t cg_size(const agis_ctx* ctx) { return 5 * ctx->n_src + 4 * ctx->N + ctx->n_cells; }

// Block sums of two values, one result pair per block.
__device__ __forceinline__ void block_sum2(double a, double b, double* __restrict__ part) {
    __shared__ double red[2][CG_THREADS / 64];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m, 64);
        b += __shfl_xor(b, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < CG_THREADS / 64; ++w) {
            sa += red[0][w];
            sb += red[1][w];
        }
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}

// out[0..1] = sums of the CG_BLOCKS partial pairs (one block)
__global__ __launch_bounds__(CG_THREADS) void k_cg_finish(const double* __restrict__ part, double* __restrict__ out) {
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < CG_BLOCKS; q += CG_THREADS) {
        a += part[2 * q];
        b += part[2 * q + 1];
    }
    __shared__ double red[2][CG_THREADS];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = CG_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

// r and z at the evaluated point from what the blocks left behind: the
// source right-hand sides are already in r (written by the S pass) and the
// calibration ones too (written by the C solve); the attitude right-hand
// side of coefficient n sums the entries of the (up to) four knot
// intervals n-3..n that it spans; z copies the three block updates.
__global__ __launch_bounds__(CG_THREADS) void k_cg_gather(int64_t n_src, int64_t N, int64_t K, int64_t n_cells,
                                                       const double* __restrict__ iv_sums,
                                                       const double* __restrict__ ds, const double* __restrict__ da,
                                                       const double* __restrict__ dc, double* __restrict__ r,
                                                       double* __restrict__ z) {
    const int64_t off_a = 5 * n_src, off_c = off_a + 4 * N, n = off_c + n_cells;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < off_a) {
            z[e] = ds[e];
        } else if (e < off_c) {
            const int64_t u = e - off_a, nc = u >> 2;
            const int q = (int)(u & 3);
            double s = 0.0;
            for (int k = 3; k >= 0; --k) {
                const int64_t j = nc - k;
                if (j >= 0 && j < K) s += iv_sums[j * IV_SUMS + 100 + 4 * k + q];
            }
            r[e] = s;
            z[e] = da[u];
        } else {
            z[e] = dc[e - off_c];
        }
    }
}

// state <- state + f v: alpha by f v_alpha* / cos delta (delta before the
// step), every other unknown additively
__global__ __launch_bounds__(CG_THREADS) void k_cg_step_state(int64_t n_src, int64_t N, int64_t n_cells,
                                                           const double* __restrict__ v, double f,
                                                           double* __restrict__ s, double* __restrict__ a,
                                                           double* __restrict__ c) {
    const int64_t na = 4 * N, items = n_src + na + n_cells;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < items;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < n_src) {
            double* x = s + 5 * e;
            const double* u = v + 5 * e;
            const double cd = cos(x[1]);
            x[0] += f * u[0] / cd;
#pragma unroll
            for (int k = 1; k < 5; ++k) x[k] += f * u[k];
        } else if (e < n_src + na) {
            const int64_t u = e - n_src;
            a[u] += f * v[5 * n_src + u];
        } else {
            const int64_t u = e - n_src - na;
            c[u] += f * v[5 * n_src + na + u];
        }
    }
}

// out[0] = sum a (b - c) (c optional), out[1] = sum a b
__global__ __launch_bounds__(CG_THREADS) void k_cg_dot(int64_t n, const double* __restrict__ a,
                                                    const double* __restrict__ b, const double* __restrict__ c,
                                                    double* __restrict__ part) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double ab = a[e] * b[e];
        s0 += c ? a[e] * (b[e] - c[e]) : ab;
        s1 += ab;
    }
    block_sum2(s0, s1, part);
}

// out[0] = a'b1, out[1] = a'b2
__global__ __launch_bounds__(CG_THREADS) void k_cg_dot2(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b1, const double* __restrict__ b2,
                                                     double* __restrict__ part) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        s0 += a[e] * b1[e];
        s1 += a[e] * b2[e];
    }
    block_sum2(s0, s1, part);
}

// p'N p at the current state, over the observations of knot intervals
// [b * 64, (b + 1) * 64) (block b): per observation W (J_R p)^2 + lambda^2 W (J_D p)^2
// with J_R p = -A . p_src + sum_n B_n dR/dq . p_att(n) + p_cal (A the design
// row -dR/ds of Sect. 5.1.3, dR/dq of eq:dfadq) and J_D p = sum_n -2 q~ B_n
// . p_att(n) (eq:dDldan); the source's triad comes from its direction r.
template <typename SigT>
__global__ __launch_bounds__(64) void k_cg_quad(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                const double* __restrict__ ot, const double* __restrict__ oeta,
                                                const SigT* __restrict__ osig, const int32_t* __restrict__ ocellfov,
                                                const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                                const double* __restrict__ knots, const KnotTab* __restrict__ ktab,
                                                const double* __restrict__ a, const double* __restrict__ c,
                                                const double* __restrict__ p, int64_t n_src, int64_t N,
                                                double* __restrict__ part) {
    const int lane = threadIdx.x;
    const double* pa = p + 5 * n_src;
    const double* pc = pa + 4 * N;
    double acc = 0.0;
    const int64_t j0 = (int64_t)blockIdx.x * 64, j1 = j0 + 64 < K ? j0 + 64 : K;
    for (int64_t j = j0; j < j1; ++j) {
        // the interval's table entry and coefficients are the same for all
        // lanes (a flat loop over the block's observations with a per-lane
        // interval lookup measured slower: 4.3 instead of 3.5 ms at 1.6e8
        // observations)
        const KnotTab kt = ktab[j];
        for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
            const int32_t i = osrc[l];
            const SrcPrep sp = prep[i];
            const int32_t cf = ocellfov[l], cell = cf >> 1;
            // across scan: pseudo-cell n_cells, no calibration unknown
            const bool ac = cf >= k.ac_cf0;
            ObsEval o;
            observe(k, ot[l], oeta[l], c[cell], sp.r, sp.mu, sp.plx, a + 4 * j, knots + (j + 1), kt, o, ac);
            const double cd = sqrt(sp.r[0] * sp.r[0] + sp.r[1] * sp.r[1]);
            const double icd = 1.0 / cd;
            const double pv[3] = {-sp.r[1] * icd, sp.r[0] * icd, 0.0};
            const double qv[3] = {-sp.r[2] * sp.r[0] * icd, -sp.r[2] * sp.r[1] * icd, cd};
            double A[5], g[4];
            source_partials(o, pv, qv, sp.r, A, ac);
            attitude_partial(o, g, ac);
            const double* ps = p + 5 * (int64_t)i;
            double jr = 0.0, jd = 0.0;
            if (!ac) jr = pc[cell];
#pragma unroll
            for (int e = 0; e < 5; ++e) jr -= A[e] * ps[e];
#pragma unroll
            for (int kn = 0; kn < 4; ++kn) {
                const double* pn = pa + 4 * (j + kn);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    jr += o.B[kn] * g[q] * pn[q];
                    jd += -2.0 * o.qraw[q] * o.B[kn] * pn[q];
                }
            }
            const double sg = (double)osig[l];
            const double W = 1.0 / (sg * sg);
            acc += W * jr * jr + k.lam2 * W * jd * jd;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) part[blockIdx.x] = acc;
}

// out[0] = sum of the n partials (one block of CG_THREADS, fixed order)
__global__ __launch_bounds__(CG_THREADS) void k_cg_quad_sum(int64_t n, const double* __restrict__ part,
                                                         double* __restrict__ out) {
    __shared__ double red[CG_THREADS];
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += CG_THREADS) acc += part[q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = CG_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// p <- z + beta p
__global__ __launch_bounds__(CG_THREADS) void k_cg_direction(int64_t n, double beta, const double* __restrict__ z,
                                                          double* __restrict__ p) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = z[e] + beta * p[e];
}

static unsigned cg_grid(int64_t n) {
    const int64_t b = (n + CG_THREADS - 1) / CG_THREADS;
    return (unsigned)(b < 1 ? 1 : (b > CG_BLOCKS ? CG_BLOCKS : b));
}

void launch_cg_gather(agis_ctx* ctx, double* r, double* z) {
    const int64_t n = cg_size(ctx);
    if (n == 0) return;
    k_cg_gather<<<cg_grid(n), CG_THREADS, 0, ctx->stream>>>(ctx->n_src, ctx->N, ctx->K, ctx->n_cells, ctx->iv_sums,
                                                            ctx->ds, ctx->da, ctx->dc, r, z);
}

void launch_cg_step_state(agis_ctx* ctx, const double* v, double f) {
    const int64_t items = ctx->n_src + 4 * ctx->N + ctx->n_cells;
    if (items == 0) return;
    k_cg_step_state<<<cg_grid(items), CG_THREADS, 0, ctx->stream>>>(ctx->n_src, ctx->N, ctx->n_cells, v, f, ctx->s,
                                                                    ctx->a, ctx->c);
}

// The reductions always run CG_BLOCKS blocks (idle ones add zeros), so the
// finishing kernel reads a fixed number of partials.
void launch_cg_dot(agis_ctx* ctx, const double* a, const double* b, const double* c, double* out) {
    k_cg_dot<<<CG_BLOCKS, CG_THREADS, 0, ctx->stream>>>(cg_size(ctx), a, b, c, ctx->cg_part);
    k_cg_finish<<<1, CG_THREADS, 0, ctx->stream>>>(ctx->cg_part, out);
}

void launch_cg_dot2(agis_ctx* ctx, const double* a, const double* b1, const double* b2, double* out) {
    k_cg_dot2<<<CG_BLOCKS, CG_THREADS, 0, ctx->stream>>>(cg_size(ctx), a, b1, b2, ctx->cg_part);
    k_cg_finish<<<1, CG_THREADS, 0, ctx->stream>>>(ctx->cg_part, out);
}

int64_t cg_quad_blocks(const agis_ctx* ctx) { return (ctx->K + 63) / 64; }

void launch_cg_quad(agis_ctx* ctx, const double* p, double* part, double* out) {
    const int64_t nb = cg_quad_blocks(ctx);
    if (nb == 0) {
        k_cg_quad_sum<<<1, CG_THREADS, 0, ctx->stream>>>(0, part, out);
        return;
    }
    if (ctx->frozen)
        k_cg_quad<double><<<(unsigned)nb, 64, 0, ctx->stream>>>(
            ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig_eff, ctx->t_cellfov, ctx->t_src, ctx->prep,
            ctx->knots, ctx->ktab, ctx->a, ctx->c, p, ctx->n_src, ctx->N, part);
    else
        k_cg_quad<float><<<(unsigned)nb, 64, 0, ctx->stream>>>(
            ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig, ctx->t_cellfov, ctx->t_src, ctx->prep,
            ctx->knots, ctx->ktab, ctx->a, ctx->c, p, ctx->n_src, ctx->N, part);
    k_cg_quad_sum<<<1, CG_THREADS, 0, ctx->stream>>>(nb, part, out);
}

void launch_cg_direction(agis_ctx* ctx, double beta) {
    const int64_t n = cg_size(ctx);
    if (n == 0) return;
    k_cg_direction<<<cg_grid(n), CG_THREADS, 0, ctx->stream>>>(n, beta, ctx->cg_z, ctx->cg_p);
}

}  // namespace agis
