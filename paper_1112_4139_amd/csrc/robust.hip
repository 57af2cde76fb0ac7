// Robust weighting (Sect. 5.1.2 and 5.2.5).
//
//   k_s_rows<G>     S block, pass 0: G lanes per source evaluate the model at
//                   the current parameters and store, per observation (by-source
//                   order), the design row -dR/ds (its alpha*, delta and
//                   parallax entries, and tau, the proper-motion entries
//                   being the first two times tau), h = R and
//                   sigma~^2 = sigma^2 + eps_a^2(t) as six columns in HBM.
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
// the lower one is found by eight 8-bit radix-selection passes over an
// order-preserving integer image of the doubles (held in registers, up to
// 2,048 per block), with the digit histogram in LDS (integer counts: the
// result does not depend on the order of the adds); the upper one by a count
// and a minimum over the same keys.
#include <algorithm>
#include <cfloat>

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

// One radix step of the selection of the k-th smallest key: from the
// 256-bin histogram of the current digit, the digit holding rank k and the
// number of keys in the lower digits (every lane receives both).
__device__ __forceinline__ void radix_digit(const uint32_t* hist, int64_t k, int& digit_out, uint32_t& below_out) {
    const int lane = threadIdx.x;
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
    digit_out = __shfl(digit, src, 64);
    below_out = __shfl(below, src, 64);
}

// k-th smallest (0-based, k < n) of v[0..n) by the whole 64-thread block,
// reading v on every pass (any n).
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
        int digit;
        uint32_t below;
        radix_digit(hist, k, digit, below);
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

// Keys held in registers: key r of lane l is element l + 64 r (n <= 64 KR).
constexpr int KR = 32;

__device__ __forceinline__ void load_keys(const double* __restrict__ v, int64_t n, uint64_t (&kr)[KR]) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < KR; ++r) kr[r] = lane + 64 * r < n ? order_key(v[lane + 64 * r]) : ~0ull;
}

// k-th smallest key of the n register-held keys.  Where every active lane
// of a slot has the same digit (the leading digits of values of one sign
// and magnitude), one lane adds their count: LDS atomics to one address
// from all lanes would serialise.
__device__ uint64_t reg_select(const uint64_t (&kr)[KR], int64_t n, int64_t k, uint32_t* hist) {
    const int lane = threadIdx.x;
    const int nr = (int)((n + 63) / 64);
    uint64_t prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = lane; b < 256; b += 64) hist[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            if (r < nr && lane + 64 * r < n && (kr[r] & mask) == prefix) {
                // the active lanes only: the first one's digit, and who shares it
                const uint32_t dg = (uint32_t)(kr[r] >> shift) & 255u;
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                const uint64_t am = __ballot(true);
                const uint64_t same = __ballot(dg == d0);
                if (same == am) {
                    if (lane == __ffsll((unsigned long long)am) - 1) atomicAdd(&hist[d0], (uint32_t)__popcll(am));
                } else {
                    atomicAdd(&hist[dg], 1u);
                }
            }
        }
        __syncthreads();
        int digit;
        uint32_t below;
        radix_digit(hist, k, digit, below);
        prefix |= (uint64_t)digit << shift;
        mask |= 0xFFull << shift;
        k -= (int64_t)below;
        __syncthreads();
    }
    return prefix;
}

// Type-7 p-quantile of the n register-held keys: the order statistic j by
// selection, j + 1 as the same key if more than j + 1 keys are <= it, else
// as the smallest key above it.
__device__ double reg_quantile7(const uint64_t (&kr)[KR], int64_t n, double p, uint32_t* hist) {
    if (n <= 0) return 0.0;
    const int lane = threadIdx.x;
    const double h = (double)(n - 1) * p;
    const int64_t j = (int64_t)floor(h);
    const uint64_t kj = reg_select(kr, n, j, hist);
    const double xj = key_value(kj);
    if (j + 1 >= n) return xj;
    uint32_t cle = 0;
    uint64_t mn = ~0ull;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        if (lane + 64 * r < n) {
            cle += kr[r] <= kj ? 1u : 0u;
            if (kr[r] > kj && kr[r] < mn) mn = kr[r];
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cle += __shfl_xor(cle, o, 64);
        const uint32_t lo = __shfl_xor((uint32_t)mn, o, 64), hi = __shfl_xor((uint32_t)(mn >> 32), o, 64);
        const uint64_t other = ((uint64_t)hi << 32) | lo;
        mn = other < mn ? other : mn;
    }
    const uint64_t kj1 = (int64_t)cle >= j + 2 ? kj : mn;
    return xj + (h - (double)j) * (key_value(kj1) - xj);
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
                                                   double* __restrict__ col, int64_t n_obs,
                                                   const int32_t* __restrict__ order) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    if (kg >= n_src) return;
    const int64_t i = order[kg];
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
        for (int e = 0; e < 3; ++e) col[e * n_obs + l] = A[e];
        col[3 * n_obs + l] = o.tau;              // A[3] = A[0] tau, A[4] = A[1] tau
        col[4 * n_obs + l] = o.R;
        col[5 * n_obs + l] = sg * sg + eps_a2[(ell - 3) / eps_bucket];
    }
}

// ------------------------------------------------ S, initial downweights
// REG: keys of sets up to reg_limit in registers (fewer wavefronts per SIMD,
// pays for large sets); otherwise re-read on every pass (small sets).
template <bool REG>
__global__ __launch_bounds__(64) void k_s_sigma(int64_t n_src, const int64_t* __restrict__ off,
                                                const double* __restrict__ h, double* __restrict__ vs,
                                                int64_t reg_limit, const int32_t* __restrict__ order) {
    __shared__ uint32_t hist[256];
    if ((int64_t)blockIdx.x >= n_src) return;
    const int64_t i = order[blockIdx.x];         // the largest sets first
    const int64_t l0 = off[i], n = off[i + 1] - l0;
    double q5, q1;
    if (REG && n <= reg_limit) {
        uint64_t kr[KR];
        load_keys(h + l0, n, kr);
        q5 = reg_quantile7(kr, n, 5.0 / 6.0, hist);
        q1 = reg_quantile7(kr, n, 1.0 / 6.0, hist);
    } else {
        q5 = block_quantile7(h + l0, n, 5.0 / 6.0, hist);
        q1 = block_quantile7(h + l0, n, 1.0 / 6.0, hist);
    }
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
                                                double* __restrict__ svar, const int32_t* __restrict__ order) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int leader = (threadIdx.x & 63) & ~(G - 1);
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = kg < n_src;
    const int64_t i = valid ? order[kg] : 0;
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
            for (int e = 0; e < 3; ++e) A[e] = col[e * n_obs + l];
            const double tau = col[3 * n_obs + l];
            A[3] = A[0] * tau;                   // as the design row forms them
            A[4] = A[1] * tau;
            const double h = col[4 * n_obs + l], s2 = col[5 * n_obs + l];
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

// The inner iteration with the excess source noise (robust mode 2,
// Sect. 5.1.2): four rounds as in k_s_irls, the weights of a round after the
// first w(R_l / (sigma~_l^2 + eps_i^2)^1/2) from the previous round's
// solution and eps_i (eq:wl); within a round, for those w_l, eps_i^2 = y
// solves Q(y) = nu (eq:epsi) by up to EPS_STEPS rational steps
// dy = (1 - Q/nu) Q / Q' from y = 0, Q'(y) = -sum w_l R_l^2 / (sigma~_l^2 +
// y)^2, nu = n_i - n_out - 5 with n_out the observations with w_l < 0.2;
// each y costs one accumulation and one residual pass.  D of eq:D (from
// the last round's Q(0)) and eps_i^2 are stored per source.
constexpr int EPS_STEPS = 3;

template <int G>
__global__ __launch_bounds__(256) void k_s_irls_eps(int64_t n_src, const int64_t* __restrict__ off,
                                                    const double* __restrict__ col, int64_t n_obs,
                                                    const double* __restrict__ vs, double* __restrict__ s,
                                                    SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                    double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                    double* __restrict__ svar, const int32_t* __restrict__ order,
                                                    double* __restrict__ eps2_out, double* __restrict__ D_out) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int leader = (threadIdx.x & 63) & ~(G - 1);
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = kg < n_src;
    const int64_t i = valid ? order[kg] : 0;
    const int64_t l0 = valid ? off[i] : 0, l1 = valid ? off[i + 1] : 0;
    const double vsi = valid ? vs[i] : 0.0;
    double dw[5] = {0.0, 0.0, 0.0, 0.0, 0.0};      // solution the round's weights come from
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};       // current solution
    double y = 0.0, D = 0.0;
    double acc[21];
    // w_l of the round (it) from dw and the previous round's eps_i^2 (yw)
    auto weight_of = [&](int it, const double* A, double h, double s2, double yw) {
        if (it == 0) return vsi > 0.0 ? down_weight(h / vsi) : 1.0;
        double R = h;
#pragma unroll
        for (int e = 0; e < 5; ++e) R -= A[e] * dw[e];
        return down_weight(R / sqrt(s2 + yw));
    };
    auto load = [&](int64_t l, double* A, double& h, double& s2) {
#pragma unroll
        for (int e = 0; e < 3; ++e) A[e] = col[e * n_obs + l];
        const double tau = col[3 * n_obs + l];
        A[3] = A[0] * tau;
        A[4] = A[1] * tau;
        h = col[4 * n_obs + l];
        s2 = col[5 * n_obs + l];
    };
    for (int it = 0; it < INNER_SOLVES; ++it) {
        const double yw = y;
        // accumulation at y; the first one also counts the outliers
        auto accumulate = [&](double yacc, double* nout) {
#pragma unroll
            for (int e = 0; e < 21; ++e) acc[e] = 0.0;
            double no = 0.0;
            for (int64_t l = l0 + gl; l < l1; l += G) {
                double A[5], h, s2;
                load(l, A, h, s2);
                const double wl = weight_of(it, A, h, s2, yw);
                no += wl < 0.2 ? 1.0 : 0.0;
                const double W = wl / (s2 + yacc);
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
            if (nout) *nout = group_sum<G>(no);
        };
        auto solve = [&]() {
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
        };
        // Q(y) and Q'(y) at the current solution
        auto chi2 = [&](double yq, double& Q, double& Qp) {
            double q = 0.0, qp = 0.0;
            for (int64_t l = l0 + gl; l < l1; l += G) {
                double A[5], h, s2;
                load(l, A, h, s2);
                const double wl = weight_of(it, A, h, s2, yw);
                double R = h;
#pragma unroll
                for (int e = 0; e < 5; ++e) R -= A[e] * d[e];
                const double v = s2 + yq;
                q += wl / v * R * R;
                qp -= wl * R * R / (v * v);
            }
            Q = group_sum<G>(q);
            Qp = group_sum<G>(qp);
        };
        double nout = 0.0;
        y = 0.0;
        accumulate(y, &nout);
        const double nu = (double)(l1 - l0) - nout - 5.0;
        solve();
        double Q, Qp;
        chi2(y, Q, Qp);
        D = nu > 0.0 ? (Q - nu) / sqrt(2.0 * nu) : 0.0;
        for (int step = 0; step < EPS_STEPS; ++step) {
            if (!(nu > 0.0 && Q > nu && Qp < 0.0)) break;
            y += (1.0 - Q / nu) * Q / Qp;
            if (y < 0.0) y = 0.0;
            accumulate(y, nullptr);
            solve();
            chi2(y, Q, Qp);
        }
#pragma unroll
        for (int e = 0; e < 5; ++e) dw[e] = d[e];
    }
    if (!valid || gl != 0) return;
    eps2_out[i] = y;
    D_out[i] = D;
    const double* si = s + 5 * i;
    const double alpha = si[0], delta = si[1], plx = si[2], pma = si[3], pmd = si[4];
    source_finish(acc, i, alpha, delta, plx, pma, pmd, cos(delta), s, prep, ds, qsrc, sdef, svar, nullptr, y);
}

// ------------------------------------------------ excess attitude noise
__global__ __launch_bounds__(64) void k_ac_resid(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                 const double* __restrict__ ot, const double* __restrict__ oeta,
                                                 const float* __restrict__ osig,
                                                 const int32_t* __restrict__ ocellfov,
                                                 const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                                 const double* __restrict__ knots,
                                                 const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                 const double* __restrict__ c, int robust, double* __restrict__ v) {
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
        v[l] = o.R * o.R - sg * sg - (robust == 2 ? sp.pad : 0.0);       // e09 with eps_i^2 (mode 2)
    }
}

// Frozen weights: the robust weight of the A/C pass, W = w(R / sigma~) /
// sigma~^2 with sigma~^2 = sigma^2 + eps_a^2 of the interval's bucket
// (eq:dw, eq:W), at the current parameters, stored as sigma_eff = 1 / sqrt(W)
// in FP32 (W = 0: the largest finite float).
__global__ __launch_bounds__(64) void k_freeze_sigma(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                     const double* __restrict__ ot, const double* __restrict__ oeta,
                                                     const float* __restrict__ osig,
                                                     const int32_t* __restrict__ ocellfov,
                                                     const int32_t* __restrict__ osrc,
                                                     const SrcPrep* __restrict__ prep,
                                                     const double* __restrict__ knots,
                                                     const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ eps_a2, int eps_bucket, int robust,
                                                     float* __restrict__ sig_eff) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    if (j >= K) return;
    double a4[16], kn[6];
    for (int e = 0; e < 16; ++e) a4[e] = a[4 * j + e];
    for (int e = 0; e < 6; ++e) kn[e] = knots[j + 1 + e];
    const KnotTab kt = ktab[j];
    const double eps2 = eps_a2[j / eps_bucket];
    for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
        const SrcPrep sp = prep[osrc[l]];
        ObsEval o;
        observe(k, ot[l], oeta[l], c[ocellfov[l] >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o);
        const double sg = (double)osig[l];
        const double s2 = sg * sg + eps2 + (robust == 2 ? sp.pad : 0.0);
        const double W = down_weight(o.R / sqrt(s2)) / s2;
        float se = W > 0.0 ? (float)(1.0 / sqrt(W)) : FLT_MAX;
        if (!(se <= FLT_MAX)) se = FLT_MAX;
        sig_eff[l] = se;
    }
}

__global__ void k_gather_f32(int64_t n, const int32_t* __restrict__ from, const float* __restrict__ src,
                             float* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[from[i]];
}

template <bool REG>
__global__ __launch_bounds__(64) void k_bucket_eps(int64_t n_buckets, int64_t K, int eps_bucket,
                                                   const int64_t* __restrict__ iv_off, const double* __restrict__ v,
                                                   double* __restrict__ eps_a2, int64_t reg_limit) {
    __shared__ uint32_t hist[256];
    const int64_t b = blockIdx.x;
    if (b >= n_buckets) return;
    const int64_t j0 = b * eps_bucket;
    const int64_t j1 = j0 + eps_bucket < K ? j0 + eps_bucket : K;
    const int64_t l0 = iv_off[j0], n = iv_off[j1] - l0;
    double q;
    if (REG && n <= reg_limit) {
        uint64_t kr[KR];
        load_keys(v + l0, n, kr);
        q = reg_quantile7(kr, n, 0.68, hist);
    } else {
        q = block_quantile7(v + l0, n, 0.68, hist);
    }
    if (threadIdx.x == 0) eps_a2[b] = q > 0.0 ? q : 0.0;
}

// Largest set whose keys go to registers; larger sets (or all, with the
// context's limit at 0) are read from memory on every radix pass.
inline int64_t select_reg_limit(const agis_ctx* ctx) {
    return ctx->select_reg_limit < 64 * KR ? ctx->select_reg_limit : 64 * KR;
}

// The register kernel pays for mean set sizes from ~256 up to about three
// quarters of its capacity (measured: sets of ~160 run faster in the lean
// kernel, ~800 and ~1,200 in the register one; at ~2,400 most sets exceed the
// capacity and re-read their values with fewer wavefronts per SIMD).
inline bool select_in_registers(const agis_ctx* ctx, int64_t n_values, int64_t n_sets) {
    const int64_t lim = select_reg_limit(ctx);
    return lim > 0 && n_sets > 0 && n_values >= ctx->select_reg_min_mean * n_sets &&
           (ctx->select_reg_min_mean == 0 || 4 * n_values <= 3 * lim * n_sets);
}

inline unsigned groups_grid(int64_t n_items, int items_per_block) {
    return (unsigned)((n_items + items_per_block - 1) / items_per_block);
}

}  // namespace

#define AGIS_ROWS_LAUNCH(G)                                                                                      \
    k_s_rows<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                                      \
        ctx->k, ctx->n_src, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots,   \
        ctx->ktab, ctx->a, ctx->c, ctx->s, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->rcol, ctx->n_obs, ctx->src_order)
#define AGIS_IRLS_LAUNCH(G)                                                                                      \
    if (ctx->cfg.robust == 2)                                                                                    \
        k_s_irls_eps<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                              \
            ctx->n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc,      \
            ctx->sdef, ctx->svar, ctx->src_order, ctx->src_eps2, ctx->src_D);                                    \
    else                                                                                                         \
        k_s_irls<G><<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                                  \
            ctx->n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc,      \
            ctx->sdef, ctx->svar, ctx->src_order)

void launch_source_update_robust(agis_ctx* ctx) {
    if (ctx->n_src == 0) return;
    switch (ctx->s_group) {
        case 8: AGIS_ROWS_LAUNCH(8); break;
        case 16: AGIS_ROWS_LAUNCH(16); break;
        case 32: AGIS_ROWS_LAUNCH(32); break;
        default: AGIS_ROWS_LAUNCH(64); break;
    }
    (select_in_registers(ctx, ctx->n_obs, ctx->n_src) ? k_s_sigma<true> : k_s_sigma<false>)
        <<<(unsigned)ctx->n_src, 64, 0, ctx->stream>>>(ctx->n_src, ctx->src_off, ctx->rcol + 4 * ctx->n_obs, ctx->vs,
                                                       select_reg_limit(ctx), ctx->src_order);
    switch (ctx->s_group) {
        case 8: AGIS_IRLS_LAUNCH(8); break;
        case 16: AGIS_IRLS_LAUNCH(16); break;
        case 32: AGIS_IRLS_LAUNCH(32); break;
        default: AGIS_IRLS_LAUNCH(64); break;
    }
}

void launch_freeze_sigma(agis_ctx* ctx) {
    if (ctx->K > 0)
        k_freeze_sigma<<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(
            ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig, ctx->t_cellfov, ctx->t_src, ctx->prep,
            ctx->knots, ctx->ktab, ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->cfg.robust, ctx->t_sig_eff);
    if (ctx->n_obs > 0) {
        const int64_t b = std::min<int64_t>((ctx->n_obs + 255) / 256, 65536);
        k_gather_f32<<<(unsigned)b, 256, 0, ctx->stream>>>(ctx->n_obs, ctx->s_from_t, ctx->t_sig_eff,
                                                           ctx->s_sig_eff);
    }
}

void launch_excess_noise(agis_ctx* ctx) {
    if (ctx->K == 0 || ctx->n_buckets == 0) return;
    k_ac_resid<<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig,
                                                         ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots, ctx->ktab,
                                                         ctx->a, ctx->c, ctx->cfg.robust, ctx->rcol);
    (select_in_registers(ctx, ctx->n_obs, ctx->n_buckets) ? k_bucket_eps<true> : k_bucket_eps<false>)
        <<<(unsigned)ctx->n_buckets, 64, 0, ctx->stream>>>(ctx->n_buckets, ctx->K, ctx->cfg.eps_bucket, ctx->iv_off,
                                                           ctx->rcol, ctx->eps_a2, select_reg_limit(ctx));
}

}  // namespace agis
