// Shared by the plain and the robust source updates and the A/C pass: the
// downweighting function, a group reduction, and the per-source tail of the
// S block (Sect. 5.1): Algorithms C1-C3 on the 5x5 normal equations, the
// diagonal of the inverse (first-order variances, Sect. 5.1.1), Q_i of
// eq:Qi, the update (alpha through d_1 / cos delta) and the per-source record
// the time-ordered pass gathers.
#pragma once

#include "model.h"

namespace agis {

// acc: the 15 upper-triangle entries of N (row-major), the 5 of b and h'Wh.
// rhs (optional, [n_src][5]) receives b; eps_i2 goes into the record.
__device__ __forceinline__ void source_finish(const double acc[21], int64_t i, double alpha, double delta,
                                              double plx, double pma, double pmd, double cd, double* __restrict__ s,
                                              SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                              double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                              double* __restrict__ svar, double* __restrict__ rhs = nullptr,
                                              double eps_i2 = 0.0) {
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
    if (rhs)
        for (int rr = 0; rr < 5; ++rr) rhs[5 * i + rr] = acc[15 + rr];
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
    pr.pad = eps_i2;                      // the source's excess noise eps_i^2 (robust mode 2)
    prep[i] = pr;
}

// Downweighting function w(z) of eq:dw.
__device__ __forceinline__ double down_weight(double z) {
    const double a = fabs(z);
    if (a <= 2.0) return 1.0;
    if (a < 3.0) {
        const double t = a - 2.0;
        return 1.0 - 1.773735 * t * t + 1.141615 * t * t * t;
    }
    return exp(-a / 3.0);
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace agis
