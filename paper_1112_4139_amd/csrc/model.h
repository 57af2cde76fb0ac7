// Device-side observation model of the astrometric core solution for one
// along-scan or across-scan observation: proper direction (Sect. 3.2),
// attitude quaternion from the cubic B-spline (Sect. 3.3, Appendix B),
// instrument angles and field angles (eq:srsprop1, eq:srspropeta), residual
// (eq:resAL, eq:resAC), and the partial derivatives used by the S and A
// blocks (Sect. 5.1.3, 5.2.3-5.2.4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace agis {

// Per-run constants, passed by value to every kernel.
struct DevConsts {
    double gamma_half;   // Gamma_c / 2
    double t_ep;         // reference epoch [s]
    double inv_year;     // 1 / year [1/s]
    double au_c;         // light time for one astronomical unit [s]
    double lam2;         // lambda^2 of the attitude regularisation
    double eph_r, eph_L0, eph_Lrate, cos_obl, sin_obl;
    double t_fr;
    double year_s;
    double cos_half_gamma, sin_half_gamma;   // rounded cos, sin of Gamma_c / 2
    double half_gamma_err;                   // Gamma_c/2 - atan2(sin_half_gamma, cos_half_gamma)
    int32_t ac_cf0;                          // 2 n_cells: cell/fov codes from here on are across scan
    int64_t n_buckets;                       // excess-noise buckets per component (robust)
    double defl;                             // 0, or GM_sun / (c^2 AU) [rad AU]: the Sun's light deflection
    const double* gpar;                      // device [2]: g0 (gamma = 1 + g0), g1 (held at zero)
};

// Slot in the excess attitude noise array of a record with cell/fov code
// cf in knot interval j: the component (0 along scan, 1 across scan in the
// preceding, 2 in the following field of view) times the buckets per
// component, plus the interval's bucket.
__device__ __forceinline__ int64_t eps_slot(const DevConsts& k, int32_t cf, int64_t j, int eps_bucket) {
    const int64_t comp = cf >= k.ac_cf0 ? 1 + (cf & 1) : 0;
    return comp * k.n_buckets + j / eps_bucket;
}

// Source data gathered per observation by the time-ordered pass: barycentric
// direction r at t_ep, proper-motion vector p mu_a* + q mu_d, parallax.
struct SrcPrep {
    double r[3];
    double mu[3];
    double plx;
    double pad;
};

// Per knot interval [tau_l, tau_l+1): sine and cosine of the observer's
// orbital longitude at tau_l, 1 / (tau_l+1 - tau_l) when the six knots
// tau_l-2..tau_l+3 are equally spaced (0 otherwise), and tau_l.
struct KnotTab {
    double sL, cL;
    double inv_dt;
    double tau;
};

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// 1/sqrt(x) to ~1 ulp: hardware estimate and two Newton-Raphson steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

// 1/x to ~1 ulp: hardware estimate and two Newton-Raphson steps.
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    y = y * (2.0 - x * y);
    return y;
}

// The four non-zero cubic B-splines B_{l-3..l}(t) on an arbitrary knot
// sequence (Appendix B): the Cox-de Boor recursion in t, raised from order 1
// (the indicator of [tau_l, tau_l+1)) to order 4, each order-k function the
// sum of its two order-(k-1) neighbours weighted by (t - tau_i) /
// (tau_{i+k-1} - tau_i) and (tau_{i+k} - t) / (tau_{i+k} - tau_{i+1}).  kn
// points at tau_{l-2}, so kn[0..5] = tau_{l-2..l+3}; every denominator spans
// the interval [tau_l, tau_l+1) and is positive.
__device__ __forceinline__ void bspline4(const double* __restrict__ kn, double t, double B[4]) {
    // knot tau_{l+j} for j = -2..3
    auto tk = [&](int j) { return kn[j + 2]; };
    // order 2: B_{l-1}, B_l
    const double h0 = tk(1) - tk(0);
    const double b2m1 = (tk(1) - t) / h0, b20 = (t - tk(0)) / h0;
    // order 3: B_{l-2}, B_{l-1}, B_l
    const double b3m2 = (tk(1) - t) / (tk(1) - tk(-1)) * b2m1;
    const double b3m1 = (t - tk(-1)) / (tk(1) - tk(-1)) * b2m1 + (tk(2) - t) / (tk(2) - tk(0)) * b20;
    const double b30 = (t - tk(0)) / (tk(2) - tk(0)) * b20;
    // order 4: B_{l-3} .. B_l
    B[0] = (tk(1) - t) / (tk(1) - tk(-2)) * b3m2;
    B[1] = (t - tk(-2)) / (tk(1) - tk(-2)) * b3m2 + (tk(2) - t) / (tk(2) - tk(-1)) * b3m1;
    B[2] = (t - tk(-1)) / (tk(2) - tk(-1)) * b3m1 + (tk(3) - t) / (tk(3) - tk(0)) * b30;
    B[3] = (t - tk(0)) / (tk(3) - tk(0)) * b30;
}

// Attitude matrix A = S'C of a unit quaternion (eq:quat2mat), row-major.
__device__ __forceinline__ void quat2mat(const double q[4], double A[9]) {
    const double x = q[0], y = q[1], z = q[2], w = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z);
    A[1] = 2.0 * (x * y + z * w);
    A[2] = 2.0 * (x * z - y * w);
    A[3] = 2.0 * (x * y - z * w);
    A[4] = 1.0 - 2.0 * (x * x + z * z);
    A[5] = 2.0 * (y * z + x * w);
    A[6] = 2.0 * (x * z + y * w);
    A[7] = 2.0 * (y * z - x * w);
    A[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Attitude matrix of the rotation represented by any non-zero quaternion:
// eq:quat2mat written in the homogeneous form (w^2 + x^2 - y^2 - z^2, ...)
// and divided by |q|^2, with inv_n2 = 1/|q|^2.  For a unit quaternion it is
// eq:quat2mat itself; a rounding error in |q| only scales the matrix, which
// leaves every direction computed from it unchanged.
__device__ __forceinline__ void quat2mat_h(const double q[4], double inv_n2, double A[9]) {
    const double x = q[0], y = q[1], z = q[2], w = q[3];
    const double xx = x * x, yy = y * y, zz = z * z, ww = w * w;
    const double s2 = 2.0 * inv_n2;
    A[0] = (ww + xx - yy - zz) * inv_n2;
    A[1] = (x * y + z * w) * s2;
    A[2] = (x * z - y * w) * s2;
    A[3] = (x * y - z * w) * s2;
    A[4] = (ww - xx + yy - zz) * inv_n2;
    A[5] = (y * z + x * w) * s2;
    A[6] = (x * z + y * w) * s2;
    A[7] = (y * z - x * w) * s2;
    A[8] = (ww - xx - yy + zz) * inv_n2;
}

// Everything one observation contributes; filled by observe().
struct ObsEval {
    double R;          // residual eta_obs + c - eta (across scan: zeta_obs - zeta)
    double ubar[3];    // coordinate direction <r + tau mu - plx b>
    double vc[3];      // v_G / c
    double b[3];       // observer position [AU]
    double tau;        // (t_B - t_ep) [yr]
    double Su[3];      // proper direction in the SRS
    double rho;        // sqrt(Su_x^2 + Su_y^2) = cos(zeta)
    double inv_rho;    // 1 / rho
    double q[4];       // normalised attitude quaternion
    double qraw[4];    // sum a_n B_n (not normalised)
    double D;          // 1 - |qraw|^2 (eq:Dl)
    double B[4];       // B_{l-3..l}(t)
    double A[9];       // attitude matrix
    double dudg[3];    // d(coordinate direction)/d g0 of the light deflection (0 without it)
};

// Observation model (eq:roemer, eq:astro-standard, eq:classAberr,
// eq:qspline, eq:srsprop, eq:srsprop1, eq:srspropeta, eq:resAL) for the
// circular barycentric orbit of the synthetic world.  a4: the four
// coefficients a_{l-3..l} (x,y,z,w each); kn: tau_{l-2..l+3} (read only when
// the knots are not equally spaced); kt: the interval's table entry.
// Evaluated with per-interval tables and without library transcendentals:
//  * the ephemeris from sin/cos of the orbital longitude at tau_l rotated by
//    the small angle d = Lrate (t - tau_l) (Taylor series to d^6);
//  * on equally spaced knots the cubic B-splines in closed form
//    ((1-u)^3, 3u^3 - 6u^2 + 4, -3u^3 + 3u^2 + 3u + 1, u^3) / 6 with
//    u = (t - tau_l) / (tau_l+1 - tau_l), otherwise the general recursion
//    of bspline4;
//  * the field angle as atan(y'/x') of the SRS direction rotated by the
//    field's Gamma_c/2 (odd series to z^9 for |z| < 1e-2, atan2 otherwise);
//  * normalisations by Newton-refined reciprocal square roots.
// Every replacement equals the plain form to rounding.  ac: an across-scan
// observation; eta_obs then holds the observed zeta, cal is zero and R is
// zeta_obs - zeta, with zeta = atan(z / rho) (the same odd series for
// |z / rho| < 1e-2, atan2 otherwise).
// DEFL: with the Sun's light deflection (k.defl, gamma = 1 + k.gpar[0]);
// the instances without it are the plain model.
template <bool DEFL = false>
__device__ __forceinline__ void observe(const DevConsts& k, double t, double eta_obs, double cal,
                                            const double r[3], const double mu[3], double plx,
                                            const double* __restrict__ a4, const double* __restrict__ kn,
                                            const KnotTab& kt, ObsEval& o, bool ac = false) {
    double v[3];
    {
        const double d = k.eph_Lrate * (t - kt.tau);
        double sL, cL;
        if (fabs(d) < 1e-2) {
            const double d2 = d * d;
            const double sd = d * (1.0 - d2 * (1.0 / 6.0 - d2 * (1.0 / 120.0)));
            const double cd = 1.0 - d2 * (0.5 - d2 * (1.0 / 24.0 - d2 * (1.0 / 720.0)));
            sL = kt.sL * cd + kt.cL * sd;
            cL = kt.cL * cd - kt.sL * sd;
        } else {
            sincos(k.eph_L0 + k.eph_Lrate * t, &sL, &cL);
        }
        const double bx = k.eph_r * cL, by = k.eph_r * sL;
        o.b[0] = bx;
        o.b[1] = k.cos_obl * by;
        o.b[2] = k.sin_obl * by;
        const double w = k.eph_r * k.eph_Lrate;
        const double vx = -w * sL, vy = w * cL;
        v[0] = vx;
        v[1] = k.cos_obl * vy;
        v[2] = k.sin_obl * vy;
    }
    const double tB = t + dot3(r, o.b) * k.au_c;
    o.tau = (tB - k.t_ep) * k.inv_year;
    double ub[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ub[c] = r[c] + o.tau * mu[c] - plx * o.b[c];
    const double iub = rsqrt_nr(dot3(ub, ub));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o.ubar[c] = ub[c] * iub;
        o.vc[c] = v[c] * k.au_c;
    }
    // the Sun's light deflection (gamma = 1 + g0), first order in GM/(c^2 r):
    // the coordinate direction moves by (1 + gamma) GM/(c^2 r) (e - (e.u) u) /
    // (1 + e.u), e the unit vector from the Sun (the barycentre here) to
    // the observer at distance r
    double uu[3];
    if constexpr (DEFL) {
        const double ib = rsqrt_nr(dot3(o.b, o.b));
        const double eu = dot3(o.b, o.ubar) * ib;
        const double f = k.defl * ib / (1.0 + eu);
        const double gam1 = 2.0 + k.gpar[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.dudg[c] = f * (o.b[c] * ib - eu * o.ubar[c]);
            uu[c] = o.ubar[c] + gam1 * o.dudg[c] + o.vc[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.dudg[c] = 0.0;
            uu[c] = o.ubar[c] + o.vc[c];
        }
    }
    const double iuu = rsqrt_nr(dot3(uu, uu));
    double u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = uu[c] * iuu;

    if (kt.inv_dt > 0.0) {
        const double x = (t - kt.tau) * kt.inv_dt, x1 = 1.0 - x;
        const double x2 = x * x, x3 = x2 * x;
        const double s6 = 1.0 / 6.0;
        o.B[0] = x1 * x1 * x1 * s6;
        o.B[1] = (3.0 * x3 - 6.0 * x2 + 4.0) * s6;
        o.B[2] = (-3.0 * x3 + 3.0 * x2 + 3.0 * x + 1.0) * s6;
        o.B[3] = x3 * s6;
    } else {
        bspline4(kn, t, o.B);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        o.qraw[c] = a4[c] * o.B[0] + a4[4 + c] * o.B[1] + a4[8 + c] * o.B[2] + a4[12 + c] * o.B[3];
    const double n2 = o.qraw[0] * o.qraw[0] + o.qraw[1] * o.qraw[1] + o.qraw[2] * o.qraw[2] + o.qraw[3] * o.qraw[3];
    o.D = 1.0 - n2;
    const double iq = rsqrt_nr(n2);
#pragma unroll
    for (int c = 0; c < 4; ++c) o.q[c] = o.qraw[c] * iq;
    quat2mat_h(o.qraw, iq * iq, o.A);
    o.Su[0] = o.A[0] * u[0] + o.A[1] * u[1] + o.A[2] * u[2];
    o.Su[1] = o.A[3] * u[0] + o.A[4] * u[1] + o.A[5] * u[2];
    o.Su[2] = o.A[6] * u[0] + o.A[7] * u[1] + o.A[8] * u[2];
    const double rho2 = o.Su[0] * o.Su[0] + o.Su[1] * o.Su[1];
    o.inv_rho = rsqrt_nr(rho2);
    o.rho = rho2 * o.inv_rho;
    if (ac) {
        const double z = o.Su[2] * o.inv_rho, z2 = z * z;
        const double zeta = fabs(z) < 1e-2
                                ? z * (1.0 + z2 * (-1.0 / 3.0 + z2 * (1.0 / 5.0 + z2 * (-1.0 / 7.0 + z2 * (1.0 / 9.0)))))
                                : atan2(o.Su[2], o.rho);
        o.R = eta_obs - zeta;
        return;
    }
    // eta = phi - f Gamma_c / 2 with f = sign(phi): rotate (x, y) by -f Gamma_c/2
    const double f = o.Su[1] >= 0.0 ? 1.0 : -1.0;
    const double xr = o.Su[0] * k.cos_half_gamma + f * o.Su[1] * k.sin_half_gamma;
    const double yr = o.Su[1] * k.cos_half_gamma - f * o.Su[0] * k.sin_half_gamma;
    double eta;
    if (xr > 0.0 && fabs(yr) < 1e-2 * xr) {
        // the (cos, sin) pair rotates by atan2(sin, cos) = Gamma_c/2 - half_gamma_err
        const double z = yr * rcp_nr(xr), z2 = z * z;
        eta = z * (1.0 + z2 * (-1.0 / 3.0 + z2 * (1.0 / 5.0 + z2 * (-1.0 / 7.0 + z2 * (1.0 / 9.0))))) -
              f * k.half_gamma_err;
    } else {
        const double phi = atan2(o.Su[1], o.Su[0]);
        eta = phi >= 0.0 ? phi - k.gamma_half : phi + k.gamma_half;
    }
    o.R = eta_obs + cal - eta;
}

// Design row -dR/ds for (alpha*, delta, parallax, mu_a*, mu_d):
// eq:ubardiff, eq:duds, eq:srspropdiff with eq:srsprop1diffsol; the AL unit
// vector m of eq:srspqr is taken back to celestial coordinates once (across
// scan the AC unit vector n, and no factor sec(zeta)).
__device__ __forceinline__ void source_partials(const ObsEval& o, const double p[3], const double q[3],
                                                const double r[3], double Ad[5], bool ac = false) {
    const double inv_rho = o.inv_rho;
    double m[3];
    double secz = inv_rho;
    if (ac) {
        // n = (-sin zeta cos phi, -sin zeta sin phi, cos zeta)
        const double ns0 = -o.Su[2] * o.Su[0] * inv_rho, ns1 = -o.Su[2] * o.Su[1] * inv_rho, ns2 = o.rho;
        m[0] = o.A[0] * ns0 + o.A[3] * ns1 + o.A[6] * ns2;
        m[1] = o.A[1] * ns0 + o.A[4] * ns1 + o.A[7] * ns2;
        m[2] = o.A[2] * ns0 + o.A[5] * ns1 + o.A[8] * ns2;
        secz = 1.0;
    } else {
        const double ms0 = -o.Su[1] * inv_rho, ms1 = o.Su[0] * inv_rho;   // (-sin phi, cos phi, 0)
        m[0] = o.A[0] * ms0 + o.A[3] * ms1;
        m[1] = o.A[1] * ms0 + o.A[4] * ms1;
        m[2] = o.A[2] * ms0 + o.A[5] * ms1;
    }
    const double f = 1.0 - dot3(o.ubar, o.vc);
    const double mu_ = dot3(m, o.ubar);
    const double rb = dot3(r, o.b);
    double dpl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dpl[c] = -(o.b[c] - r[c] * rb);
    const double a0 = (f * dot3(m, p) - mu_ * dot3(o.vc, p)) * secz;
    const double a1 = (f * dot3(m, q) - mu_ * dot3(o.vc, q)) * secz;
    Ad[0] = a0;
    Ad[1] = a1;
    Ad[2] = (f * dot3(m, dpl) - mu_ * dot3(o.vc, dpl)) * secz;
    Ad[3] = a0 * o.tau;
    Ad[4] = a1 * o.tau;
}

// The global design entries (Sect. 5.4): -dR/dg0, the light deflection's
// derivative through the first-order aberration and the attitude, and the
// parallax entry of the source row (the pseudo-parameter g1, a global
// parallax shift); r: the source's direction.
__device__ __forceinline__ void global_partials(const ObsEval& o, const double r[3], double& a_g0, double& a_plx,
                                                bool ac = false) {
    const double inv_rho = o.inv_rho;
    double m[3];
    double secz = inv_rho;
    if (ac) {
        const double ns0 = -o.Su[2] * o.Su[0] * inv_rho, ns1 = -o.Su[2] * o.Su[1] * inv_rho, ns2 = o.rho;
        m[0] = o.A[0] * ns0 + o.A[3] * ns1 + o.A[6] * ns2;
        m[1] = o.A[1] * ns0 + o.A[4] * ns1 + o.A[7] * ns2;
        m[2] = o.A[2] * ns0 + o.A[5] * ns1 + o.A[8] * ns2;
        secz = 1.0;
    } else {
        const double ms0 = -o.Su[1] * inv_rho, ms1 = o.Su[0] * inv_rho;
        m[0] = o.A[0] * ms0 + o.A[3] * ms1;
        m[1] = o.A[1] * ms0 + o.A[4] * ms1;
        m[2] = o.A[2] * ms0 + o.A[5] * ms1;
    }
    const double f = 1.0 - dot3(o.ubar, o.vc);
    const double mu_ = dot3(m, o.ubar);
    const double rb = dot3(r, o.b);
    double dpl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dpl[c] = -(o.b[c] - r[c] * rb);
    a_plx = (f * dot3(m, dpl) - mu_ * dot3(o.vc, dpl)) * secz;
    a_g0 = (f * dot3(m, o.dudg) - mu_ * dot3(o.vc, o.dudg)) * secz;
}

// dR/dq = 2 sec(zeta) q {S'n, 0} (eq:dfadq), n of eq:srspqr; across scan
// dR/dq = -2 q {S'm, 0}.
__device__ __forceinline__ void attitude_partial(const ObsEval& o, double g[4], bool ac = false) {
    const double inv_rho = o.inv_rho;
    if (ac) {
        const double m0 = -o.Su[1] * inv_rho, m1 = o.Su[0] * inv_rho;
        const double* q = o.q;
        g[0] = -2.0 * (q[3] * m0 - q[2] * m1);
        g[1] = -2.0 * (q[3] * m1 + q[2] * m0);
        g[2] = -2.0 * (q[0] * m1 - q[1] * m0);
        g[3] = -2.0 * (-(q[0] * m0 + q[1] * m1));
        return;
    }
    const double sz = o.Su[2];
    const double n0 = -sz * o.Su[0] * inv_rho, n1 = -sz * o.Su[1] * inv_rho, n2 = o.rho;
    const double* q = o.q;
    // {q_v, q_w} {n, 0} = {q_w n + q_v x n, -q_v . n}
    const double s = 2.0 * inv_rho;
    g[0] = s * (q[3] * n0 + q[1] * n2 - q[2] * n1);
    g[1] = s * (q[3] * n1 + q[2] * n0 - q[0] * n2);
    g[2] = s * (q[3] * n2 + q[0] * n1 - q[1] * n0);
    g[3] = s * (-(q[0] * n0 + q[1] * n1 + q[2] * n2));
}

// Modified Cholesky factorisation U'U = N of a small dense symmetric
// positive semidefinite system (Appendix C: Algorithm C1's rule that a
// non-positive pivot makes its whole row of U zero and counts one rank
// defect; no pivoting), in right-looking form: each pivot row, once formed,
// is subtracted from the trailing rows as an outer product.  U holds the
// upper triangle of N row-major on entry and the factor on exit; returns the
// defect count.
template <int NN>
__device__ __forceinline__ int small_chol_factor(double U[NN * NN]) {
    int d = 0;
#pragma unroll
    for (int p = 0; p < NN; ++p) {
        const double piv = U[p * NN + p];
        if (piv > 0.0) {
            const double up = sqrt(piv);
            U[p * NN + p] = up;
#pragma unroll
            for (int c = p + 1; c < NN; ++c) U[p * NN + c] /= up;
            // trailing rows r > p, columns c >= r
#pragma unroll
            for (int r = p + 1; r < NN; ++r)
#pragma unroll
                for (int c = r; c < NN; ++c) U[r * NN + c] -= U[p * NN + r] * U[p * NN + c];
        } else {
            ++d;
#pragma unroll
            for (int c = p; c < NN; ++c) U[p * NN + c] = 0.0;
        }
    }
    return d;
}

// Solves U'U x = b with the factor of small_chol_factor (Algorithms C2 and
// C3: an unknown whose pivot is zero is set to zero), both triangular solves
// column by column: a solved unknown is removed from the remaining
// right-hand sides at once.  x holds b on entry.
template <int NN>
__device__ __forceinline__ void small_chol_subst(const double U[NN * NN], double x[NN]) {
    // U' y = b
#pragma unroll
    for (int p = 0; p < NN; ++p) {
        const double up = U[p * NN + p];
        x[p] = up > 0.0 ? x[p] / up : 0.0;
#pragma unroll
        for (int r = p + 1; r < NN; ++r) x[r] -= U[p * NN + r] * x[p];
    }
    // U x = y
#pragma unroll
    for (int p = NN - 1; p >= 0; --p) {
        const double up = U[p * NN + p];
        x[p] = up > 0.0 ? x[p] / up : 0.0;
#pragma unroll
        for (int r = 0; r < p; ++r) x[r] -= U[r * NN + p] * x[p];
    }
}

template <int NN>
__device__ __forceinline__ int small_chol_solve(double U[NN * NN], double x[NN]) {
    const int d = small_chol_factor<NN>(U);
    small_chol_subst<NN>(U, x);
    return d;
}

// Rotation quaternion Q(phi) of a rotation vector (eq:qrot).
__device__ __forceinline__ void qrot(const double phi[3], double out[4]) {
    const double ang = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (ang > 0.0) {
        double s, c;
        sincos(0.5 * ang, &s, &c);
        out[0] = phi[0] / ang * s;
        out[1] = phi[1] / ang * s;
        out[2] = phi[2] / ang * s;
        out[3] = c;
    } else {
        out[0] = 0.0;
        out[1] = 0.0;
        out[2] = 0.0;
        out[3] = 1.0;
    }
}

// Hamilton product {x, y, z, w} (eq:quatmult).
__device__ __forceinline__ void qmul(const double a[4], const double b[4], double o[4]) {
    o[0] = a[3] * b[0] + a[0] * b[3] + a[1] * b[2] - a[2] * b[1];
    o[1] = a[3] * b[1] - a[0] * b[2] + a[1] * b[3] + a[2] * b[0];
    o[2] = a[3] * b[2] + a[0] * b[1] - a[1] * b[0] + a[2] * b[3];
    o[3] = a[3] * b[3] - a[0] * b[0] - a[1] * b[1] - a[2] * b[2];
}

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace agis
