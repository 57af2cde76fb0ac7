/*
 * AGIS CPU oracle -- TEST INFRASTRUCTURE ONLY (see agis_oracle.h).
 *
 * Plain double-precision C (or x87 extended with ORC_EXTENDED), one formula
 * per paper equation, in the order the paper gives them.  No blocking, fusion or algebraic short-cuts beyond what
 * the equations state; loops over independent sources / segments may run in
 * parallel (results do not depend on the thread count).
 *
 * Citations name sections, equation labels and algorithms of Lindegren et
 * al. (2012), "The astrometric core solution for the Gaia mission".
 */
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

/* The same source also builds as a reference in x87 extended precision
 * (64-bit significand): every "double" below, including those of the header,
 * becomes "long double" and <tgmath.h> picks the matching libm routines.
 * The floating-point error of the FP64 build is measured against it. */
#ifdef ORC_EXTENDED
#define double long double
#endif
#include "agis_oracle.h"

#define M_ORDER 4

/* ========================================================================
 * Appendix A.1, quaternion algebra: product (eq:quatmult), conjugate
 * (eq:quatconj), inverse (eq:quatinv).  Quaternions are {x, y, z, w}.
 * ====================================================================== */
void orc_qmul(const double a[4], const double b[4], double out[4]) {
    double r[4];
    r[0] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    r[1] = -a[0] * b[2] + a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[2] = a[0] * b[1] - a[1] * b[0] + a[2] * b[3] + a[3] * b[2];
    r[3] = -a[0] * b[0] - a[1] * b[1] - a[2] * b[2] + a[3] * b[3];
    memcpy(out, r, sizeof r);
}

void orc_qconj(const double a[4], double out[4]) {
    out[0] = -a[0]; out[1] = -a[1]; out[2] = -a[2]; out[3] = a[3];
}

void orc_qinv(const double a[4], double out[4]) {
    double n2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3];
    out[0] = -a[0] / n2; out[1] = -a[1] / n2; out[2] = -a[2] / n2; out[3] = a[3] / n2;
}

/* Frame rotation (eq:quatframerot): {out, 0} = q^-1 {v, 0} q. */
void orc_frame_rotate(const double q[4], const double v[3], double out[3]) {
    double qi[4], vq[4] = {v[0], v[1], v[2], 0.0}, t[4], r[4];
    orc_qinv(q, qi);
    orc_qmul(qi, vq, t);
    orc_qmul(t, q, r);
    out[0] = r[0]; out[1] = r[1]; out[2] = r[2];
}

/* Vector rotation (eq:quatvecrot): {out, 0} = q {v, 0} q^-1. */
void orc_vector_rotate(const double q[4], const double v[3], double out[3]) {
    double qi[4], vq[4] = {v[0], v[1], v[2], 0.0}, t[4], r[4];
    orc_qinv(q, qi);
    orc_qmul(q, vq, t);
    orc_qmul(t, qi, r);
    out[0] = r[0]; out[1] = r[1]; out[2] = r[2];
}

/* Attitude matrix from a unit quaternion (eq:quat2mat), row-major. */
void orc_quat2mat(const double q[4], double A[9]) {
    double x = q[0], y = q[1], z = q[2], w = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z); A[1] = 2.0 * (x * y + z * w);       A[2] = 2.0 * (x * z - y * w);
    A[3] = 2.0 * (x * y - z * w);       A[4] = 1.0 - 2.0 * (x * x + z * z); A[5] = 2.0 * (y * z + x * w);
    A[6] = 2.0 * (x * z + y * w);       A[7] = 2.0 * (y * z - x * w);       A[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Rotation quaternion Q(phi) of a rotation vector (eq:qrot). */
void orc_qrot(const double phi[3], double out[4]) {
    double ang = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (ang > 0.0) {
        double s = sin(0.5 * ang);
        out[0] = phi[0] / ang * s; out[1] = phi[1] / ang * s; out[2] = phi[2] / ang * s;
        out[3] = cos(0.5 * ang);
    } else {
        out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 1.0;
    }
}

/* ========================================================================
 * Appendix B: left index (tau_l <= t < tau_{l+1}, restricted to the spline
 * interval [tau_{M-1}, tau_N]; t = tau_N belongs to the last interval) and
 * the M = 4 non-zero B-splines at a time.
 * ====================================================================== */
int64_t orc_left_index(const double* knots, int64_t n_knots, double t) {
    int64_t N = n_knots - M_ORDER;
    int64_t lo = M_ORDER - 1, hi = N - 1;       /* answer in [lo, hi] */
    if (t >= knots[N]) return N - 1;
    if (t <= knots[lo]) return lo;
    while (lo < hi) {                            /* largest l with tau_l <= t */
        int64_t mid = (lo + hi + 1) / 2;
        if (knots[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* The B-splines of order M on the knot sequence (Appendix B, Sect. B.2: they
 * are fixed by the knots alone; the definition is de Boor's): order 1 is
 * the indicator of [tau_i, tau_{i+1}), and order k is
 *   B_{i,k}(t) = (t - tau_i) / (tau_{i+k-1} - tau_i) B_{i,k-1}(t)
 *              + (tau_{i+k} - t) / (tau_{i+k} - tau_{i+1}) B_{i+1,k-1}(t),
 * a term whose knot difference is zero being left out.  At t in
 * [tau_ell, tau_ell+1) only B_{ell-M+1..ell} can be non-zero (Sect. B.3);
 * b[m] = B_{ell-M+1+m, M}(t). */
static double bspline_term(const double* knots, int64_t i, int k, double t, double lower_i, double lower_next) {
    double v = 0.0;
    double den_left = knots[i + k - 1] - knots[i];
    double den_right = knots[i + k] - knots[i + 1];
    if (den_left != 0.0) v += (t - knots[i]) / den_left * lower_i;
    if (den_right != 0.0) v += (knots[i + k] - t) / den_right * lower_next;
    return v;
}

void orc_bspline(const double* knots, int64_t ell, double t, double b[4]) {
    /* level[k][m]: B_{ell-M+1+m, k}(t), m = 0..M-1; zero off the support */
    double level[M_ORDER + 1][M_ORDER + 1];
    memset(level, 0, sizeof level);
    level[1][M_ORDER - 1] = 1.0;                     /* B_{ell,1}: t lies in [tau_ell, tau_ell+1) */
    for (int k = 2; k <= M_ORDER; ++k)
        for (int m = 0; m < M_ORDER; ++m) {
            int64_t i = ell - M_ORDER + 1 + m;
            level[k][m] = bspline_term(knots, i, k, t, level[k - 1][m], level[k - 1][m + 1]);
        }
    for (int m = 0; m < M_ORDER; ++m) b[m] = level[M_ORDER][m];
}

/* ========================================================================
 * Appendix C: the modified Cholesky decomposition N = U'U of a symmetric
 * positive semidefinite matrix (Algorithm C1) and the two triangular solves
 * (Algorithms C2, C3).  Dense row-major storage, upper triangle.
 *
 * C1 forms U column by column.  In column j, each entry above the diagonal
 * comes from its row's pivot U_ii: U_ij = (N_ij - sum_{k<i} U_ki U_kj) /
 * U_ii, or 0 when that pivot is not positive; then the pivot of column j is
 * the square root of N_jj - sum_{k<j} U_kj^2 when that is positive, else 0,
 * and each zero pivot counts one rank defect d.  The solves skip unknowns
 * whose pivot is zero (they are set to 0), which gives one valid solution of
 * a singular system.
 * ====================================================================== */
/* sum over k in [k_from, k_to) of U_ka U_kb */
static double column_dot(const double* U, int n, int a, int b, int k_from, int k_to) {
    double acc = 0.0;
    for (int k = k_from; k < k_to; ++k) acc += U[k * n + a] * U[k * n + b];
    return acc;
}

/* Entry (i, j), i <= j, of the factor from the entries above it (C1's rule). */
static double factor_entry(double* U, int n, int i, int j, int k_from, int* defect) {
    double rest = U[i * n + j] - column_dot(U, n, i, j, k_from, i);
    if (i < j) return U[i * n + i] > 0.0 ? rest / U[i * n + i] : 0.0;
    if (rest > 0.0) return sqrt(rest);
    *defect += 1;
    return 0.0;
}

int orc_chol_c1(double* U, int n) {
    int d = 0;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i <= j; ++i) U[i * n + j] = factor_entry(U, n, i, j, 0, &d);
        for (int i = j + 1; i < n; ++i) U[i * n + j] = 0.0;         /* lower triangle */
    }
    return d;
}

/* U' y = b (C2): y_i from the rows above it. */
void orc_chol_c2(const double* U, int n, double* y) {
    for (int i = 0; i < n; ++i) {
        double piv = U[i * n + i];
        double known = 0.0;
        for (int k = 0; k < i; ++k) known += U[k * n + i] * y[k];
        y[i] = piv > 0.0 ? (y[i] - known) / piv : 0.0;
    }
}

/* U x = y (C3): x_i from the unknowns after it. */
void orc_chol_c3(const double* U, int n, double* x) {
    for (int i = n - 1; i >= 0; --i) {
        double piv = U[i * n + i];
        double known = 0.0;
        for (int k = i + 1; k < n; ++k) known += U[i * n + k] * x[k];
        x[i] = piv > 0.0 ? (x[i] - known) / piv : 0.0;
    }
}

/* The same three algorithms restricted to a band envelope of half-width hb
 * (Appendix C: the factor of a band matrix keeps its envelope, no fill-in).
 * Entries outside the envelope are zero in N and in U, so every sum runs
 * over the envelope only, in the dense order. */
#define UBX(j, jj) UB[(int64_t)(j) * (hb + 1) + ((jj) - (j))]
static double band_column_dot(const double* UB, int hb, int a, int b, int k_from, int k_to) {
    double acc = 0.0;
    for (int k = k_from; k < k_to; ++k) acc += UBX(k, a) * UBX(k, b);
    return acc;
}

int orc_band_c1(double* UB, int n, int hb) {
    int d = 0;
    for (int j = 0; j < n; ++j) {
        int top = j - hb > 0 ? j - hb : 0;          /* first row of column j inside the envelope */
        for (int i = top; i <= j; ++i) {
            double rest = UBX(i, j) - band_column_dot(UB, hb, i, j, top, i);
            if (i < j) {
                UBX(i, j) = UBX(i, i) > 0.0 ? rest / UBX(i, i) : 0.0;
            } else if (rest > 0.0) {
                UBX(j, j) = sqrt(rest);
            } else {
                UBX(j, j) = 0.0;
                d += 1;
            }
        }
    }
    return d;
}

void orc_band_c2(const double* UB, int n, int hb, double* y) {
    for (int i = 0; i < n; ++i) {
        int top = i - hb > 0 ? i - hb : 0;
        double known = 0.0;
        for (int k = top; k < i; ++k) known += UBX(k, i) * y[k];
        y[i] = UBX(i, i) > 0.0 ? (y[i] - known) / UBX(i, i) : 0.0;
    }
}

void orc_band_c3(const double* UB, int n, int hb, double* x) {
    for (int i = n - 1; i >= 0; --i) {
        int last = i + hb < n - 1 ? i + hb : n - 1;
        double known = 0.0;
        for (int k = i + 1; k <= last; ++k) known += UBX(i, k) * x[k];
        x[i] = UBX(i, i) > 0.0 ? (x[i] - known) / UBX(i, i) : 0.0;
    }
}
#undef UBX

/* ========================================================================
 * Sect. 3.2: normal triad of a source (eq:normal-triad).
 * ====================================================================== */
void orc_normal_triad(double alpha, double delta, double p[3], double q[3], double r[3]) {
    double sa = sin(alpha), ca = cos(alpha), sd = sin(delta), cd = cos(delta);
    p[0] = -sa;      p[1] = ca;       p[2] = 0.0;
    q[0] = -sd * ca; q[1] = -sd * sa; q[2] = cd;
    r[0] = cd * ca;  r[1] = cd * sa;  r[2] = sd;
}

/* Barycentric position [AU] and velocity [AU/s] of the observer: the
 * synthetic world's circular orbit in the ecliptic, rotated to the
 * equatorial frame (auxiliary data of eq:astro). */
void orc_ephemeris(const orc_world_t* w, double t, double b[3], double v[3]) {
    double L = w->eph_L0 + w->eph_Lrate * t;
    double ce = cos(w->eps_obl), se = sin(w->eps_obl);
    double be[3] = {w->eph_radius_au * cos(L), w->eph_radius_au * sin(L), 0.0};
    double ve[3] = {-w->eph_radius_au * w->eph_Lrate * sin(L), w->eph_radius_au * w->eph_Lrate * cos(L), 0.0};
    b[0] = be[0]; b[1] = ce * be[1] - se * be[2]; b[2] = se * be[1] + ce * be[2];
    v[0] = ve[0]; v[1] = ce * ve[1] - se * ve[2]; v[2] = se * ve[1] + ce * ve[2];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Everything the model computes for one observation. */
typedef struct {
    int64_t ell;
    double B[4];
    double qraw[4], D, q[4];
    double p[3], qv[3], r[3];
    double bG[3], vG[3], vc[3];
    double tau;                 /* (t_B - t_ep) in years */
    double ubar[3], u[3], Su[3];
    double dudg[3];             /* d(coordinate direction)/d g0 of the light deflection */
    double phi, zeta, eta, R;
    int f;
    int ac;                     /* 1: across-scan observation (cell < 0) */
} orc_fwd_t;

/* Shifted Legendre polynomial of degree r = 0, 1, 2, orthogonal on [0, 1]
 * (eq:etazeta). */
static double shifted_legendre(int r, double x) {
    if (r == 0) return 1.0;
    if (r == 1) return 2.0 * x - 1.0;
    return 6.0 * x * x - 6.0 * x + 1.0;
}

/* Index of the first of the three geometric coefficients of a record: an
 * along-scan record's cell and CCD (the AL term of eq:etazeta); with the AC
 * calibration an across-scan record's cell and CCD among the AC groups,
 * which follow all the AL ones (the AC term); -1 for an across-scan record
 * without it. */
static int64_t geo_index(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l) {
    if (obs->cell[l] >= 0) return 3 * ((int64_t)obs->cell[l] * w->geo_ccds + obs->ccd[l]);
    if (!obs->ac_cell) return -1;
    return 3 * ((st->n_cells + (int64_t)obs->ac_cell[l]) * w->geo_ccds + obs->ccd[l]);   /* AC cells follow */
}

/* Argument of the shifted Legendre polynomials: the AC pixel coordinate
 * mapped to [0, 1] (eq:etazeta). */
static double geo_x(const orc_obs_t* obs, int64_t l) { return ((double)obs->mu[l] - 13.5) / 1966.0; }

/* Pixel columns of the small-scale AL term (eq:etazeta): m = 14 .. 1979. */
#define GEO_COLS 1966

/* Number of long intervals k of the small-scale AL term: the days of the
 * cells (two cells a day) in runs of geo_small_days; 0 without the term. */
static int64_t small_intervals(const orc_world_t* w, const orc_state_t* st) {
    if (w->geo_ccds <= 0 || w->geo_small_days <= 0) return 0;
    return (st->n_cells / 2 + w->geo_small_days - 1) / w->geo_small_days;
}

/* First small-scale coefficient: after the AL groups and, with ac_cell,
 * the AC groups. */
static int64_t small_base(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st) {
    return (st->n_cells + (obs->ac_cell ? (int64_t)w->geo_ac_cells : 0)) * w->geo_ccds * 3;
}

/* The nearest pixel column m = round(mu) of eq:etazeta as 0 .. 1965 (a
 * coordinate of exactly 1979.5 stays on the last column). */
static int64_t geo_column(const orc_obs_t* obs, int64_t l) {
    int64_t m = (int64_t)floor((double)obs->mu[l] + 0.5);
    if (m > 1979) m = 1979;
    return m - 14;
}

/* Index of an along-scan record's small-scale coefficient (its long
 * interval, CCD and column), or -1 (across scan, or no small-scale term). */
static int64_t small_index(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l) {
    if (small_intervals(w, st) == 0 || obs->cell[l] < 0) return -1;
    const int64_t k = (obs->cell[l] / 2) / w->geo_small_days;
    return small_base(w, obs, st) + (k * w->geo_ccds + obs->ccd[l]) * GEO_COLS + geo_column(obs, l);
}

/* The geometric calibration of a record (eq:etazeta): sum over r of its
 * group's coefficients times L*_r(x), plus along scan the small-scale
 * coefficient of its column when the world has that term; 0 without the
 * geometric model, or across scan without the AC calibration. */
static double geo_term(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l) {
    if (w->geo_ccds <= 0) return 0.0;
    const int64_t g = geo_index(w, obs, st, l);
    if (g < 0) return 0.0;
    const double x = geo_x(obs, l);
    double v = 0.0;
    for (int r = 0; r < 3; ++r) v += st->geo[g + r] * shifted_legendre(r, x);
    const int64_t q = small_index(w, obs, st, l);
    if (q >= 0) v += st->geo[q];
    return v;
}

/* Sect. 3.2-3.5: the computed field angles and the residual: eq:resAL for
 * an along-scan observation, eq:resAC (observed minus computed zeta, no
 * calibration term) for an across-scan one, marked by cell < 0. */
static void forward_one(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                        int64_t l, orc_fwd_t* o) {
    const double t = obs->t[l];
    const double* s = st->s + 5 * (int64_t)obs->src[l];
    /* eq:qspline with Algorithm B1 */
    o->ell = orc_left_index(w->knots, w->n_knots, t);
    orc_bspline(w->knots, o->ell, t, o->B);
    for (int c = 0; c < 4; ++c) o->qraw[c] = 0.0;
    for (int k = 0; k < M_ORDER; ++k) {
        const double* an = st->a + 4 * (o->ell - M_ORDER + 1 + k);
        for (int c = 0; c < 4; ++c) o->qraw[c] += an[c] * o->B[k];
    }
    double n2 = o->qraw[0] * o->qraw[0] + o->qraw[1] * o->qraw[1] + o->qraw[2] * o->qraw[2] + o->qraw[3] * o->qraw[3];
    o->D = 1.0 - n2;                                   /* eq:Dl */
    double nq = sqrt(n2);
    for (int c = 0; c < 4; ++c) o->q[c] = o->qraw[c] / nq;
    /* eq:normal-triad, eq:roemer, eq:astro-standard (mu_r = 0) */
    orc_normal_triad(s[0], s[1], o->p, o->qv, o->r);
    orc_ephemeris(w, t, o->bG, o->vG);
    double tB = t + dot3(o->r, o->bG) * w->au_m / w->c_mps;
    o->tau = (tB - w->t_ep) / w->year_s;
    double ub[3];
    for (int k = 0; k < 3; ++k)
        ub[k] = o->r[k] + o->tau * (o->p[k] * s[3] + o->qv[k] * s[4]) - s[2] * o->bG[k];
    double nub = sqrt(dot3(ub, ub));
    for (int k = 0; k < 3; ++k) o->ubar[k] = ub[k] / nub;
    /* light deflection by the Sun (eq:astro, with gamma = 1 + g0 of
     * eq:gammaPPN), to first order in GM/(c^2 r) for a source at infinity:
     * the coordinate direction moves by (1 + gamma) GM/(c^2 r) (e - (e.u)u) /
     * (1 + e.u) towards e, the unit vector from the Sun to the observer at
     * distance r (the Sun sits at the barycentre of the synthetic world) */
    double ud[3];
    for (int k = 0; k < 3; ++k) {
        ud[k] = o->ubar[k];
        o->dudg[k] = 0.0;
    }
    if (w->defl > 0.0) {
        const double rb = sqrt(dot3(o->bG, o->bG));
        double e[3];
        for (int k = 0; k < 3; ++k) e[k] = o->bG[k] / rb;
        const double eu = dot3(e, o->ubar);
        const double f = w->defl / rb / (1.0 + eu);
        for (int k = 0; k < 3; ++k) {
            o->dudg[k] = f * (e[k] - eu * o->ubar[k]);
            ud[k] = o->ubar[k] + (2.0 + st->g0) * o->dudg[k];
        }
    }
    /* eq:classAberr */
    for (int k = 0; k < 3; ++k) o->vc[k] = o->vG[k] * w->au_m / w->c_mps;
    double uu[3];
    for (int k = 0; k < 3; ++k) uu[k] = ud[k] + o->vc[k];
    double nu = sqrt(dot3(uu, uu));
    for (int k = 0; k < 3; ++k) o->u[k] = uu[k] / nu;
    /* eq:srsprop, eq:srsprop1, eq:srspropeta */
    orc_frame_rotate(o->q, o->u, o->Su);
    o->phi = atan2(o->Su[1], o->Su[0]);
    o->zeta = atan2(o->Su[2], sqrt(o->Su[0] * o->Su[0] + o->Su[1] * o->Su[1]));
    o->f = o->phi >= 0.0 ? 1 : -1;
    o->eta = o->phi - o->f * 0.5 * w->gamma_c;
    /* eq:resAL with the generic calibration model (eq:generic1); eq:resAC */
    o->ac = obs->cell[l] < 0;
    o->R = o->ac ? obs->eta_obs[l] + geo_term(w, obs, st, l) - o->zeta
                 : obs->eta_obs[l] + geo_term(w, obs, st, l) + st->c[obs->cell[l]] - o->eta;
}

/* Sect. 5.1.3: design row -dR/ds for (alpha*, delta, parallax, mu_alpha*,
 * mu_delta): eq:ubardiff, eq:duds, eq:srspropdiff, eq:srspqr,
 * eq:srsprop1diffsol.  Along scan d phi = sec(zeta) m'du, across scan
 * d zeta = n'du, with m and n of eq:srspqr in the SRS. */
static void source_partials(const orc_fwd_t* o, double A[5]) {
    double dub[5][3];
    for (int k = 0; k < 3; ++k) {
        double Ib = o->bG[k] - o->r[k] * dot3(o->r, o->bG);
        dub[0][k] = o->p[k];
        dub[1][k] = o->qv[k];
        dub[2][k] = -Ib;
        dub[3][k] = o->p[k] * o->tau;
        dub[4][k] = o->qv[k] * o->tau;
    }
    double ubv = dot3(o->ubar, o->vc);
    double sp = sin(o->phi), cp = cos(o->phi), sz = sin(o->zeta), cz = cos(o->zeta);
    double m[3] = {-sp, cp, 0.0};
    double n[3] = {-sz * cp, -sz * sp, cz};
    for (int j = 0; j < 5; ++j) {
        double du[3];
        double vd = dot3(o->vc, dub[j]);
        for (int k = 0; k < 3; ++k) du[k] = (1.0 - ubv) * dub[j][k] - o->ubar[k] * vd;
        double dSu[3];
        orc_frame_rotate(o->q, du, dSu);
        A[j] = o->ac ? dot3(n, dSu) : dot3(m, dSu) / cz;
    }
}

/* Sect. 5.4: the global design entry -dR/dg0, in analogy with the source
 * partials: the deflection's derivative d(ubar)/dg0 through the aberration
 * (to first order in v/c) and the attitude into the field angle. */
static double global_partial(const orc_fwd_t* o) {
    const double ubv = dot3(o->ubar, o->vc);
    const double vd = dot3(o->vc, o->dudg);
    double du[3], dSu[3];
    for (int k = 0; k < 3; ++k) du[k] = (1.0 - ubv) * o->dudg[k] - o->ubar[k] * vd;
    orc_frame_rotate(o->q, du, dSu);
    const double sp = sin(o->phi), cp = cos(o->phi), sz = sin(o->zeta), cz = cos(o->zeta);
    const double m[3] = {-sp, cp, 0.0};
    const double n[3] = {-sz * cp, -sz * sp, cz};
    return o->ac ? dot3(n, dSu) : dot3(m, dSu) / cz;
}

/* Sect. 5.2.3: dR_AL/dq = -(eq:dfadq) = 2 sec(zeta) q {S'n, 0}; across
 * scan dR_AC/dq = -(eq:dfadq) = -2 q {S'm, 0}. */
static void attitude_partial(const orc_fwd_t* o, double g[4]) {
    double sp = sin(o->phi), cp = cos(o->phi), sz = sin(o->zeta), cz = cos(o->zeta);
    double v[4] = {-sz * cp, -sz * sp, cz, 0.0};
    double f = 2.0 / cz;
    if (o->ac) {
        v[0] = -sp;
        v[1] = cp;
        v[2] = 0.0;
        f = -2.0;
    }
    double t[4];
    orc_qmul(o->q, v, t);
    for (int c = 0; c < 4; ++c) g[c] = f * t[c];
}

void orc_observe(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                 int64_t i0, int64_t i1,
                 double* eta, double* phi, double* zeta, int8_t* f, double* R,
                 double* dsrc, double* dq, double* bspl, int64_t* ell, double* qraw, double* D) {
#pragma omp parallel for schedule(static)
    for (int64_t l = i0; l < i1; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        if (eta) eta[l] = o.eta;
        if (phi) phi[l] = o.phi;
        if (zeta) zeta[l] = o.zeta;
        if (f) f[l] = (int8_t)o.f;
        if (R) R[l] = o.R;
        if (dsrc) source_partials(&o, dsrc + 5 * l);
        if (dq) attitude_partial(&o, dq + 4 * l);
        if (bspl) for (int k = 0; k < 4; ++k) bspl[4 * l + k] = o.B[k];
        if (ell) ell[l] = o.ell;
        if (qraw) for (int k = 0; k < 4; ++k) qraw[4 * l + k] = o.qraw[k];
        if (D) D[l] = o.D;
    }
}

/* Observations grouped by source, each group in input order (stable). */
static void group_by_source(const orc_obs_t* obs, int64_t n_src, int64_t** off_out, int64_t** idx_out) {
    int64_t* off = (int64_t*)calloc((size_t)n_src + 1, sizeof(int64_t));
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(obs->n > 0 ? obs->n : 1));
    for (int64_t l = 0; l < obs->n; ++l) off[obs->src[l] + 1] += 1;
    for (int64_t i = 0; i < n_src; ++i) off[i + 1] += off[i];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_src > 0 ? n_src : 1));
    for (int64_t i = 0; i < n_src; ++i) pos[i] = off[i];
    for (int64_t l = 0; l < obs->n; ++l) idx[pos[obs->src[l]]++] = l;
    free(pos);
    *off_out = off;
    *idx_out = idx;
}

/* ========================================================================
 * Sect. 5.1.2 and 5.2.5: robust weighting.
 * ====================================================================== */
/* eq:dw: 1 up to |z| = 2, a cubic in t = |z| - 2 up to 3, exp(-|z|/3) beyond. */
double orc_weight_function(double z) {
    double a = fabs(z);
    if (a <= 2.0) return 1.0;
    if (a < 3.0) {
        double t = a - 2.0;
        return 1.0 - 1.773735 * t * t + 1.141615 * t * t * t;
    }
    return exp(-a / 3.0);
}

static int cmp_real(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

double orc_quantile(const double* x, int64_t n, double p) {
    if (n <= 0) return 0.0;
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    memcpy(y, x, sizeof(double) * (size_t)n);
    qsort(y, (size_t)n, sizeof(double), cmp_real);
    double h = (double)(n - 1) * p;
    int64_t j = (int64_t)floor(h);
    double q = j + 1 < n ? y[j] + (h - (double)j) * (y[j + 1] - y[j]) : y[n - 1];
    free(y);
    return q;
}

/* Knot interval of an observation (left index l, interval l - 3) and its
 * excess-noise bucket. */
static int64_t bucket_of(const orc_world_t* w, int64_t ell) { return (ell - (M_ORDER - 1)) / w->eps_bucket; }

/* The attitude component an observation measures (Sect. 3.6: three excess
 * noise functions): along scan, or across scan in the preceding or in the
 * following field of view.  eps_a2 holds n_buckets values per component,
 * AL first, then ACP, then ACF. */
static int64_t eps_slot(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l,
                        int64_t ell) {
    int64_t comp = obs->cell[l] >= 0 ? 0 : (obs->fov[l] > 0 ? 1 : 2);
    return comp * st->n_buckets + bucket_of(w, ell);
}

/* The observation's uncertainty: sigma_l, or the frozen sigma_eff that
 * replaces it. */
static double obs_sigma(const orc_obs_t* obs, int64_t l) {
    return obs->sigma_eff ? obs->sigma_eff[l] : (double)obs->sigma[l];
}

/* sigma~_l^2 = sigma_l^2 + eps_a^2(t_l) of the observation's component
 * (eq:W with eps_i = 0). */
static double sigma_tilde2(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l,
                           int64_t ell) {
    double s = obs_sigma(obs, l);
    double v = s * s;
    if (w->robust) v += st->eps_a2[eps_slot(w, obs, st, l, ell)];
    return v;
}

/* eps_i^2 of the observation's source from the last S update (robust 2;
 * 0 otherwise or before any). */
static double source_eps2(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l) {
    return (w->robust == 2 && st->src_eps2) ? st->src_eps2[obs->src[l]] : 0.0;
}

/* Statistical weight W_l = w_l / (sigma~_l^2 + eps_i^2) (eq:W, eq:wl) for
 * the attitude and calibration updates: w_l from the residual R_l of the
 * pass, the latest excess attitude noise and (robust 2) the source's excess
 * noise (Sect. 5.2.5); w_l = 1 when not robust. */
static double weight(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t l,
                     const orc_fwd_t* o) {
    double v = sigma_tilde2(w, obs, st, l, o->ell) + source_eps2(w, obs, st, l);
    double wl = w->robust ? orc_weight_function(o->R / sqrt(v)) : 1.0;
    return wl / v;
}

/* eq e09 for each component and bucket: the observations of the component
 * in the bucket's knot intervals. */
void orc_excess_attitude_noise(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st) {
    if (!w->robust || st->n_buckets <= 0) return;
    int64_t nb = 3 * st->n_buckets;
    int64_t* cnt = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
    int64_t* bk = (int64_t*)malloc(sizeof(int64_t) * (size_t)(obs->n > 0 ? obs->n : 1));
    double* v = (double*)malloc(sizeof(double) * (size_t)(obs->n > 0 ? obs->n : 1));
    double* x = (double*)malloc(sizeof(double) * (size_t)(obs->n > 0 ? obs->n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double s = obs_sigma(obs, l);
        bk[l] = eps_slot(w, obs, st, l, o.ell);
        v[l] = o.R * o.R - s * s - source_eps2(w, obs, st, l);     /* e09 */
    }
    for (int64_t l = 0; l < obs->n; ++l) cnt[bk[l] + 1] += 1;
    for (int64_t j = 0; j < nb; ++j) cnt[j + 1] += cnt[j];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
    for (int64_t j = 0; j < nb; ++j) pos[j] = cnt[j];
    for (int64_t l = 0; l < obs->n; ++l) x[pos[bk[l]]++] = v[l];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nb; ++j) {
        double q = orc_quantile(x + cnt[j], cnt[j + 1] - cnt[j], 0.68);
        st->eps_a2[j] = q > 0.0 ? q : 0.0;
    }
    free(cnt); free(bk); free(v); free(x); free(pos);
}

/* ========================================================================
 * Sect. 5.1: source update.  For each source: eq:normS / eq:normSmat with
 * the design matrix eq:designS and h = R (eq:designSrhs), solved by
 * Algorithms C1-C3; Q_i from eq:Qi; alpha updated through d_1 = dalpha cos
 * delta (footnote to eq:ubardiff).
 * Robust (Sect. 5.1.2): initial downweights w_l = w(h_l / varsigma_i),
 * varsigma_i half the intersextile range of the h_l; then four rounds, the
 * weights of each after the first set to w(R_l / (sigma~_l^2 + eps_i^2)^1/2)
 * from the previous round's residuals R_l = h_l - A_l d (eq:wl).  robust 1:
 * eps_i = 0; robust 2: each round finds eps_i^2 for its weights (eq:epsi).
 * ====================================================================== */
#define ORC_INNER_SOLVES 4
#define ORC_EPS_STEPS 3     /* rational steps of eq:epsi (the paper finds 2-3 sufficient) */

/* eq:normS with W_l = w_l / (sigma~_l^2 + y) (eq:W), solved by C1-C3; N
 * keeps the factor (for the variances), b the solution; returns the defect. */
static int source_normals_solve(const double* Ab, const double* hb, const double* Vb, const double* wb, int64_t ni,
                                double y, double N[25], double b[5]) {
    for (int e = 0; e < 25; ++e) N[e] = 0.0;
    for (int e = 0; e < 5; ++e) b[e] = 0.0;
    for (int64_t k = 0; k < ni; ++k) {
        const double* A = Ab + 5 * k;
        double W = wb[k] / (Vb[k] + y);
        for (int r = 0; r < 5; ++r) {
            for (int c = 0; c < 5; ++c) N[5 * r + c] += A[r] * W * A[c];
            b[r] += A[r] * W * hb[k];
        }
    }
    int def = orc_chol_c1(N, 5);
    orc_chol_c2(N, 5, b);
    orc_chol_c3(N, 5, b);
    return def;
}

/* Q(y) = sum W_l R_l^2 of eq:Qi at the solution b, and its derivative
 * Q'(y) = -sum w_l R_l^2 / (sigma~_l^2 + y)^2 (the solution's own change
 * does not enter: it minimises Q). */
static void source_q(const double* Ab, const double* hb, const double* Vb, const double* wb, int64_t ni, double y,
                     const double b[5], double* Q, double* Qp) {
    double q = 0.0, qp = 0.0;
    for (int64_t k = 0; k < ni; ++k) {
        double Rk = hb[k];
        for (int c = 0; c < 5; ++c) Rk -= Ab[5 * k + c] * b[c];
        double v = Vb[k] + y;
        q += wb[k] / v * Rk * Rk;
        qp -= wb[k] * Rk * Rk / (v * v);
    }
    *Q = q;
    *Qp = qp;
}

void orc_source_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st,
                       double* d_out, double* Q_out, int32_t* defect_out, double* var_out) {
    int64_t *off, *idx;
    group_by_source(obs, st->n_src, &off, &idx);
#pragma omp parallel
    {
        int64_t cap = 0;
        double *Ab = NULL, *hb = NULL, *Vb = NULL, *wb = NULL, *xb = NULL;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < st->n_src; ++i) {
            int64_t ni = off[i + 1] - off[i];
            if (ni > cap) {
                cap = ni;
                Ab = (double*)realloc(Ab, sizeof(double) * 5 * cap);
                hb = (double*)realloc(hb, sizeof(double) * cap);
                Vb = (double*)realloc(Vb, sizeof(double) * cap);
                wb = (double*)realloc(wb, sizeof(double) * cap);
                xb = (double*)realloc(xb, sizeof(double) * cap);
            }
            for (int64_t k = 0; k < ni; ++k) {
                int64_t l = idx[off[i] + k];
                orc_fwd_t o;
                forward_one(w, obs, st, l, &o);
                source_partials(&o, Ab + 5 * k);
                hb[k] = o.R;
                Vb[k] = sigma_tilde2(w, obs, st, l, o.ell);
                wb[k] = 1.0;
            }
            int n_solve = 1;
            if (w->robust) {
                /* initial downweights: varsigma_i from the source's residuals
                 * of the observation's own kind (along scan, across scan),
                 * whose scales differ by sigma_AC / sigma_AL */
                n_solve = ORC_INNER_SOLVES;
                double vs[2];
                for (int kind = 0; kind < 2; ++kind) {
                    int64_t nk = 0;
                    for (int64_t k = 0; k < ni; ++k)
                        if ((obs->cell[idx[off[i] + k]] < 0) == kind) xb[nk++] = hb[k];
                    vs[kind] = 0.5 * (orc_quantile(xb, nk, 5.0 / 6.0) - orc_quantile(xb, nk, 1.0 / 6.0));
                }
                for (int64_t k = 0; k < ni; ++k) {
                    double v = vs[obs->cell[idx[off[i] + k]] < 0];
                    wb[k] = v > 0.0 ? orc_weight_function(hb[k] / v) : 1.0;
                }
            }
            double N[25], b[5];
            int def = 0;
            double y = 0.0, D = 0.0;          /* eps_i^2 and its significance (eq:epsi, eq:D) */
            for (int it = 0; it < n_solve; ++it) {
                if (it > 0) {
                    /* eq:wl with the previous round's solution and eps_i */
                    for (int64_t k = 0; k < ni; ++k) {
                        double Rk = hb[k];
                        for (int c = 0; c < 5; ++c) Rk -= Ab[5 * k + c] * b[c];
                        wb[k] = orc_weight_function(Rk / sqrt(Vb[k] + y));
                    }
                }
                if (w->robust == 2) {
                    /* Sect. 5.1.2: for these w_l, eps_i^2 = 0 if Q(0) <= nu, else the
                     * solution of Q(y) = nu by the steps dy = (1 - Q/nu) Q / Q'
                     * from y = 0 (three of them); nu = n_i - n_out - 5 with n_out
                     * the observations with w_l < 0.2 */
                    int64_t nout = 0;
                    for (int64_t k = 0; k < ni; ++k) nout += wb[k] < 0.2 ? 1 : 0;
                    double nu = (double)(ni - nout - 5);
                    y = 0.0;
                    double Q = 0.0, Qp = 0.0;
                    for (int step = 0; step <= ORC_EPS_STEPS; ++step) {
                        if (step > 0) {
                            if (!(nu > 0.0 && Q > nu && Qp < 0.0)) break;
                            y += (1.0 - Q / nu) * Q / Qp;
                            if (y < 0.0) y = 0.0;
                        }
                        def = source_normals_solve(Ab, hb, Vb, wb, ni, y, N, b);
                        source_q(Ab, hb, Vb, wb, ni, y, b, &Q, &Qp);
                        if (step == 0) D = nu > 0.0 ? (Q - nu) / sqrt(2.0 * nu) : 0.0;
                    }
                } else {
                    def = source_normals_solve(Ab, hb, Vb, wb, ni, 0.0, N, b);
                }
            }
            if (st->src_eps2) st->src_eps2[i] = y;
            if (st->src_D) st->src_D[i] = D;
            if (var_out) {
                /* diagonal of the inverse: C2 and C3 on the unit vectors
                 * (Appendix C.2) */
                for (int kk = 0; kk < 5; ++kk) {
                    double e[5] = {0, 0, 0, 0, 0};
                    e[kk] = 1.0;
                    orc_chol_c2(N, 5, e);
                    orc_chol_c3(N, 5, e);
                    var_out[5 * i + kk] = def > 0 ? 0.0 : e[kk];
                }
            }
            double Q = 0.0;
            for (int64_t k = 0; k < ni; ++k) {
                double Rk = hb[k];
                for (int c = 0; c < 5; ++c) Rk -= Ab[5 * k + c] * b[c];
                Q += Rk * (wb[k] / (Vb[k] + y)) * Rk;
            }
            double* s = st->s + 5 * i;
            double cosd = cos(s[1]);
            s[0] += b[0] / cosd;
            s[1] += b[1];
            s[2] += b[2];
            s[3] += b[3];
            s[4] += b[4];
            if (d_out) for (int c = 0; c < 5; ++c) d_out[5 * i + c] = b[c];
            if (Q_out) Q_out[i] = Q;
            if (defect_out) defect_out[i] = def;
        }
        free(Ab); free(hb); free(Vb); free(wb); free(xb);
    }
    free(off);
    free(idx);
}

/* ========================================================================
 * Sect. 5.2: attitude update.  Normal equations eq:normAmod (with the
 * regularisation eq:Dl, eq:JfuncMod, eq:dDldan), the partials eq:dfadq times
 * B_n, and the overlapping segmentation of Sect. 5.2.2: segment K uses the
 * data in [tau_{x_K - L}, tau_{x_{K+1} + L}) and supplies the updates for
 * x_K - 1 <= n <= x_{K+1} - 2 (M = 4).  Each segment is solved with
 * Algorithms C1-C3 on the band envelope.
 * ====================================================================== */
int64_t orc_num_segments(const orc_world_t* w) {
    int64_t K = w->n_knots - 2 * M_ORDER + 1;    /* number of knot intervals N - 3 */
    return (K + w->seg_len - 1) / w->seg_len;
}

typedef struct {
    int64_t lo, hi;              /* knot indices bounding the data interval */
    int64_t n_lo, n_hi;          /* coefficient range of the segment system */
    int64_t keep_lo, keep_hi;    /* coefficient range whose updates are kept */
    int last;
} seg_t;

static void segment_bounds(const orc_world_t* w, int64_t K, seg_t* s) {
    int64_t N = w->n_knots - M_ORDER;
    int64_t nseg = orc_num_segments(w);
    int64_t x0 = (M_ORDER - 1) + K * (int64_t)w->seg_len;          /* x_K */
    int64_t x1 = K + 1 < nseg ? x0 + w->seg_len : N;                /* x_{K+1} */
    s->lo = K == 0 ? M_ORDER - 1 : x0 - w->seg_overlap;
    s->hi = K + 1 < nseg ? x1 + w->seg_overlap : N;
    if (s->lo < M_ORDER - 1) s->lo = M_ORDER - 1;
    if (s->hi > N) s->hi = N;
    s->n_lo = s->lo - (M_ORDER - 1);
    s->n_hi = s->hi - 1;
    s->keep_lo = K == 0 ? 0 : x0 - M_ORDER / 2 + 1;
    s->keep_hi = K + 1 < nseg ? x1 - M_ORDER / 2 : N - 1;
    s->last = K + 1 == nseg;
}

typedef struct { double t; int64_t l; } tl_t;
static int cmp_tl(const void* a, const void* b) {
    const tl_t* x = (const tl_t*)a;
    const tl_t* y = (const tl_t*)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return x->l < y->l ? -1 : (x->l > y->l ? 1 : 0);
}

static tl_t* time_order(const orc_obs_t* obs) {
    tl_t* o = (tl_t*)malloc(sizeof(tl_t) * (size_t)(obs->n > 0 ? obs->n : 1));
    for (int64_t l = 0; l < obs->n; ++l) { o[l].t = obs->t[l]; o[l].l = l; }
    qsort(o, (size_t)obs->n, sizeof(tl_t), cmp_tl);
    return o;
}

static int64_t first_at_or_after(const tl_t* o, int64_t n, double t) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (o[mid].t < t) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t solve_segment(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                             const tl_t* order, const seg_t* sg, double* d) {
    const int hb = 4 * M_ORDER - 1;
    int64_t ncoef = sg->n_hi - sg->n_lo + 1;
    int n = (int)(4 * ncoef);
    double* UB = (double*)calloc((size_t)n * (hb + 1), sizeof(double));
    double* y = (double*)calloc((size_t)n, sizeof(double));
    const double lam2 = w->lambda_reg * w->lambda_reg;
    double t_lo = w->knots[sg->lo], t_hi = w->knots[sg->hi];
    int64_t first = first_at_or_after(order, obs->n, t_lo);
    for (int64_t k = first; k < obs->n; ++k) {
        double t = order[k].t;
        if (sg->last ? (t > t_hi) : (t >= t_hi)) break;
        int64_t l = order[k].l;
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double g[4];
        attitude_partial(&o, g);
        double W = weight(w, obs, st, l, &o);
        for (int kn = 0; kn < M_ORDER; ++kn) {
            int64_t nb = o.ell - (M_ORDER - 1) + kn - sg->n_lo;
            for (int km = 0; km < M_ORDER; ++km) {
                int64_t mb = o.ell - (M_ORDER - 1) + km - sg->n_lo;
                if (mb < nb) continue;
                for (int r = 0; r < 4; ++r) {
                    for (int c = 0; c < 4; ++c) {
                        int64_t i = 4 * nb + r, j = 4 * mb + c;
                        if (j < i) continue;
                        double dRR = o.B[kn] * g[r] * o.B[km] * g[c];
                        double dDD = (-2.0 * o.qraw[r] * o.B[kn]) * (-2.0 * o.qraw[c] * o.B[km]);
                        UB[i * (hb + 1) + (j - i)] += (dRR + lam2 * dDD) * W;
                    }
                }
            }
            for (int r = 0; r < 4; ++r) {
                double dR = o.B[kn] * g[r];
                double dD = -2.0 * o.qraw[r] * o.B[kn];
                y[4 * nb + r] -= (dR * o.R + lam2 * dD * o.D) * W;
            }
        }
    }
    int64_t def = orc_band_c1(UB, n, hb);
    orc_band_c2(UB, n, hb, y);
    orc_band_c3(UB, n, hb, y);
    for (int64_t nn = sg->keep_lo; nn <= sg->keep_hi; ++nn)
        for (int c = 0; c < 4; ++c) d[4 * nn + c] = y[4 * (nn - sg->n_lo) + c];
    free(UB);
    free(y);
    return def;
}

static int64_t attitude_solve(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* d) {
    tl_t* order = time_order(obs);
    int64_t nseg = orc_num_segments(w);
    int64_t def = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : def)
    for (int64_t K = 0; K < nseg; ++K) {
        seg_t sg;
        segment_bounds(w, K, &sg);
        def += solve_segment(w, obs, st, order, &sg, d);
    }
    free(order);
    return def;
}

int64_t orc_attitude_segment(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                             int64_t K, double* d, int64_t* keep_lo, int64_t* keep_hi) {
    tl_t* order = time_order(obs);
    seg_t sg;
    segment_bounds(w, K, &sg);
    int64_t def = solve_segment(w, obs, st, order, &sg, d);
    if (keep_lo) *keep_lo = sg.keep_lo;
    if (keep_hi) *keep_hi = sg.keep_hi;
    free(order);
    return def;
}

int64_t orc_attitude_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* d_out) {
    double* d = (double*)calloc((size_t)(4 * st->n_att), sizeof(double));
    int64_t def = attitude_solve(w, obs, st, d);
    for (int64_t k = 0; k < 4 * st->n_att; ++k) st->a[k] += d[k];
    if (d_out) memcpy(d_out, d, sizeof(double) * (size_t)(4 * st->n_att));
    free(d);
    return def;
}

/* ========================================================================
 * Sect. 5.3: calibration update.  One effect with Phi = 1 per cell
 * (eq:generic2, eq:pdC), so N_cc is diagonal (eq:normC); each 1x1 system
 * goes through C1-C3; then the constraint projection eq:calCon with one
 * constraint per day, c_P + c_F = 0 (eq:cc1 for this model).
 * ====================================================================== */
/* Number of calibration unknowns: one per cell, or with the geometric
 * model three per cell and CCD, twice that with the AC calibration. */
static int64_t cal_size(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st) {
    if (w->geo_ccds <= 0) return st->n_cells;
    return small_base(w, obs, st) + small_intervals(w, st) * w->geo_ccds * GEO_COLS;
}

/* Solves A x = b (n x n, row-major, overwritten) by Gaussian elimination
 * with partial pivoting (the largest remaining entry of the column; the
 * first of equal ones), then back substitution.  Entries that are exactly
 * zero take no part in a row operation (they would leave it unchanged). */
static void solve_gauss_pp(double* A, double* b, int64_t n, double* x) {
    int64_t* cols = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (p != k) {
            for (int64_t j = 0; j < n; ++j) {
                const double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
            const double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        int64_t nz = 0;
        for (int64_t j = k + 1; j < n; ++j)
            if (A[k * n + j] != 0.0) cols[nz++] = j;
        for (int64_t i = k + 1; i < n; ++i) {
            if (A[i * n + k] == 0.0) continue;
            const double f = A[i * n + k] / A[k * n + k];
            for (int64_t t = 0; t < nz; ++t) A[i * n + cols[t]] -= f * A[k * n + cols[t]];
            b[i] -= f * b[k];
            A[i * n + k] = 0.0;
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    free(cols);
}

/* The C update of one CCD n and long interval k with the small-scale term:
 * the unknowns are the small-scale coefficients of the 1966 columns
 * (dR/d delta-eta = 1) and the large-scale AL coefficients of the interval's
 * cells of that CCD (dR/dc_r = L*_r(x)), which share records and, through
 * the constant (exactly) and the two other polynomials (up to the rounding
 * of mu to m), an almost degenerate direction.  eq:normC over the interval's
 * AL records of that CCD, with the A/C weights, is solved subject to the
 * three constraints of eq:cc2 (sum over m of the update times L*_r at the
 * column centre, r = 0, 1, 2) by the Lagrange (KKT) system
 *     [N  C] [d ]   [b]
 *     [C' 0] [nu] = [0],
 * the constrained least-squares update.  An unknown without records (a
 * column or cell that no record of the block reaches) is held at zero.
 * Unknown order: the columns, the cells' coefficients, the multipliers.
 * R and W: each record's residual and weight, from the caller. */
static void small_block_solve(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, int64_t k,
                              int32_t n, const double* R, const double* W, double* d) {
    const int64_t D = w->geo_small_days;
    const int64_t c0 = 2 * k * D, c1 = (2 * (k + 1) * D < st->n_cells) ? 2 * (k + 1) * D : st->n_cells;
    const int64_t nc = c1 - c0, ne = 3 * nc, nu = GEO_COLS + ne, nk = nu + 3;
    const int64_t q0 = small_base(w, obs, st) + (k * w->geo_ccds + n) * GEO_COLS;
    int64_t n_rec = 0;
    for (int64_t l = 0; l < obs->n; ++l)
        if (obs->cell[l] >= c0 && obs->cell[l] < c1 && obs->ccd[l] == n) ++n_rec;
    if (n_rec == 0) {                                 /* every unknown held at zero */
        for (int64_t m = 0; m < GEO_COLS; ++m) d[q0 + m] = 0.0;
        for (int64_t c = c0; c < c1; ++c)
            for (int r = 0; r < 3; ++r) d[3 * (c * w->geo_ccds + n) + r] = 0.0;
        return;
    }
    double* A = (double*)calloc((size_t)(nk * nk), sizeof(double));
    double* b = (double*)calloc((size_t)nk, sizeof(double));
    double* x = (double*)calloc((size_t)nk, sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)nu, sizeof(int64_t));
    for (int64_t l = 0; l < obs->n; ++l) {
        if (obs->cell[l] < c0 || obs->cell[l] >= c1 || obs->ccd[l] != n) continue;
        const double xl = geo_x(obs, l);
        int64_t idx[4];
        double p[4];
        idx[0] = geo_column(obs, l);
        p[0] = 1.0;
        for (int r = 0; r < 3; ++r) {
            idx[1 + r] = GEO_COLS + 3 * (obs->cell[l] - c0) + r;
            p[1 + r] = shifted_legendre(r, xl);
        }
        for (int a = 0; a < 4; ++a) {
            for (int e = 0; e < 4; ++e) A[idx[a] * nk + idx[e]] += p[a] * W[l] * p[e];
            b[idx[a]] -= p[a] * R[l] * W[l];
            cnt[idx[a]] += 1;
        }
    }
    for (int64_t m = 0; m < GEO_COLS; ++m) {
        if (cnt[m] == 0) continue;
        const double xm = ((double)(m + 14) - 13.5) / 1966.0;
        for (int r = 0; r < 3; ++r) {
            A[(nu + r) * nk + m] = shifted_legendre(r, xm);
            A[m * nk + nu + r] = shifted_legendre(r, xm);
        }
    }
    for (int64_t i = 0; i < nu; ++i)
        if (cnt[i] == 0) A[i * nk + i] = 1.0;        /* held at zero: b_i = 0 */
    solve_gauss_pp(A, b, nk, x);
    for (int64_t m = 0; m < GEO_COLS; ++m) d[q0 + m] = x[m];
    for (int64_t c = c0; c < c1; ++c)
        for (int r = 0; r < 3; ++r) d[3 * (c * w->geo_ccds + n) + r] = x[GEO_COLS + 3 * (c - c0) + r];
    free(A);
    free(b);
    free(x);
    free(cnt);
}

/* Geometric calibration (Sect. 5.3 with eq:etazeta): eq:normC for each
 * group of three coefficients (cell and CCD, along or across scan), whose
 * records share no coefficient with another group, W from the A/C weights;
 * the 3x3 systems by C1-C3; then eq:calCon with the constraints: eq:cc1
 * (for each day, the AL constant terms of its two cells and all CCDs sum to
 * zero) and, with the AC calibration, eq:cc3 (for each AC cell, i.e. field
 * of view and long interval, the AC constant terms of its CCDs sum to zero); the
 * constraint columns do not overlap, so each projection subtracts the mean
 * constant term of its set.  With the small-scale AL term the AL groups of a
 * CCD and long interval share records with its small-scale coefficients, and
 * each such block is solved together under eq:cc2 (small_block_solve)
 * before the eq:cc1 projection. */
static void calibration_solve_geo(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* d) {
    const int64_t ng_al = st->n_cells * w->geo_ccds;
    const int64_t ng = small_base(w, obs, st) / 3;
    const int64_t K = small_intervals(w, st);
    double* Rl = K > 0 ? (double*)calloc((size_t)(obs->n > 0 ? obs->n : 1), sizeof(double)) : NULL;
    double* Wl = K > 0 ? (double*)calloc((size_t)(obs->n > 0 ? obs->n : 1), sizeof(double)) : NULL;
    double* N = (double*)calloc((size_t)(9 * ng), sizeof(double));
    double* b = (double*)calloc((size_t)(3 * ng), sizeof(double));
    for (int64_t l = 0; l < obs->n; ++l) {
        const int64_t g3 = geo_index(w, obs, st, l);
        if (g3 < 0) continue;                        /* across scan without the AC calibration */
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double W = weight(w, obs, st, l, &o);
        if (K > 0) {
            Rl[l] = o.R;
            Wl[l] = W;
        }
        const int64_t g = g3 / 3;
        const double x = geo_x(obs, l);
        double L[3];
        for (int r = 0; r < 3; ++r) L[r] = shifted_legendre(r, x);     /* dR/dc_r (eq:pdC) */
        for (int r = 0; r < 3; ++r) {
            for (int s = 0; s < 3; ++s) N[9 * g + 3 * r + s] += L[r] * W * L[s];
            b[3 * g + r] -= L[r] * o.R * W;
        }
    }
    for (int64_t g = (K > 0 ? ng_al : 0); g < ng; ++g) {     /* AL groups: below, with the small scale */
        double U[9], x[3];
        memcpy(U, N + 9 * g, sizeof U);
        memcpy(x, b + 3 * g, sizeof x);
        orc_chol_c1(U, 3);
        orc_chol_c2(U, 3, x);
        orc_chol_c3(U, 3, x);
        memcpy(d + 3 * g, x, sizeof x);
    }
    /* with the small-scale term, the AL groups and the small-scale
     * coefficients by CCD and long interval (eq:cc2 inside) */
    for (int64_t k = 0; k < K; ++k)
        for (int32_t n = 0; n < w->geo_ccds; ++n) small_block_solve(w, obs, st, k, n, Rl, Wl, d);
    free(Rl);
    free(Wl);
    /* eq:calCon for eq:cc1: C has one column per day, with ones at the
     * constant terms of the day's 2 geo_ccds groups; C'C = 2 geo_ccds I */
    const int64_t per_day = 2 * w->geo_ccds;
    for (int64_t j = 0; (j + 1) * per_day <= ng_al; ++j) {
        double ctd = 0.0;
        for (int64_t k = 0; k < per_day; ++k) ctd += d[3 * (j * per_day + k)];
        const double z = ctd / (double)per_day;
        for (int64_t k = 0; k < per_day; ++k) d[3 * (j * per_day + k)] -= z;
    }
    /* eq:calCon for eq:cc3: one column per AC cell, with ones at the
     * constant terms of the cell's geo_ccds AC groups; C'C = geo_ccds I */
    for (int64_t c = 0; ng > ng_al && c < w->geo_ac_cells; ++c) {
        const int64_t g0 = ng_al + c * w->geo_ccds;
        double ctd = 0.0;
        for (int64_t k = 0; k < w->geo_ccds; ++k) ctd += d[3 * (g0 + k)];
        const double z = ctd / (double)w->geo_ccds;
        for (int64_t k = 0; k < w->geo_ccds; ++k) d[3 * (g0 + k)] -= z;
    }
    free(N);
    free(b);
}

/* The calibration update d (cal_size entries) applied to the state. */
static void apply_calibration(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, const double* d) {
    if (w->geo_ccds > 0) {
        for (int64_t k = 0; k < cal_size(w, obs, st); ++k) st->geo[k] += d[k];
    } else {
        for (int64_t c = 0; c < st->n_cells; ++c) st->c[c] += d[c];
    }
}

static void calibration_solve(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* d) {
    if (w->geo_ccds > 0) {
        calibration_solve_geo(w, obs, st, d);
        return;
    }
    double* Nc = (double*)calloc((size_t)st->n_cells, sizeof(double));
    double* bc = (double*)calloc((size_t)st->n_cells, sizeof(double));
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double W = weight(w, obs, st, l, &o);
        int32_t c = obs->cell[l];
        if (c < 0) continue;                        /* across scan: no calibration term */
        Nc[c] += 1.0 * W * 1.0;
        bc[c] -= 1.0 * o.R * W;
    }
    for (int64_t c = 0; c < st->n_cells; ++c) {
        double U = Nc[c], x = bc[c];
        orc_chol_c1(&U, 1);
        orc_chol_c2(&U, 1, &x);
        orc_chol_c3(&U, 1, &x);
        d[c] = x;
    }
    /* C = one column per day with ones at (2j, 2j+1); columns orthogonal,
     * C'C = 2 I */
    for (int64_t j = 0; 2 * j + 1 < st->n_cells; ++j) {
        double ctd = d[2 * j] + d[2 * j + 1];
        double z = ctd / 2.0;
        d[2 * j] -= z;
        d[2 * j + 1] -= z;
    }
    free(Nc);
    free(bc);
}

void orc_calibration_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* d_out) {
    const int64_t nc = cal_size(w, obs, st);
    double* d = (double*)calloc((size_t)nc, sizeof(double));
    calibration_solve(w, obs, st, d);
    apply_calibration(w, obs, st, d);
    if (d_out) memcpy(d_out, d, sizeof(double) * (size_t)nc);
    free(d);
}

/* Sect. 4.6 (order of the blocks): S with a^k, c^k; then A and C both with
 * s^{k+1}, a^k, c^k (the S[AC] variant of eq:precondS(CAG) without G).
 * Robust: the excess attitude noise is re-estimated from the residuals after
 * the source update and used by the A and C weights (Sect. 5.2.5). */
/* Sect. 5.4, eq:normG for g = (g0, g1): g0 of eq:gammaPPN and the
 * pseudo-parameter g1, a global shift of all parallaxes (its design entry is
 * each observation's parallax entry), solved with g0 but never applied; the
 * 2x2 system sum A_g W A_g' d = sum A_g W R (A_g = -dR/dg, W the A/C
 * weights) by C1-C3.  Returns the update of g0. */
static double global_solve(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st) {
    double N[4] = {0.0, 0.0, 0.0, 0.0}, b[2] = {0.0, 0.0};
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        const double W = weight(w, obs, st, l, &o);
        double As[5];
        source_partials(&o, As);
        const double Ag[2] = {global_partial(&o), As[2]};
        for (int r = 0; r < 2; ++r) {
            for (int c = 0; c < 2; ++c) N[2 * r + c] += Ag[r] * W * Ag[c];
            b[r] += Ag[r] * W * o.R;
        }
    }
    orc_chol_c1(N, 2);
    orc_chol_c2(N, 2, b);
    orc_chol_c3(N, 2, b);
    return b[0];
}

double orc_global_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st) {
    const double d = global_solve(w, obs, st);
    st->g0 += d;
    return d;
}

void orc_iterate_sac(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* var) {
    orc_source_update(w, obs, st, NULL, NULL, NULL, var);
    orc_excess_attitude_noise(w, obs, st);
    double* da = (double*)calloc((size_t)(4 * st->n_att), sizeof(double));
    double* dc = (double*)calloc((size_t)cal_size(w, obs, st), sizeof(double));
    attitude_solve(w, obs, st, da);
    calibration_solve(w, obs, st, dc);
    /* S[ACG]: the global update from the same residuals and weights */
    const double dg = w->ppn ? global_solve(w, obs, st) : 0.0;
    for (int64_t k = 0; k < 4 * st->n_att; ++k) st->a[k] += da[k];
    apply_calibration(w, obs, st, dc);
    st->g0 += dg;
    free(da);
    free(dc);
}

/* ========================================================================
 * Right-hand sides of the three normal-equation blocks at the current state
 * (eq:normS, eq:normAmod with the regularisation of eq:JfuncMod, eq:normC),
 * summed over all observations: the vector b - N x of the linearised
 * problem that the conjugate-gradient scheme of Sect. 4.7 works with.
 * rs: [n_src][5] sum A' W R with A the design row -dR/ds; ra: [n_att][4]
 * -sum (dR/da R + lambda^2 dD/da D) W; rc: [n_cells] -sum R W.  Not robust:
 * W = 1 / sigma^2 in all three, as in the block solves.
 * ====================================================================== */
void orc_normal_rhs(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* rs, double* ra,
                    double* rc) {
    const double lam2 = w->lambda_reg * w->lambda_reg;
    memset(rs, 0, sizeof(double) * (size_t)(5 * st->n_src));
    memset(ra, 0, sizeof(double) * (size_t)(4 * st->n_att));
    memset(rc, 0, sizeof(double) * (size_t)st->n_cells);
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double W = weight(w, obs, st, l, &o);
        double A[5], g[4];
        source_partials(&o, A);
        attitude_partial(&o, g);
        double* bs = rs + 5 * (int64_t)obs->src[l];
        for (int k = 0; k < 5; ++k) bs[k] += A[k] * W * o.R;
        for (int kn = 0; kn < M_ORDER; ++kn) {
            double* bn = ra + 4 * (o.ell - (M_ORDER - 1) + kn);
            for (int r = 0; r < 4; ++r) {
                double dR = o.B[kn] * g[r];
                double dD = -2.0 * o.qraw[r] * o.B[kn];
                bn[r] -= (dR * o.R + lam2 * dD * o.D) * W;
            }
        }
        if (!o.ac) rc[obs->cell[l]] -= 1.0 * o.R * W;
    }
}

/* The quadratic form v' N v of the normal matrix of the three blocks at the
 * current state: sum over the observations of W (J_R v)^2 + lambda^2 W
 * (J_D v)^2, with J_R v = -A . v_src + sum_n B_n dR/dq . v_att(n) + v_cal
 * (A the design row -dR/ds) and J_D v = sum_n -2 q~ B_n . v_att(n).
 * v: [n_src][5], then [n_att][4], then [n_cells]. */
double orc_normal_quadratic(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, const double* v) {
    const double lam2 = w->lambda_reg * w->lambda_reg;
    const double* va = v + 5 * st->n_src;
    const double* vc = va + 4 * st->n_att;
    double sum = 0.0;
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double W = weight(w, obs, st, l, &o);
        double A[5], g[4];
        source_partials(&o, A);
        attitude_partial(&o, g);
        const double* vs = v + 5 * (int64_t)obs->src[l];
        double jr = o.ac ? 0.0 : vc[obs->cell[l]], jd = 0.0;
        for (int k = 0; k < 5; ++k) jr -= A[k] * vs[k];
        for (int kn = 0; kn < M_ORDER; ++kn) {
            const double* vn = va + 4 * (o.ell - (M_ORDER - 1) + kn);
            for (int r = 0; r < 4; ++r) {
                jr += o.B[kn] * g[r] * vn[r];
                jd += -2.0 * o.qraw[r] * o.B[kn] * vn[r];
            }
        }
        sum += W * jr * jr + lam2 * W * jd * jd;
    }
    return sum;
}

/* Frozen weights (the switch of the hybrid scheme, Sect. 4.7): each
 * observation's A/C weight W_l at the current state, as sigma_eff =
 * 1 / sqrt(W_l) (W_l = 0, or sigma_eff beyond it: the largest finite
 * float), in input order.  A problem with these in place of sigma and no
 * robust weighting is the fixed weighted least-squares problem CG then
 * solves. */
void orc_frozen_sigma(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* sig) {
    for (int64_t l = 0; l < obs->n; ++l) {
        orc_fwd_t o;
        forward_one(w, obs, st, l, &o);
        double W = weight(w, obs, st, l, &o);
        double se = W > 0.0 ? 1.0 / sqrt(W) : (double)FLT_MAX;
        if (!(se <= (double)FLT_MAX)) se = (double)FLT_MAX;
        sig[l] = se;
    }
}

/* ========================================================================
 * Sect. 6.1: frame rotator.
 * Fit: least squares of eq:cond-mu3 over all sources taken as S_PM,
 * comparison epoch t = t_ep, with the position differences of eq:fr-Delta1
 * (t_P = t_ep), each equation weighted by the inverse variance of its
 * parameter (unit weights without variances); normal equations solved by
 * C1-C3.
 * Apply: the five rigorous steps of Sect. 6.1.2 for every source and
 * eq:fr-q4 with eq:RF4 for every attitude coefficient.
 * ====================================================================== */
void orc_frame_fit(const orc_world_t* w, const orc_state_t* st, const double* s_ref, const double* var,
                   double eps_omega[6]) {
    double N[36] = {0}, b[6] = {0};
    double tau = (w->t_ep - w->t_fr) / w->year_s;
    for (int64_t i = 0; i < st->n_src; ++i) {
        const double* s = st->s + 5 * i;
        const double* h = s_ref + 5 * i;
        double pt[3], qt[3], rt[3], ph[3], qh[3], rh[3];
        orc_normal_triad(s[0], s[1], pt, qt, rt);
        orc_normal_triad(h[0], h[1], ph, qh, rh);
        double dr[3] = {rt[0] - rh[0], rt[1] - rh[1], rt[2] - rh[2]};
        double rows[4][6], rhs[4];
        for (int k = 0; k < 3; ++k) {
            rows[0][k] = 0.0;        rows[0][3 + k] = qt[k];
            rows[1][k] = 0.0;        rows[1][3 + k] = -pt[k];
            rows[2][k] = qt[k];      rows[2][3 + k] = tau * qt[k];
            rows[3][k] = -pt[k];     rows[3][3 + k] = -tau * pt[k];
        }
        rhs[0] = s[3] - h[3];
        rhs[1] = s[4] - h[4];
        rhs[2] = dot3(pt, dr);
        rhs[3] = dot3(qt, dr);
        /* weights: inverse variances of mu_a*, mu_d, alpha*, delta */
        const int vidx[4] = {3, 4, 0, 1};
        double wt[4] = {1.0, 1.0, 1.0, 1.0};
        if (var) {
            for (int e = 0; e < 4; ++e) {
                double v = var[5 * i + vidx[e]];
                wt[e] = (v > 0.0 && isfinite(v)) ? 1.0 / v : 0.0;
            }
        }
        for (int e = 0; e < 4; ++e) {
            for (int r = 0; r < 6; ++r) {
                for (int c = 0; c < 6; ++c) N[6 * r + c] += rows[e][r] * wt[e] * rows[e][c];
                b[r] += rows[e][r] * wt[e] * rhs[e];
            }
        }
    }
    orc_chol_c1(N, 6);
    orc_chol_c2(N, 6, b);
    orc_chol_c3(N, 6, b);
    memcpy(eps_omega, b, sizeof b);
}

/* f(t) = Q[(t - t_fr) omega] Q(eps)  (eq:fr1) */
static void frame_quat(const orc_world_t* w, const double eo[6], double t, double f[4]) {
    double dt = (t - w->t_fr) / w->year_s;
    double wv[3] = {dt * eo[3], dt * eo[4], dt * eo[5]};
    double qw[4], qe[4];
    orc_qrot(wv, qw);
    orc_qrot(eo, qe);
    orc_qmul(qw, qe, f);
}

void orc_frame_apply(const orc_world_t* w, orc_state_t* st, const double eo[6]) {
    double f[4], fi[4];
    frame_quat(w, eo, w->t_ep, f);                                  /* step 1 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < st->n_src; ++i) {
        double* s = st->s + 5 * i;
        double pt[3], qt[3], rt[3];
        orc_normal_triad(s[0], s[1], pt, qt, rt);                   /* step 2 */
        double rC[3], mut[3], muC[3];
        orc_frame_rotate(f, rt, rC);                                /* step 3, eq:fr-r */
        double wxr[3] = {eo[4] * rt[2] - eo[5] * rt[1], eo[5] * rt[0] - eo[3] * rt[2], eo[3] * rt[1] - eo[4] * rt[0]};
        for (int k = 0; k < 3; ++k) mut[k] = pt[k] * s[3] + qt[k] * s[4] - wxr[k];   /* eq:mu-agis */
        orc_frame_rotate(f, mut, muC);                              /* eq:fr-mu */
        double alpha = atan2(rC[1], rC[0]);                         /* step 4, eq:fr-ad */
        double delta = atan2(rC[2], sqrt(rC[0] * rC[0] + rC[1] * rC[1]));
        double p[3], q[3], r[3];
        orc_normal_triad(alpha, delta, p, q, r);
        s[0] = alpha;
        s[1] = delta;
        s[3] = dot3(p, muC);                                        /* step 5, eq:fr-mu-icrs */
        s[4] = dot3(q, muC);
    }
    (void)fi;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < st->n_att; ++n) {
        double tbar = 0.5 * (w->knots[n] + w->knots[n + M_ORDER]);  /* eq:RF4 */
        double fn[4], fni[4], r[4];
        frame_quat(w, eo, tbar, fn);
        orc_qinv(fn, fni);
        orc_qmul(fni, st->a + 4 * n, r);                            /* eq:fr-q4 */
        memcpy(st->a + 4 * n, r, sizeof r);
    }
}
