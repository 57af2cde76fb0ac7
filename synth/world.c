/*
 * Synthetic observing world: a simplified Gaia-like nominal scanning law and
 * the search for field-of-view transits of fixed star directions.
 *
 * This file is INPUT GENERATION ONLY.  It decides *when* a star is observed
 * and what the nominal satellite orientation is; it never evaluates the
 * astrometric solution's observation model (no proper direction, no
 * aberration, no B-spline attitude, no residuals).  Both the HIP solver and
 * the CPU oracle consume its output as plain arrays.
 *
 * Geometry (all angles in radians, time t in seconds from the reference epoch):
 *   - Gaia's heliocentric ecliptic longitude  L(t) = L0 + Lrate * t
 *     (circular orbit); the Sun as seen from Gaia is s = -(cos L, sin L, 0).
 *   - The spin axis z makes the solar aspect angle xi with s and precesses
 *     around it: z = cos(xi) s + sin(xi) (cos(nu) eN + sin(nu) (s x eN)),
 *     nu = nu0 + 2 pi t / Pprec, eN = ecliptic pole.
 *   - The scan phase Omega = Omega0 + wspin * t measures the SRS x-axis from
 *     e1 = <eN x z> toward e2 = z x e1; y = z x x.
 *   - Preceding / following viewing directions are at in-plane angle
 *     +Gamma/2 / -Gamma/2 from x (the SRS triad definition of the paper,
 *     Sect. 3.1).
 *   - Ecliptic -> equatorial by a rotation of eps_obl about the X axis.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double L0, Lrate;          /* Gaia orbital longitude [rad], rate [rad/s] */
    double xi;                 /* solar aspect angle [rad] */
    double nu0, Pprec;         /* precession phase [rad], period [s] */
    double Omega0, wspin;      /* scan phase [rad], spin rate [rad/s] */
    double gamma;              /* basic angle [rad] */
    double eps_obl;            /* obliquity of the ecliptic [rad] */
    double zeta_max;           /* across-scan half width [rad] */
} syn_law_t;

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void unit3(double a[3]) {
    double n = sqrt(dot3(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}

/* Spin axis z and in-plane reference axes e1, e2, all in ecliptic coordinates. */
static void spin_frame(const syn_law_t* w, double t, double z[3], double e1[3], double e2[3]) {
    double L = w->L0 + w->Lrate * t;
    double s[3] = {-cos(L), -sin(L), 0.0};
    double eN[3] = {0.0, 0.0, 1.0};
    double sxn[3];
    cross3(s, eN, sxn);
    double nu = w->nu0 + 2.0 * M_PI * t / w->Pprec;
    double cx = cos(w->xi), sx = sin(w->xi), cn = cos(nu), sn = sin(nu);
    for (int k = 0; k < 3; ++k) z[k] = cx * s[k] + sx * (cn * eN[k] + sn * sxn[k]);
    unit3(z);
    cross3(eN, z, e1);
    unit3(e1);
    cross3(z, e1, e2);
}

static void ecl_to_equ(double eps, const double v[3], double o[3]) {
    double c = cos(eps), s = sin(eps);
    o[0] = v[0];
    o[1] = c * v[1] - s * v[2];
    o[2] = s * v[1] + c * v[2];
}
static void equ_to_ecl(double eps, const double v[3], double o[3]) {
    double c = cos(eps), s = sin(eps);
    o[0] = v[0];
    o[1] = c * v[1] + s * v[2];
    o[2] = -s * v[1] + c * v[2];
}

static double wrap_2pi(double a) {
    a = fmod(a, 2.0 * M_PI);
    if (a < 0) a += 2.0 * M_PI;
    return a;
}
static double wrap_pi(double a) {
    a = wrap_2pi(a + M_PI) - M_PI;
    return a;
}

/* Nominal SRS axes x, y, z in equatorial coordinates at time t. */
void syn_nominal_axes(const syn_law_t* w, double t, double x[3], double y[3], double z[3]) {
    double ze[3], e1[3], e2[3], xe[3], ye[3];
    spin_frame(w, t, ze, e1, e2);
    double Om = w->Omega0 + w->wspin * t;
    double c = cos(Om), s = sin(Om);
    for (int k = 0; k < 3; ++k) xe[k] = c * e1[k] + s * e2[k];
    cross3(ze, xe, ye);
    ecl_to_equ(w->eps_obl, xe, x);
    ecl_to_equ(w->eps_obl, ye, y);
    ecl_to_equ(w->eps_obl, ze, z);
}

/*
 * Unit quaternion {qx,qy,qz,qw} of the nominal orientation, in the paper's
 * convention: its frame rotation takes equatorial coordinates to SRS
 * coordinates, and the rows of the direction-cosine matrix are x', y', z'.
 * Conversion by Shepperd's method (largest-pivot branch); qw >= 0 is NOT
 * enforced here, the caller makes the sequence sign-continuous.
 */
void syn_nominal_quat(const syn_law_t* w, int64_t n, const double* t, double* q) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[3], y[3], z[3];
        syn_nominal_axes(w, t[i], x, y, z);
        /* A = [x'; y'; z'] (rows); quaternion such that A = quat2mat(q). */
        double A[3][3] = {{x[0], x[1], x[2]}, {y[0], y[1], y[2]}, {z[0], z[1], z[2]}};
        double tr = A[0][0] + A[1][1] + A[2][2];
        double qx, qy, qz, qw;
        if (tr >= A[0][0] && tr >= A[1][1] && tr >= A[2][2]) {
            double r = sqrt(1.0 + tr);
            qw = 0.5 * r;
            double f = 0.5 / r;
            qx = (A[1][2] - A[2][1]) * f;
            qy = (A[2][0] - A[0][2]) * f;
            qz = (A[0][1] - A[1][0]) * f;
        } else if (A[0][0] >= A[1][1] && A[0][0] >= A[2][2]) {
            double r = sqrt(1.0 + A[0][0] - A[1][1] - A[2][2]);
            qx = 0.5 * r;
            double f = 0.5 / r;
            qw = (A[1][2] - A[2][1]) * f;
            qy = (A[0][1] + A[1][0]) * f;
            qz = (A[0][2] + A[2][0]) * f;
        } else if (A[1][1] >= A[2][2]) {
            double r = sqrt(1.0 - A[0][0] + A[1][1] - A[2][2]);
            qy = 0.5 * r;
            double f = 0.5 / r;
            qw = (A[2][0] - A[0][2]) * f;
            qx = (A[0][1] + A[1][0]) * f;
            qz = (A[1][2] + A[2][1]) * f;
        } else {
            double r = sqrt(1.0 - A[0][0] - A[1][1] + A[2][2]);
            qz = 0.5 * r;
            double f = 0.5 / r;
            qw = (A[0][1] - A[1][0]) * f;
            qx = (A[0][2] + A[2][0]) * f;
            qy = (A[1][2] + A[2][1]) * f;
        }
        q[4 * i + 0] = qx; q[4 * i + 1] = qy; q[4 * i + 2] = qz; q[4 * i + 3] = qw;
    }
}

/*
 * Transit search for one star (equatorial unit vector r) over [t0, t1).
 * For every spin revolution and each field of view the time at which the
 * star's in-plane angle equals the viewing direction (+-Gamma/2) is found by
 * a few fixed-point refinements; the transit is kept when the star's
 * across-scan angle is within zeta_max and the time lies in the revolution
 * that proposed it (so no transit is reported twice).
 * Writes at most cap transits (times and fov +1 = preceding, -1 = following)
 * and returns the number found.
 */
typedef struct {
    int64_t nrev;
    double* z;                 /* [nrev][3] spin axis at mid-revolution */
} rev_table_t;

static void rev_table_build(const syn_law_t* w, double t0, double t1, rev_table_t* tab) {
    const double P = 2.0 * M_PI / w->wspin;
    tab->nrev = (int64_t)ceil((t1 - t0) / P) + 1;
    tab->z = (double*)malloc(sizeof(double) * 3 * (size_t)tab->nrev);
    for (int64_t k = 0; k < tab->nrev; ++k) {
        double e1[3], e2[3];
        spin_frame(w, t0 + ((double)k + 0.5) * P, tab->z + 3 * k, e1, e2);
    }
}

static int64_t transits_one(const syn_law_t* w, const rev_table_t* tab, const double r_equ[3], double t0,
                            double t1, double* tt, int8_t* ff, int64_t cap) {
    double r[3];
    equ_to_ecl(w->eps_obl, r_equ, r);
    const double P = 2.0 * M_PI / w->wspin;
    /* the spin axis moves by less than 0.012 rad in half a revolution */
    const double margin = sin(w->zeta_max) + 0.015 * (2.0 * M_PI / w->wspin) / 21600.0;
    int64_t nfound = 0;
    for (int64_t k = 0; k < tab->nrev; ++k) {
        const double tk = t0 + (double)k * P;
        if (tk >= t1) break;
        if (fabs(dot3(r, tab->z + 3 * k)) > margin) continue;
        double z[3], e1[3], e2[3];
        for (int fi = 0; fi < 2; ++fi) {
            int f = fi == 0 ? +1 : -1;
            /* initial guess within [tk, tk+P) */
            spin_frame(w, tk, z, e1, e2);
            double psi = atan2(dot3(r, e2), dot3(r, e1));
            double Om = w->Omega0 + w->wspin * tk;
            double t = tk + wrap_2pi(psi - f * 0.5 * w->gamma - Om) / w->wspin;
            for (int it = 0; it < 3; ++it) {
                spin_frame(w, t, z, e1, e2);
                psi = atan2(dot3(r, e2), dot3(r, e1));
                Om = w->Omega0 + w->wspin * t;
                t += wrap_pi(psi - f * 0.5 * w->gamma - Om) / w->wspin;
            }
            if (t < tk || t >= tk + P || t < t0 || t >= t1) continue;
            spin_frame(w, t, z, e1, e2);
            if (fabs(asin(dot3(r, z))) > w->zeta_max) continue;
            if (nfound < cap) { tt[nfound] = t; ff[nfound] = (int8_t)f; }
            ++nfound;
        }
    }
    return nfound;
}

/* Insertion sort of a star's transits by time (a handful per star). */
static void sort_transits(double* t, int8_t* f, int64_t n) {
    for (int64_t i = 1; i < n; ++i) {
        double tv = t[i]; int8_t fv = f[i];
        int64_t j = i - 1;
        while (j >= 0 && t[j] > tv) { t[j + 1] = t[j]; f[j + 1] = f[j]; --j; }
        t[j + 1] = tv; f[j + 1] = fv;
    }
}

/*
 * Pass 1: count transits per star.  counts[i] receives the number for star i.
 * ra, dec: star directions [rad].
 */
void syn_count_transits(const syn_law_t* w, int64_t nsrc, const double* ra, const double* dec,
                        double t0, double t1, int64_t* counts) {
    rev_table_t tab;
    rev_table_build(w, t0, t1, &tab);
#pragma omp parallel
    {
        double tt[4096]; int8_t ff[4096];
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < nsrc; ++i) {
            double r[3] = {cos(dec[i]) * cos(ra[i]), cos(dec[i]) * sin(ra[i]), sin(dec[i])};
            counts[i] = transits_one(w, &tab, r, t0, t1, tt, ff, 4096);
        }
    }
    free(tab.z);
}

/*
 * Pass 2: fill transit times and fov codes, grouped by star (offsets[i] is
 * the prefix sum of counts), each star's transits in increasing time.
 */
void syn_fill_transits(const syn_law_t* w, int64_t nsrc, const double* ra, const double* dec,
                       double t0, double t1, const int64_t* offsets, double* t_out, int8_t* f_out) {
    rev_table_t tab;
    rev_table_build(w, t0, t1, &tab);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nsrc; ++i) {
        double r[3] = {cos(dec[i]) * cos(ra[i]), cos(dec[i]) * sin(ra[i]), sin(dec[i])};
        int64_t cap = offsets[i + 1] - offsets[i];
        int64_t n = transits_one(w, &tab, r, t0, t1, t_out + offsets[i], f_out + offsets[i], cap);
        (void)n;
        sort_transits(t_out + offsets[i], f_out + offsets[i], cap);
    }
    free(tab.z);
}
