/*
 * AGIS CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision implementation of the source (S), attitude
 * (A) and calibration (C) updating blocks and the frame rotator of the
 * astrometric core solution (Lindegren et al. 2012, arXiv:1112.4139), written
 * from the paper's equations and algorithms in their order.  It exists to
 * check the GPU library; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header or
 * table with the GPU library.
 *
 * Units: t in seconds from the reference epoch; angles in radians; proper
 * motions and frame spin in radians per Julian year; ephemeris in AU.
 */
#ifndef AGIS_ORACLE_H
#define AGIS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n_knots;          /* N + M, M = 4 */
    const double* knots;      /* non-decreasing knot sequence tau_0..tau_{N+3} */
    double gamma_c;           /* conventional basic angle [rad] */
    double t_ep;              /* reference epoch of the astrometric parameters [s] */
    double t_fr;              /* frame rotator epoch [s] */
    double lambda_reg;        /* attitude regularisation lambda */
    int32_t seg_len;          /* attitude segment length [knot intervals] */
    int32_t seg_overlap;      /* L: half overlap [knot intervals] */
    double eph_radius_au;     /* circular barycentric orbit radius [AU] */
    double eph_L0;            /* orbital longitude at t = 0 [rad] */
    double eph_Lrate;         /* orbital angular rate [rad/s] */
    double eps_obl;           /* ecliptic obliquity [rad] */
    double au_m;              /* astronomical unit [m] */
    double c_mps;             /* speed of light [m/s] */
    double year_s;            /* Julian year [s] */
    int32_t robust;           /* 0: w_l = 1, eps = 0; 1: downweighting and excess attitude noise;
                                 2: also the excess source noise eps_i of eq:epsi */
    int32_t eps_bucket;       /* knot intervals per excess-attitude-noise bucket (robust) */
    int32_t geo_ccds;         /* 0: one calibration offset per cell; n > 0: the large-scale AL
                                 geometric calibration of eq:etazeta, three shifted-Legendre
                                 coefficients per cell and CCD (n CCDs) in the AC pixel coordinate */
    int32_t geo_ac_cells;     /* with the AC term (obs ac_cell): its cells, each a field of view
                                 and a long interval k of eq:etazeta */
    double defl;              /* 0: no light deflection; else GM_sun / (c^2 AU) [rad AU]: the Sun's
                                 gravitational light deflection with gamma = 1 + g0 (eq:gammaPPN) */
    int32_t ppn;              /* 1: the global block solves g0 (eq:normG) in each iteration */
    int32_t geo_small_days;   /* with the geometric calibration, 0 or the days of a long interval k
                                 of the small-scale AL term delta-eta of eq:etazeta: one value per
                                 CCD, long interval and pixel column m = round(mu) (1966), under
                                 eq:cc2 */
} orc_world_t;

typedef struct {
    int64_t n;
    const double* t;          /* observation time [s] */
    const double* eta_obs;    /* observed AL field angle without calibration, or the
                                 observed AC field angle zeta (cell < 0) [rad] */
    const float* sigma;       /* formal AL (AC) uncertainty [rad] */
    const int32_t* src;       /* source index */
    const int8_t* fov;        /* +1 preceding, -1 following */
    const int32_t* cell;      /* calibration cell; -1: across-scan observation (eq:resAC) */
    const double* sigma_eff;  /* NULL, or the uncertainty that replaces sigma: the frozen
                                 sigma_eff of the hybrid scheme (orc_frozen_sigma) [rad] */
    const int8_t* ccd;        /* geometric calibration: CCD index of the record (else NULL) */
    const float* mu;          /* geometric calibration: AC pixel coordinate, 13.5 .. 1979.5 */
    const int32_t* ac_cell;   /* NULL, or with the geometric calibration the AC calibration cell
                                 (0 .. geo_ac_cells - 1) of each across-scan record (-1 for
                                 along-scan ones): the large-scale AC term of eq:etazeta with
                                 eq:cc3 */
} orc_obs_t;

typedef struct {
    int64_t n_src, n_att, n_cells;
    double* s;                /* [n_src][5] alpha, delta, parallax, pm_alpha*, pm_delta */
    double* a;                /* [n_att][4] x, y, z, w */
    double* c;                /* [n_cells] */
    int64_t n_buckets;        /* ceil((N - 3) / eps_bucket) when robust, else 0 */
    double* eps_a2;           /* [3][n_buckets] excess attitude variance eps_a^2 [rad^2] of the
                                 AL, ACP and ACF components (Sect. 3.6) */
    double* src_eps2;         /* [n_src] excess source variance eps_i^2 of the last S update (robust 2; may be NULL) */
    double* src_D;            /* [n_src] its significance D of eq:D (robust 2; may be NULL) */
    double* geo;              /* [n_cells][geo_ccds][3] geometric calibration coefficients
                                 (eq:etazeta, r = 0, 1, 2) [rad], followed with ac_cell by the
                                 AC ones [geo_ac_cells][geo_ccds][3], then with geo_small_days the
                                 small-scale ones [K][geo_ccds][1966], K = ceil(n_cells / 2 /
                                 geo_small_days); NULL when geo_ccds = 0 */
    double g0;                /* global parameter of eq:gammaPPN: gamma = 1 + g0 */
} orc_state_t;

/* --- Appendix A: quaternions -------------------------------------------- */
void orc_qmul(const double a[4], const double b[4], double out[4]);
void orc_qconj(const double a[4], double out[4]);
void orc_qinv(const double a[4], double out[4]);
void orc_frame_rotate(const double q[4], const double v[3], double out[3]);
void orc_vector_rotate(const double q[4], const double v[3], double out[3]);
void orc_quat2mat(const double q[4], double A[9]);
void orc_qrot(const double phi[3], double out[4]);

/* --- Appendix B: B-splines ---------------------------------------------- */
int64_t orc_left_index(const double* knots, int64_t n_knots, double t);
void orc_bspline(const double* knots, int64_t ell, double t, double b[4]);

/* --- Appendix C: modified Cholesky (dense, row-major n x n) --------------- */
int orc_chol_c1(double* U, int n);
void orc_chol_c2(const double* U, int n, double* y);
void orc_chol_c3(const double* U, int n, double* x);
/* band storage: UB[j*(hb+1) + k] is element (j, j+k), 0 <= k <= hb */
int orc_band_c1(double* UB, int n, int hb);
void orc_band_c2(const double* UB, int n, int hb, double* y);
void orc_band_c3(const double* UB, int n, int hb, double* x);

/* --- Sect. 3: observation model ------------------------------------------ */
/* Per observation: computed field angle eta, instrument angles phi, zeta,
 * field index f, residual R (with calibration), design row -dR/ds (5),
 * dR/dq (4), B-spline values (4) and left index, unnormalised attitude
 * quaternion (4) and D = 1 - |sum a_n B_n|^2.  Any output pointer may be NULL. */
void orc_observe(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                 int64_t i0, int64_t i1,
                 double* eta, double* phi, double* zeta, int8_t* f, double* R,
                 double* dsrc, double* dq, double* bspl, int64_t* ell, double* qraw, double* D);
void orc_ephemeris(const orc_world_t* w, double t, double b[3], double v[3]);
void orc_normal_triad(double alpha, double delta, double p[3], double q[3], double r[3]);

/* --- Sect. 5.1.2, 5.2.5: robust weighting ------------------------------------ */
/* Downweighting function w(z) (eq:dw). */
double orc_weight_function(double z);
/* p-quantile of x[0..n-1] by linear interpolation between order statistics
 * at (n - 1) p (Hyndman-Fan type 7); n = 0 gives 0.  x is not modified. */
double orc_quantile(const double* x, int64_t n, double p);
/* Excess attitude noise (eq e09) per component and bucket from the
 * residuals at the current state: eps_a2[a n_buckets + j] = max(0,
 * F_0.68(R_l^2 - sigma_l^2 - eps_i^2)) over the observations of component a
 * (0 along scan, 1 across scan in the preceding, 2 in the following field of
 * view) in bucket j (knot intervals [j B, (j + 1) B)); 0 for an empty set.
 * Needs robust >= 1. */
void orc_excess_attitude_noise(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st);

/* --- Sect. 5: update blocks ----------------------------------------------- */
/* S block for all sources; updates st->s in place.  Optional outputs:
 * d[n_src][5] updates, Q[n_src] = R'WR after the solve, defect[n_src],
 * var[n_src][5] the diagonal of the inverse normal matrix (first-order
 * variances, Sect. 5.1.1 / eq:cov).  With robust = 1 each source runs the
 * inner iteration of Sect. 5.1.2 (initial downweights from half the
 * intersextile range of its residuals, then four solves with the weights
 * re-derived from the updated residuals; excess source noise 0). */
void orc_source_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st,
                       double* d, double* Q, int32_t* defect, double* var);
/* A block (all segments); residuals from the current state.  d[n_att][4]
 * receives the applied update (may be NULL); returns the summed defect. */
int64_t orc_attitude_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* d);
/* One segment K only: solve and return the kept updates in d[n_att][4]
 * (entries outside the kept range are left untouched); no state change. */
int64_t orc_attitude_segment(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st,
                             int64_t K, double* d, int64_t* keep_lo, int64_t* keep_hi);
int64_t orc_num_segments(const orc_world_t* w);
/* C block; d[n_cells] receives the applied update (may be NULL). */
/* d (may be NULL) receives the update: [n_cells], or with the geometric
 * calibration [n_cells][geo_ccds][3] (followed by the AC groups' with
 * ac_cell, then the small-scale coefficients with geo_small_days). */
void orc_calibration_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* d);
/* S[AC]: S, then A and C from the same post-S residuals. */
void orc_iterate_sac(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st, double* var);
/* Sect. 5.4: the global update of g0 from eq:normG at the current state
 * (W from the A/C weights), solved jointly with the pseudo-parameter g1 (a
 * global parallax shift, never applied), applied; returns the update (0
 * without a pivot). */
double orc_global_update(const orc_world_t* w, const orc_obs_t* obs, orc_state_t* st);

/* Right-hand sides b - N x of the S, A and C normal equations at the current
 * state, summed over all observations (no robust weighting). */
void orc_normal_rhs(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* rs, double* ra,
                    double* rc);

/* v' N v for the normal matrix of the S, A and C blocks at the current state;
 * v holds the source, then the attitude, then the calibration unknowns. */
double orc_normal_quadratic(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, const double* v);

/* Frozen weights: sigma_eff = 1 / sqrt(W_l) of every observation at the
 * current state, W_l the A/C weight (eq:dw, eq:W); input order. */
void orc_frozen_sigma(const orc_world_t* w, const orc_obs_t* obs, const orc_state_t* st, double* sig);

/* --- Sect. 6.1: frame rotator --------------------------------------------- */
/* eps_omega = (eps_X, eps_Y, eps_Z [rad], omega_X, omega_Y, omega_Z [rad/yr]).
 * var[n_src][5] (may be NULL: unit weights) weights each condition equation
 * by the inverse variance of its parameter; a source with a zero or
 * non-finite variance gets zero weight. */
void orc_frame_fit(const orc_world_t* w, const orc_state_t* st, const double* s_ref, const double* var,
                   double eps_omega[6]);
void orc_frame_apply(const orc_world_t* w, orc_state_t* st, const double eps_omega[6]);

#ifdef __cplusplus
}
#endif
#endif
