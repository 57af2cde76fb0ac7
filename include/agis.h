/*
 * libagis -- the per-iteration source (S), attitude (A) and calibration (C)
 * updating blocks and the frame rotator of the Gaia astrometric core
 * solution (Lindegren et al. 2012, "The astrometric core solution for the
 * Gaia mission", arXiv:1112.4139), on one AMD Instinct MI355X (gfx950).
 *
 * C ABI: plain pointers and sizes.  Every call returns AGIS_OK (0) or a
 * negative error code; agis_last_error() then describes the failure.  No C++
 * exception crosses the interface.  A context owns all device memory it
 * allocates; caller buffers are only read or written during the call.  One
 * context must not be used from two host threads at once.  Rank deficiency
 * of a block system is not an error: it is counted (Algorithm C1's defect d)
 * in the statistics.
 *
 * Units: times in seconds from the reference epoch of the astrometric
 * parameters; angles in radians; proper motions and the frame spin in radians
 * per Julian year (year_s seconds); the observer ephemeris in astronomical
 * units (a circular barycentric orbit, see agis_config_t).
 *
 * Pointers marked "where" are host memory when where == AGIS_HOST and device
 * memory of the context's GPU when where == AGIS_DEVICE (for instance the
 * data pointer of a torch tensor on that device; the copy is ordered on the
 * context's stream).
 */
#ifndef AGIS_H
#define AGIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AGIS_VERSION 100

enum {
    AGIS_OK = 0,
    AGIS_E_INVALID_ARG = -1, /* null pointer, bad enum, bad size */
    AGIS_E_SHAPE = -2,       /* sizes inconsistent with the configuration */
    AGIS_E_RANGE = -3,       /* index or time outside its valid range */
    AGIS_E_DEVICE = -4,      /* HIP runtime error */
    AGIS_E_OOM = -5,         /* device allocation failed */
    AGIS_E_NUMERIC = -6,     /* non-finite value detected */
    AGIS_E_STATE = -7        /* call out of order (e.g. update before load) */
};

enum { AGIS_HOST = 0, AGIS_DEVICE = 1 };
enum { AGIS_FP64 = 0, AGIS_MIXED = 1 };

typedef struct agis_ctx agis_ctx_t;

/*
 * Method constants and the synthetic world's auxiliary data.
 *   knots      : B-spline knot sequence tau_0..tau_{N+3} for cubic splines
 *                (order M = 4, Sect. 3.3 and Appendix B), non-decreasing,
 *                copied at create.  Observation times must lie in
 *                [tau_3, tau_N].
 *   gamma_c    : conventional basic angle Gamma_c (eq:srspropeta).
 *   t_ep, t_fr : reference epoch of the astrometric parameters (eq:uniform)
 *                and frame rotator epoch (eq:fr1) [s].
 *   lambda_reg : attitude regularisation lambda (eq:JfuncMod).
 *   seg_len, seg_overlap : attitude segments of seg_len knot intervals with
 *                L = seg_overlap intervals on each side (Sect. 5.2.2).
 *   eph_*      : observer ephemeris b_G(t) = R_x(eps_obl) eph_radius_au
 *                (cos L, sin L, 0), L = eph_L0 + eph_Lrate t, and its time
 *                derivative v_G (the auxiliary data of eq:astro).
 *   au_m, c_mps, year_s : astronomical unit [m], speed of light [m/s],
 *                Julian year [s].
 *   precision  : AGIS_FP64 or AGIS_MIXED.  MIXED keeps the observation
 *                model and residuals, the 5x5 and band Cholesky, the
 *                calibration solve and the frame rotator in FP64; the partials
 *                and the normal-equation sums of the S block and the A/C pass
 *                are single precision with compensated (Kahan) sums (in the
 *                A/C pass per 64-observation chunk of matrix-core sums).  The
 *                robust source inner iteration always runs in FP64.
 *   device     : HIP device ordinal; stream: hipStream_t or NULL (the
 *                context then creates its own default-priority stream).
 *   robust     : 0 = statistical weights W = 1/sigma^2; 1 = robust weighting
 *                (Sect. 5.1.2, 5.2.5): W = w(z)/sigma~^2 with the downweighting
 *                function w of eq:dw and sigma~^2 = sigma^2 + eps_a^2(t) of
 *                the attitude component the record measures (Sect. 3.6:
 *                along scan, across scan in the preceding or in the
 *                following field of view); the source update runs the inner
 *                iteration (initial downweights from half the intersextile
 *                range of the source's residuals of the record's kind,
 *                along or across scan, then four solves; excess source
 *                noise 0); the excess attitude noise eps_a (eq e09, 68th
 *                percentile of R^2 - sigma^2 over a component's records) is
 *                re-estimated per component and bucket after every source
 *                update and used by the attitude and calibration weights.
 *                2 = as 1 plus the excess source noise eps_i (Sect. 5.1.2):
 *                each round of the inner iteration fixes its w_l and solves
 *                Q(eps_i^2) = nu = n_i - n_out - 5 (n_out: w_l < 0.2) by up
 *                to three rational steps dy = (1 - Q/nu) Q / Q' from 0
 *                (eq:epsi; 0 when Q(0) <= nu), W_l = w_l / (sigma~_l^2 +
 *                eps_i^2) (eq:W, eq:wl); eps_i^2 also enters the attitude
 *                and calibration weights and eq e09 (R^2 - sigma^2 - eps_i^2).
 *   eps_bucket : knot intervals per eps_a bucket (robust only, >= 1).
 *   eps_a_init : eps_a of every bucket before the first estimate [rad].
 */
typedef struct {
    int64_t n_knots;
    const double* knots;
    double gamma_c;
    double t_ep, t_fr;
    double lambda_reg;
    int32_t seg_len, seg_overlap;
    double eph_radius_au, eph_L0, eph_Lrate, eps_obl;
    double au_m, c_mps, year_s;
    int32_t precision;
    int32_t device;
    void* stream;
    int32_t robust;
    int32_t eps_bucket;
    double eps_a_init;
    double defl;            /* 0, or GM_sun / (c^2 AU) [rad AU]: the Sun's light deflection in the model */
    int32_t ppn;            /* 1: the global block solves g0 (gamma = 1 + g0) in each iteration */
} agis_config_t;

/*
 * One observation record per element (Sect. 3.5, eq:synth with eq:resAL or
 * eq:resAC; the AL and AC components of an observation are separate
 * records), SoA:
 *   t       [n] observation time [s]
 *   eta_obs [n] along scan: observed AL field angle of the fiducial line,
 *               without the calibration term [rad] (model value eta_obs +
 *               c_cell); across scan: the observed AC field angle zeta [rad]
 *   sigma   [n] formal AL or AC standard uncertainty [rad], float32, > 0
 *   src     [n] source index in [0, n_src)
 *   fov     [n] field of view: +1 preceding, -1 following
 *   cell    [n] calibration cell in [0, n_cells), or -1 for an across-scan
 *               observation (no calibration parameter); cells are grouped in
 *               constraint pairs (2j, 2j+1) with c_2j + c_2j+1 = 0
 *               (eq:calCon); within one knot interval all AL observations of
 *               one field of view must share a cell, and each cell must cover
 *               a contiguous run of knot intervals (AGIS_E_SHAPE otherwise).
 * Across-scan observations enter the S and A blocks, the residuals, the
 * chi^2 and conjugate gradients; a context with robust != 0 refuses them
 * (AGIS_E_INVALID_ARG at load: the excess attitude noise of eq e09 is
 * estimated for the AL component only).
 */
typedef struct {
    int64_t n;
    const double* t;
    const double* eta_obs;
    const float* sigma;
    const int32_t* src;
    const int8_t* fov;
    const int32_t* cell;
} agis_obs_soa_t;

typedef struct {
    int64_t n_obs;           /* observations used */
    int64_t n_units;         /* sources / coefficients / cells updated */
    int64_t defect;          /* summed rank-defect count of Algorithm C1 */
    double rms_update[5];    /* RMS of the update per component: sources
                                (alpha*, delta, parallax, mu_alpha*, mu_delta);
                                attitude (x, y, z, w); calibration (value) */
    double max_update[5];
    double chi2;             /* sum of W R^2 after the S solve (eq:Qi summed) */
    double ms;               /* device time of the block [ms] */
} agis_block_stats_t;

typedef struct {
    agis_block_stats_t s, a, c;
    double eps_omega[6];     /* frame rotator parameters applied (0 if none) */
    double ms;               /* device time of the whole iteration [ms] */
} agis_iter_stats_t;

/* One step of the conjugate-gradient scheme (agis_cg_iterate). */
typedef struct {
    double alpha;            /* step length taken (0 at the start of a cycle or on breakdown) */
    double beta;             /* coefficient of the previous direction in the new one */
    double rho;              /* r'z after the step */
    int32_t cycle_start;     /* 1: this evaluation started a cycle (frame rotator, r, z, p = z at x) */
    int32_t breakdown;       /* 1: p'N p <= 0 or not finite; no move, the next step starts a cycle */
    double ms;               /* device time of the step [ms] */
} agis_cg_stats_t;

int agis_version(void);

/* Create a context on cfg->device; copies *cfg and the knots. */
int agis_create(const agis_config_t* cfg, agis_ctx_t** out);
void agis_destroy(agis_ctx_t* ctx);
/* Message of the last failed call on ctx (owned by ctx, valid until its
 * next call); with ctx == NULL, the last agis_create failure. */
const char* agis_last_error(const agis_ctx_t* ctx);

/* Observation store (Sect. 3.5 observation records).  Validates every
 * index and time, then builds the two device orders the blocks stream:
 * by (source, time) for S and by time for A and C, with left indices
 * (tau_l <= t < tau_{l+1}; t = tau_N in the last interval), source and knot
 * interval offsets.  n_src and n_cells fix the parameter vector sizes. */
int agis_load_observations(agis_ctx_t* ctx, const agis_obs_soa_t* obs, int64_t n_src, int64_t n_cells,
                           int where);

/* Parameters.  Sources [n][5] (alpha, delta, parallax, pm_alpha*, pm_delta);
 * attitude [N][4] B-spline coefficients (x, y, z, w) of eq:qspline;
 * calibration [n_cells]. */
int agis_set_sources(agis_ctx_t* ctx, int64_t n, const double* s5, int where);
int agis_get_sources(agis_ctx_t* ctx, int64_t n, double* s5, int where);
int agis_set_attitude(agis_ctx_t* ctx, int64_t n, const double* a4, int where);
int agis_get_attitude(agis_ctx_t* ctx, int64_t n, double* a4, int where);
int agis_set_calibration(agis_ctx_t* ctx, int64_t n, const double* c, int where);
int agis_get_calibration(agis_ctx_t* ctx, int64_t n, double* c, int where);

/*
 * Large-scale geometric calibration (Sect. 3.4, eq:etazeta, its large-scale
 * terms with one gate): per calibration cell (day and field of view) and
 * CCD, three coefficients c_r of the shifted Legendre polynomials L*_0..2
 * (orthogonal on [0, 1]) in x = (mu - 13.5) / 1966, mu the record's
 * across-scan pixel coordinate; an along-scan record's model value is
 * eta_obs + sum_r c_r L*_r(x) in place of eta_obs + c_cell.  Optionally the
 * across-scan term too: per AC cell (a field of view and a long interval,
 * numbered by the caller) and CCD three coefficients, an across-scan
 * record's residual then being zeta_obs + sum_r c_r L*_r(x) - zeta.  The C
 * block solves each group's 3x3 normal equations (eq:normC with eq:pdC) by
 * the modified Cholesky and applies eq:calCon for eq:cc1 (the AL constant
 * terms of a day's two cells and all CCDs sum to zero) and eq:cc3 (the AC
 * constant terms of an AC cell's CCDs sum to zero).  Optionally the
 * small-scale AL term delta-eta too: with small_days > 0 (at most 30) one
 * value per CCD, long interval k (runs of small_days days from the first
 * cell's day) and pixel column m = round(mu) in 14..1979, added to an
 * along-scan record's model value.  It shares the records of the AL groups
 * of its CCD and interval, which makes them one block: eq:normC over the
 * block's AL groups and 1966 values is solved exactly under eq:cc2 (for r =
 * 0, 1, 2 the update's values times L*_r((m - 13.5) / 1966) sum to zero),
 * the constrained least-squares update; a column or cell without records
 * keeps a zero update; then eq:cc1 as above.
 *
 * agis_load_geometry enables it after agis_load_observations: ccd [n] the
 * CCD index in [0, n_ccd) and mu [n] the pixel coordinate in [13.5, 1979.5]
 * of every record, in the input order of the observations (n = the loaded
 * count); ac_cell [n] (NULL, or with n_ac_cells > 0) each across-scan
 * record's AC cell in [0, n_ac_cells) (along-scan records' values are
 * ignored, and so are across-scan records' ccd and mu without ac_cell);
 * host or device memory by `where`; small_days: 0, or the long interval of
 * the small-scale term [days]; the coefficients start at zero and the
 * cell offsets are held at zero.  agis_set/get_geo_calibration: n = 3
 * (n_cells + n_ac_cells) n_ccd + K n_ccd 1966 values, [n_cells][n_ccd][3] AL,
 * [n_ac_cells][n_ccd][3] AC, then [K][n_ccd][1966] small-scale with K =
 * ceil(n_cells / 2 / small_days) (0 without it) [rad].  AGIS_E_SHAPE on a
 * count mismatch, AGIS_E_INVALID_ARG on an index, cell or coordinate out of
 * range, on small_days < 0 or above 30, or on 2^21 or more groups with it,
 * AGIS_E_STATE for the geometry in robust mode 2, for agis_set_calibration
 * while it is on, and for conjugate gradients and the recorded-update
 * schemes (agis_learned_*, agis_asi_step), which carry the cell offsets
 * only.  Loading observations again turns it off; so does an
 * agis_load_geometry rejected for a record's index, cell or coordinate (the
 * context then uses the cell offsets, which are zero if the model had been
 * on); a call refused for its arguments (n_ccd, n_ac_cells, small_days, the
 * group count) changes nothing.
 */
/*
 * Global block (Sect. 5.4, eq:normG) with the PPN parameter gamma = 1 + g0
 * (eq:gammaPPN): with cfg.defl > 0 the model deflects the coordinate
 * direction by the Sun's gravity, (1 + gamma) GM/(c^2 r) (e - (e.u)u) /
 * (1 + e.u) to first order (e the unit vector from the Sun, taken at the
 * barycentre, to the observer at distance r), before aberration; with
 * cfg.ppn each agis_iterate also solves g = (g0, g1) from eq:normG with the
 * A/C weights and residuals (S[ACG]) and applies the update of g0; g1 is
 * the pseudo-parameter of a global parallax shift, solved with g0 and never
 * applied.  agis_global_update: that solve and update alone at the current
 * parameters (dg, may be NULL: the update of g0 and the value of g1);
 * AGIS_E_STATE without cfg.ppn.  agis_set_global: g0 (0 at creation).
 * agis_get_global: out[0] g0, out[1] the last update of g0, out[2] the last
 * g1.  With the deflection (FP64 only; AGIS_E_INVALID_ARG at creation
 * otherwise, and for ppn without it), conjugate gradients, the
 * recorded-update schemes and frozen weights are refused (AGIS_E_STATE):
 * they carry s, a and c and the plain model only; the robust S block takes
 * the HBM-column path.
 */
int agis_global_update(agis_ctx_t* ctx, double dg[2]);
int agis_set_global(agis_ctx_t* ctx, double g0);
int agis_get_global(agis_ctx_t* ctx, double out[3]);

int agis_load_geometry(agis_ctx_t* ctx, int64_t n, const int8_t* ccd, const float* mu, int32_t n_ccd,
                       const int32_t* ac_cell, int32_t n_ac_cells, int32_t small_days, int where);
int agis_set_geo_calibration(agis_ctx_t* ctx, int64_t n, const double* c, int where);
int agis_get_geo_calibration(agis_ctx_t* ctx, int64_t n, double* c, int where);
/* The basic-angle offset per short interval (day) j, a monitored quantity
 * and not a parameter (Sect. 3.4, eq:DeltaGamma): the mean over the AF CCDs
 * of the preceding field of view's AL constant term minus the following
 * one's, (1/n_ccd) sum_n (c_0(P, n, j) - c_0(F, n, j)), which the paper
 * writes with its 62 AF CCDs.  out [n_days] (n_days = n_cells / 2) [rad],
 * host or device memory by `where`; AGIS_E_STATE without the geometric
 * calibration, AGIS_E_SHAPE on a count mismatch. */
int agis_basic_angle(agis_ctx_t* ctx, int64_t n_days, double* out, int where);

/* S block (Sect. 5.1): per source, eq:normS with the design matrix of
 * eq:designS at the current (s, a, c), solved by Algorithms C1-C3;
 * alpha is updated by d_1 / cos(delta). */
int agis_source_update(agis_ctx_t* ctx, agis_block_stats_t* st);
/* A block (Sect. 5.2): regularised band normal equations eq:normAmod per
 * overlapping segment, Algorithms C1-C3 on the band, updates kept by the
 * selection rule of Sect. 5.2.2. */
int agis_attitude_update(agis_ctx_t* ctx, agis_block_stats_t* st);
/* C block (Sect. 5.3): per-cell normal equations eq:normC (Phi = 1), then
 * the constraint projection eq:calCon. */
int agis_calibration_update(agis_ctx_t* ctx, agis_block_stats_t* st);
/* A and C together from one pass of residuals at the current parameters
 * (the bracketed pair of the S[ACG] scheme, Sect. 4.6, without G). */
int agis_attitude_calibration_update(agis_ctx_t* ctx, agis_block_stats_t* st_a, agis_block_stats_t* st_c);

/* Frame rotator (Sect. 6.1).  The reference catalogue s_ref [n_src][5]
 * defines the S_PM comparison of eq:cond-mu3 at t = t_ep (eq:fr-Delta1).
 * frame_fit solves the weighted least squares for eps_omega = (eps_X,
 * eps_Y, eps_Z [rad], omega_X, omega_Y, omega_Z [rad/yr]) over all sources:
 * each condition equation is weighted by the inverse formal variance of its
 * parameter from the last source update (the diagonal of the inverse 5x5
 * normal matrix, Sect. 5.1.1; Sect. 6.1.4 asks for a weighted fit without
 * fixing the weights); a parameter whose variance is zero or not finite (a
 * singular source system, or no source update yet with variance 0) gets
 * weight 0, and before any source update every variance is 1 (unit
 * weights).  frame_apply transforms all sources rigorously (Sect. 6.1.2)
 * and all attitude coefficients by eq:fr-q4. */
int agis_set_frame_reference(agis_ctx_t* ctx, int64_t n, const double* s_ref5, int where);
int agis_frame_fit(agis_ctx_t* ctx, double eps_omega[6]);
int agis_frame_apply(agis_ctx_t* ctx, const double eps_omega[6]);

/* n_iter simple iterations S[AC] (Sect. 4.5, 4.6), each followed by the frame
 * rotator when a reference is set.  per_iter may be NULL or hold n_iter
 * entries. */
int agis_iterate(agis_ctx_t* ctx, int32_t n_iter, agis_iter_stats_t* per_iter);
/* The same n_iter iterations replayed from a HIP graph of one iteration
 * (captured on the first call, and again after agis_load_observations or
 * agis_set_frame_reference); the results equal agis_iterate's bit for bit.
 * Saves the per-kernel launch cost where the kernels are short; records no
 * per-block times (agis_kernel_times keeps those of the last agis_iterate). */
int agis_iterate_graph(agis_ctx_t* ctx, int32_t n_iter);
/* Times the source update with 8, 16 and 32 lanes per source on the loaded
 * problem (twice each, from the current state, restored bit for bit
 * afterwards: sources, their derived data and variances) and keeps the
 * fastest; *s_group (may be NULL) receives it.  The default, 16, is the best
 * for ~160 observations per source.  In robust mode 1 it then times the
 * paths of the S block the same way (per-observation columns in HBM with
 * the intersextile order statistics selected together or one after the
 * other; the rows in HBM and the inner iteration per source in LDS; the
 * whole block per source in LDS; the whole block per source with its rows
 * in registers) and keeps the fastest; the paths give the same numbers up
 * to the order of their sums (the register path forms the weights of the
 * first three inner rounds from FP32 copies of the design row, which moves
 * them by rounding of ~1e-7 relative in R). */
int agis_autotune(agis_ctx_t* ctx, int32_t* s_group);
/* The launch choices in effect: out[0] lanes per source of the S block,
 * out[1] the robust S path (0 HBM columns, 1 rows in HBM then LDS, 2 all in
 * LDS, 3 rows in registers), out[2] 1 if the columns path selects both
 * intersextile order statistics in one set of radix passes, out[3] 1 if
 * the excess attitude noise is estimated in one kernel, out[4] the inner
 * rounds of the columns path: 0 every record re-read from the columns each
 * round, 1 (2) 32 (64) lanes per source keeping their first 8 records in
 * registers across the rounds.  out: 5 ints. */
int agis_get_tuning(const agis_ctx_t* ctx, int32_t out[5]);

/* Residuals R_l (eq:resAL) at the current parameters, in the input order of
 * agis_load_observations. */
int agis_residuals(agis_ctx_t* ctx, double* R, int where);

/* Sizes of the loaded problem (any pointer may be NULL). */
int agis_problem_size(const agis_ctx_t* ctx, int64_t* n_obs, int64_t* n_src, int64_t* n_att, int64_t* n_cells,
                      int64_t* n_segments);

/* Device time [ms] of the last launch of each hot kernel, measured with
 * HIP events on the context stream: [0] source update (in the robust mode
 * every launch of the inner iteration), [1] attitude and calibration
 * accumulation, [2] band solve, [3] calibration solve, [4] frame rotator,
 * [5] excess attitude noise estimate (robust mode; 0 otherwise). */
int agis_kernel_times(const agis_ctx_t* ctx, double ms[6]);

/* Excess attitude noise (robust mode): eps_a^2 [rad^2] per attitude
 * component and bucket of eps_bucket knot intervals, component-major: the
 * n_b = ceil((N - 3) / eps_bucket) buckets of the along-scan component, then
 * those of across scan in the preceding field of view (fov +1), then those of
 * the following one (fov -1); n = 3 n_b.  A component without records in a
 * bucket estimates 0 there.  Set before an update to impose values; read
 * after one to inspect the estimate.  AGIS_E_STATE when the context is not
 * robust; AGIS_E_SHAPE when n differs. */
int agis_set_excess_noise(agis_ctx_t* ctx, int64_t n, const double* eps_a2, int where);
int agis_get_excess_noise(agis_ctx_t* ctx, int64_t n, double* eps_a2, int where);
/* Re-estimate eps_a^2 per bucket from the residuals at the current
 * parameters (eq e09), as the iteration does after the source update. */
int agis_excess_noise_update(agis_ctx_t* ctx);
/* Excess source noise (robust mode 2, Sect. 5.1.2) of the last source
 * update: eps_i^2 [rad^2] and its significance D = (Q(0) - nu) /
 * (2 nu)^1/2 (eq:D; 0 when nu <= 0) of each of the n = n_src sources; zero
 * before the first update.  AGIS_E_STATE unless robust mode 2;
 * AGIS_E_SHAPE when n differs. */
int agis_get_source_noise(agis_ctx_t* ctx, int64_t n, double* eps_i2, double* D, int where);

/*
 * Learned extrapolation of the simple iteration (an extension of the paper's
 * method: it generalises the accelerated simple iteration of Sect. 4.7,
 * whose premise is that the updates decay geometrically along the slowest
 * eigenvectors of the iteration).  Two MLPs, which = 0 for sources and 1 for
 * attitude coefficients, map per unit the last four recorded updates u_k
 * (newest first), normalised by their RMS s, and two descriptors (sources:
 * log(n_obs + 1)/5 and the sine of the ecliptic latitude; coefficients: sine
 * and cosine of twice the coefficient's angle about its z axis) to four
 * mixing coefficients c; the candidate is x + sum_k c_k u_k, a step inside
 * the span of the unit's recent updates (sources: alpha moves by the mixed
 * d alpha* over cos delta).
 * Inputs F = 22 / 18 (the first 20 / 16 are the normalised updates, newest
 * first, components d alpha*, d delta, d parallax, d mu_alpha*, d mu_delta /
 * d a_x, d a_y, d a_z, d a_w), outputs O = 4, two hidden layers of 64 with
 * tanh.  Weights [F*64 W1][64 b1][64*64 W2][64 b2][O*64 W3][O b3]
 * (row-major, row = output unit) in FP32; the forward and backward passes
 * use them rounded to BF16 with FP32 accumulation.  Training targets T have
 * NC = 5 / 4 columns: the displacement to learn in units of s.
 */
/* Start a history: the current parameters (sources, attitude, calibration)
 * become the anchor. */
int agis_learned_reset(agis_ctx_t* ctx);
/* Record (current - anchor) as the newest update; the current parameters
 * become the anchor.  A "record" may follow any number of iterations. */
int agis_learned_record(agis_ctx_t* ctx);
/* Features X [n][F] and scales s [n] of every unit from the last four
 * recorded updates (AGIS_E_STATE with fewer than four). */
int agis_learned_features(agis_ctx_t* ctx, int32_t which, int64_t n, float* X, float* scale, int where);
/* Weights: Glorot-uniform from a SplitMix64 stream (biases 0); load n =
 * the network's weight count FP32 weights in the layout above (from host
 * or device memory; the Adam moments and step count restart at zero); get
 * them back. */
int agis_mlp_init(agis_ctx_t* ctx, int32_t which, uint64_t seed);
int agis_mlp_load(agis_ctx_t* ctx, int32_t which, int64_t n, const float* w, int where);
int agis_mlp_get_weights(agis_ctx_t* ctx, int32_t which, int64_t n, float* w, int where);
/* Y [n][4] = MLP(X [n][F]), the mixing coefficients. */
int agis_mlp_forward(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, float* Y, int where);
/* Gradient of L = sum_i |yhat_i - T_i|^2 / (2 n), yhat_i[c] = sum_k
 * MLP(X_i)[k] X_i[k NC + c] (T [n][NC]), with respect to the weights
 * (grad [NW], same layout) and L, at the current weights. */
int agis_mlp_gradient(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T, float* grad,
                      float* loss, int where);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, rate lr) on the gradient of L
 * over the whole batch (X [n][F], T [n][NC], host or device); *loss (host,
 * may be NULL) receives L at the weights before the step. */
int agis_mlp_train_step(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T, int where,
                        float lr, float* loss);
/* steps Adam steps (beta 0.9, 0.999, eps 1e-8, rate lr) on minibatches of
 * `batch` samples drawn from (X, T) by a counter-based hash of (seed, step);
 * loss_out (host, may be NULL) receives each step's minibatch loss. */
int agis_mlp_train(agis_ctx_t* ctx, int32_t which, int64_t n, const float* X, const float* T, int where,
                   int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss_out);
/* sum over observations of R^2 / sigma^2 at the current parameters. */
int agis_chi2(agis_ctx_t* ctx, double* q);
/* The same sum as agis_chi2, bit for bit, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): it allocates nothing.  Its partial sums live in a
 * per-GPU static scratch array of 1 MiB (131,072 doubles), so it handles at
 * most 131,071 x 64 = 8,388,544 knot intervals (AGIS_E_SHAPE beyond).  *q
 * is host memory (where = AGIS_HOST) or device memory of the context's GPU
 * (AGIS_DEVICE).  Every call on one GPU shares that GPU's scratch array:
 * calls that overlap on one GPU (two host threads, or two streams running
 * at once) race and must be serialised by the caller. */
int agis_chi2_noalloc(agis_ctx_t* ctx, double* q, int where);
/* Ungated: x <- x + s MLP(features) for sources and coefficients, then a new
 * history starts from x.  AGIS_E_STATE with fewer than four records. */
int agis_learned_apply(agis_ctx_t* ctx);
/* Gated learned step, two S[AC] iterations: from the current state x0 one
 * plain iteration gives x1, and one iteration from the candidate x0 + s y
 * gives c1.  The one iteration damps what the MLP gets wrong along the
 * well-determined directions, along which sum W R^2 is steep.  c1 is kept
 * (the history restarts from it) when q_cand = sum W R^2 (c1), with W the
 * plain weight 1 / sigma^2, is below q_plain = sum W R^2 (x1); otherwise the
 * state becomes x1 and the history goes on, its next record spanning one
 * iteration more.  Sources, attitude, calibration and, when robust, the
 * excess attitude noise are saved and restored on the device.
 * AGIS_E_STATE with fewer than four records. */
int agis_learned_step(agis_ctx_t* ctx, double* q_plain, double* q_cand, int32_t* accepted);

/* One block of the learned-accelerated scheme (agis_iterate_learned). */
typedef struct {
    int32_t iterations;      /* S[AC] iterations the block ran: m, plus 2 when gated */
    int32_t gated;           /* 1: the history held four records and the gated step ran */
    int32_t accepted;        /* 1: the candidate was kept (the history restarted from it) */
    double q_plain, q_cand;  /* the gate's sum W R^2 after the plain and the candidate iteration */
} agis_learned_stats_t;

/* n_blocks blocks of the learned-accelerated simple iteration: each runs m
 * S[AC] + frame iterations, records their change as the newest update
 * (agis_learned_record) and, once the history holds four records, takes the
 * gated learned step (agis_learned_step).  A history is started first when
 * none exists (agis_learned_reset otherwise sets where it starts).  The
 * networks are those set by agis_mlp_init / agis_mlp_load / training.
 * per_block (may be NULL) receives n_blocks entries.  n_blocks >= 0,
 * m >= 1 (else AGIS_E_INVALID_ARG). */
int agis_iterate_learned(agis_ctx_t* ctx, int32_t n_blocks, int32_t m, agis_learned_stats_t* per_block);

/*
 * Accelerated simple iteration (Sect. 4.7): when successive updates shrink
 * by a nearly constant ratio lambda, the updates still to come sum to
 * lambda / (1 - lambda) times the newest one.  Over the recorded history
 * (agis_learned_reset / agis_learned_record, a record every m iterations),
 * lambda is the least-squares ratio sum u1 u2 / sum u2^2 of the newest (u1)
 * to the previous (u2) parallax update over the sources 0, stride,
 * 2 stride, ... (parallaxes do not change with the frame orientation),
 * clamped to [0, lambda_max]; sources, attitude and calibration then move
 * by f = lambda / (1 - lambda) times their newest update (alpha by the
 * update in alpha* over cos delta) and a new history starts.  No step
 * (f = 0, history kept) when lambda <= 0.  stride >= 1, 0 <= lambda_max < 1
 * (else AGIS_E_INVALID_ARG); AGIS_E_STATE with fewer than two records.
 */
int agis_asi_step(agis_ctx_t* ctx, int32_t stride, double lambda_max, double* lambda, double* factor);

/*
 * Conjugate gradients (Sect. 4.7: the paper's baseline scheme, built on the
 * same S, A and C block solves as the simple iteration).  Preconditioned CG
 * in the Polak-Ribiere form for the normal equations linearised at the
 * current parameters, with these definitions:
 *   unknowns: per source (d alpha*, d delta, d parallax, d mu_alpha*,
 *     d mu_delta), per attitude coefficient its 4 components, per cell its
 *     calibration; a step v moves alpha by v_alpha* / cos delta and every
 *     other parameter additively;
 *   r(x): the right-hand sides b - N x of eq:normS, eq:normAmod (with the
 *     regularisation) and eq:normC at state x;
 *   z(x) = K^-1 r(x): the S, A (overlapping segments) and C (with eq:calCon)
 *     block updates, all three computed at the same state x (block Jacobi);
 *   p'N p: the quadratic form of the normal matrix at the current state,
 *     summed over the observations (weights 1 / sigma^2, the regularisation
 *     terms with lambda^2);
 *   an iteration: alpha = r'z / p'N p, x <- x + alpha p, r and z evaluated
 *     at the new x, beta = max(0, r'(z - z_old) / r_old'z_old),
 *     p <- z + beta p.
 * A cycle starts with the frame rotator (when a frame reference is set) and
 * one evaluation at x itself (r, z, p = z); it runs `restart` iterations.
 * Each call performs n_eval steps (cycle starts and iterations alike; an
 * iteration costs one pass of the three blocks, like one simple iteration,
 * plus one pass over the observations for p'N p) and keeps the CG vectors
 * for the next call; any other call that changes the parameters or the
 * problem (set_*, loads, updates, iterations, frame application,
 * accelerated or learned steps) makes the next step start a new cycle.  A
 * non-positive or non-finite p'N p leaves x unchanged and ends the cycle.
 * per_eval (optional, n_eval entries) receives the statistics of each step.
 * restart >= 1 and n_eval >= 0 (else AGIS_E_INVALID_ARG); AGIS_E_STATE in
 * the robust mode unless its weights are frozen (agis_freeze_weights):
 * robust weights change with the residuals, and the paper switches between
 * the simple iteration and CG for that reason.
 */
int agis_cg_iterate(agis_ctx_t* ctx, int32_t n_eval, int32_t restart, agis_cg_stats_t* per_eval);

/*
 * Frozen weights, the switch of the hybrid scheme (Sect. 4.7: the simple
 * iteration runs while the robust weights still change, then CG, which
 * needs a fixed normal matrix).  freeze != 0: at the current parameters and
 * excess attitude noise, every observation's weight of the A/C pass,
 * W = w(R / sigma~) / sigma~^2 with sigma~^2 = sigma^2 + eps_a^2 (eq:dw,
 * eq:W), is fixed as sigma_eff = 1 / sqrt(W) (FP64; W = 0 gives the
 * largest finite float), and from then on the S, A and C blocks, the
 * iterations and agis_cg_iterate solve the plain weighted least-squares
 * problem with sigma_eff in place of sigma (no inner iteration, no
 * excess-noise update).  freeze == 0: back to the robust weighting.
 * Calling it again re-freezes at the current parameters.  Device memory:
 * 16 bytes per observation (both orders), allocated on the first freeze.  AGIS_E_STATE
 * when the context is not robust.
 */
int agis_freeze_weights(agis_ctx_t* ctx, int32_t freeze);

#ifdef __cplusplus
}
#endif
#endif
