// Internal context of libagis and the kernel launchers shared by the host
// API (capi.hip) and the kernels (kernels.hip, store.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/agis.h"
#include "model.h"

namespace agis {

// Per-segment description of the attitude band systems (Sect. 5.2.2).
struct SegDesc {
    int64_t n_lo, n_hi;        // coefficient range of the segment system
    int64_t keep_lo, keep_hi;  // coefficients whose updates this segment supplies
    int64_t u_off;             // offset (in rows of 16) of its factor storage
};

// Number of sums per knot interval produced by the A/C pass: 10 block pairs
// (n <= m among the four B-splines) x 10 unique entries of the symmetric 4x4
// block, then 4 x 4 right-hand-side entries.
constexpr int IV_PAIRS = 10;
constexpr int IV_SUMS = IV_PAIRS * 10 + 16;
// calibration partial sums per interval: (sum W, sum W R) for fov +1 and -1
constexpr int IV_CAL = 4;

// A class of sources of the robust S block handled by the one-kernel path:
// positions [k0, k1) of the count-ordered launch, each with at most cap
// observations, blocks of nt threads.
struct SClass {
    int64_t k0, k1;
    int cap, nt;
};

struct Timers {
    hipEvent_t ev[10][2];
    bool valid[10];
};

}  // namespace agis

struct agis_ctx {
    agis_config_t cfg;
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    agis::DevConsts k;

    // knots
    int64_t n_knots = 0, N = 0, K = 0;   // N coefficients, K = N - 3 intervals
    std::vector<double> h_knots;
    double* knots = nullptr;
    agis::KnotTab* ktab = nullptr;       // [K] per-interval table of the observation model

    // observation store
    bool loaded = false;
    int64_t n_obs = 0, n_src = 0, n_cells = 0;
    bool has_ac = false;                 // some observation is across scan (input cell -1)
    // by (source, time)
    double* s_t = nullptr;
    double* s_eta = nullptr;
    float* s_sig = nullptr;
    int32_t* s_cell = nullptr;
    int32_t* s_ell = nullptr;
    int64_t* src_off = nullptr;          // [n_src + 1]
    int32_t* src_order = nullptr;        // [n_src] S-pass launch order (decreasing observation count)
    // by time
    double* t_t = nullptr;
    double* t_eta = nullptr;
    float* t_sig = nullptr;
    int32_t* t_cellfov = nullptr;         // cell * 2 + (fov < 0)
    int32_t* t_src = nullptr;
    int32_t* t_perm = nullptr;           // input index of each time-ordered observation
    int32_t* s_from_t = nullptr;         // time-order index of each (source, time)-ordered observation
    // frozen robust weights: sigma_eff = 1 / sqrt(W) of every observation in
    // both orders; while frozen, the plain kernels run with these in place
    // of sigma (one fixed weighted least-squares problem)
    double* s_sig_eff = nullptr;          // frozen sigma_eff = W^-1/2 (hybrid scheme), source order
    double* t_sig_eff = nullptr;          // the same in time order
    bool frozen = false;
    int64_t* iv_off = nullptr;           // [K + 1]
    int32_t* iv_cell = nullptr;          // [K][2] cell of the fov +1 / -1 observations (-1: none)
    int32_t* cell_iv = nullptr;          // [n_cells][2] interval range [lo, hi) of each cell

    // parameters
    double* s = nullptr;                 // [n_src][5]
    double* a = nullptr;                 // [N][4]
    double* gpar = nullptr;              // [2] global parameters: g0 (gamma = 1 + g0), g1 (held at zero)
    double* dgpar = nullptr;             // [2] the last global solve: the update of g0, the value of g1
    double* g_iv = nullptr;              // [K][5] per-interval sums of the global block (ppn only)
    double* c = nullptr;                 // [n_cells + 1]; entry n_cells (across scan) stays 0
    agis::SrcPrep* prep = nullptr;       // [n_src]
    double* s_ref = nullptr;             // [n_src][5] frame reference (optional)
    bool have_ref = false;

    // work arrays
    double* ds = nullptr;                // [n_src][5] last source update
    double* qsrc = nullptr;              // [n_src] Q_i after the S solve
    int32_t* sdef = nullptr;             // [n_src] defect per source
    double* svar = nullptr;              // [n_src][5] variances of the last S update (1 before any)
    double* iv_sums = nullptr;           // [K][IV_SUMS]
    double* iv_cal = nullptr;            // [K][IV_CAL]
    double* da = nullptr;                // [N][4]
    double* dc = nullptr;                // [n_cells]
    // large-scale AL geometric calibration (agis_load_geometry): three
    // shifted-Legendre coefficients per cell and CCD in place of the cell
    // offsets (held at zero); 0 CCDs: the cell offsets
    int32_t geo_ccds = 0;
    int32_t geo_ac_cells = 0;            // AC cells of the across-scan term (0: none)
    int64_t n_groups = 0;                // (n_cells + geo_ac_cells) * geo_ccds: AL groups, then AC
    double* geo = nullptr;               // [n_groups][3]
    double* dgeo = nullptr;              // [n_groups][3] the last update
    double* geo_sums = nullptr;          // [n_groups][9] normal equations of the last C update
    int32_t* t_geo_g = nullptr;          // time order: group of the record (-1 across scan)
    int32_t* s_geo_g = nullptr;          // source order
    float* t_geo_mu = nullptr;           // time order: across-scan pixel coordinate
    float* s_geo_mu = nullptr;           // source order
    double* t_eta0 = nullptr;            // time order: observed angles as loaded (t_eta adds the terms)
    double* s_eta0 = nullptr;            // source order
    double* geo_wr = nullptr;            // [n_al][2] W and W R of the last A/C pass (group order)
    int32_t* geo_pos = nullptr;          // time order -> position in the group order (-1 across scan)
    int64_t* geo_off = nullptr;          // [n_groups + 1] group ranges of the group order
    float* geo_mu_g = nullptr;           // group order: across-scan pixel coordinate
    int* geo_flags = nullptr;
    // small-scale AL term (eq:cc2): days of a long interval (0: none), its
    // values [K][geo_ccds][1966] after the groups' coefficients in geo and dgeo
    int32_t geo_small_days = 0;
    int64_t n_small = 0;
    int32_t* geo_coff = nullptr;         // [n_cells geo_ccds][1967] column ranges of the AL groups
    double* geo_colsum = nullptr;        // [n_cells geo_ccds][1966][4] column sums of the last C update
    double* geo_zpart = nullptr;         // [K geo_ccds][parts][packed triangle] partial sums of the block solve
    double* geo_dcol = nullptr;          // [K geo_ccds][1966][4] block diagonal, right-hand side, 1 / sqrt(diagonal)
    int32_t* seg_def = nullptr;          // [n_seg]
    std::vector<agis::SegDesc> h_segs;
    agis::SegDesc* segs = nullptr;
    double* ufac = nullptr;              // factor rows: [sum_seg 4*(n_hi-n_lo+1)][16]
    double* yfac = nullptr;              // forward-substituted right-hand sides
    int64_t ufac_rows = 0;
    double* red = nullptr;               // reduction scratch
    int64_t red_len = 0;
    double* eo = nullptr;                // [8] frame rotator parameters on device
    double* stat = nullptr;              // statistics scratch

    // robust mode: excess attitude noise per bucket, per-source varsigma,
    // and the seven by-source columns of the inner iteration (the first one
    // also holds R^2 - sigma^2 in time order for the eps_a estimate)
    int64_t n_buckets = 0;
    double* eps_a2 = nullptr;            // [n_buckets]
    double* vs = nullptr;                // [n_src][2]: along, across scan
    double* src_eps2 = nullptr;          // [n_src] robust mode 2: excess source noise eps_i^2 of the last S update
    double* src_D = nullptr;             // [n_src] ... and its significance D
    double* rcol = nullptr;              // [6][n_obs] (only when some source or bucket needs the HBM path)
    // one-kernel robust paths (robust mode 1): the classes of the S block,
    // the leading launch positions that keep the three-kernel path (more
    // observations than the LDS holds), and whether the excess-noise
    // estimate runs in one kernel (every bucket fits the LDS)
    std::vector<agis::SClass> s_classes;
    int64_t s_fallback = 0;
    int64_t eps_cap = 0;
    bool eps_fused = false;
    int robust_s_mode = 0;               // robust S block: 0 rows, varsigma and solves through HBM columns;
                                         // 1 rows to HBM columns, then varsigma and solves per source in
                                         // LDS; 2 the whole block per source in LDS (no HBM columns);
                                         // 3 the whole block per source with its rows in registers
    int sreg_rows = 4;                   // register path: rows per lane (at most 4)
    int irls_cache = 0;                  // column path, mode 1: 0 the inner rounds re-read every record;
                                         // 1 (2) 32 (64) lanes per source, each keeping its first records
                                         // in registers across the rounds
    bool robust_fused_eps = true;        // the excess-noise estimate in one kernel (values in LDS)
    int64_t robust_max_cap = INT64_MAX;  // largest source class of the one-kernel S path

    // learned extrapolation: update histories (rings of four), MLP weights
    // (FP32 master, BF16-rounded copy, Adam moments, gradient + loss) for
    // the source [0] and attitude-coefficient [1] networks, work buffers
    double* lh_anchor_s = nullptr;       // [n_src][5]
    double* lh_ring_s = nullptr;         // [4][n_src][5]
    double* lh_anchor_a = nullptr;       // [N][4]
    double* lh_ring_a = nullptr;         // [4][N][4]
    double* lh_anchor_c = nullptr;       // [n_cells]
    double* lh_ring_c = nullptr;         // [4][n_cells]
    double* asi_part = nullptr;          // accelerated iteration: block sums, result
    double* asi_out = nullptr;
    int lh_count = 0;
    float* mlp_w[2] = {nullptr, nullptr};
    float* mlp_wb[2] = {nullptr, nullptr};
    float* mlp_m1[2] = {nullptr, nullptr};
    float* mlp_m2[2] = {nullptr, nullptr};
    float* mlp_g[2] = {nullptr, nullptr};
    int mlp_t[2] = {0, 0};
    float* lf_X[2] = {nullptr, nullptr};
    float* lf_scale[2] = {nullptr, nullptr};
    float* lf_Y[2] = {nullptr, nullptr};
    double* bk_s[2] = {};                // state backups of the gated learned step
    double* bk_a[2] = {};
    double* bk_c[2] = {};
    double* bk_e[2] = {};
    double* chi2_part = nullptr;         // [ceil(K / 64)]
    double* chi2_out = nullptr;          // [2]

    // conjugate gradients (cg.hip): vectors over all unknowns, sources
    // [n_src][5], then attitude [N][4], then calibration [n_cells]
    double* rhs_s_out = nullptr;         // S pass: right-hand sides written here when set
    double* cg_r = nullptr;              // b - N x at the current iterate
    double* cg_z = nullptr;              // K^-1 r
    double* cg_p = nullptr;              // search direction
    double* cg_ry = nullptr;             // r and z at the new iterate (swapped with cg_r, cg_z)
    double* cg_zy = nullptr;
    double* cg_sy = nullptr;             // sources of the point being evaluated
    double* cg_part = nullptr;           // reduction partials [CG_BLOCKS][2] and of p'N p
    double* cg_qpart = nullptr;
    double* cg_out = nullptr;            // results [2]
    int cg_k = 0;                        // iterations done in the current cycle (0: a cycle starts)
    double cg_rho = 0.0;                 // r'z
    uint64_t cg_ver = 0;                 // state version the CG vectors belong to
    uint64_t xver = 1;                   // bumped by every call that changes the state outside CG

    // lanes per source in the S block
    int s_group = 16;
    int64_t select_reg_limit = INT64_MAX;   // robust quantiles: register-held keys up to this count
    int64_t select_reg_min_mean = 256;      // ... in the register kernel from this mean set size
    bool select_pair = true;                // ... both intersextile order statistics in one set of passes

    agis::Timers tm;
    double last_ms[6] = {0, 0, 0, 0, 0, 0};
    bool timing = true;                      // per-block HIP events (off inside a graph capture)

    // one captured iteration; rebuilt when gen (bumped by every call that
    // changes what the kernels are launched with) differs from graph_gen
    hipGraphExec_t graph_exec = nullptr;
    uint64_t gen = 1, graph_gen = 0;
};

namespace agis {

// robust mode in effect: 0, 1 or 2 (0 while the weights are frozen)
inline int robust_now(const agis_ctx* ctx) { return ctx->frozen ? 0 : ctx->cfg.robust; }

int set_error(agis_ctx* ctx, int code, const std::string& msg);
int hip_check(agis_ctx* ctx, hipError_t e, const char* what);

// store.hip
int build_store(agis_ctx* ctx, const agis_obs_soa_t* obs, int where);

// kernels.hip
void launch_prep_sources(agis_ctx* ctx);
void launch_source_update(agis_ctx* ctx);
// learned.hip
int mlp_num_weights(int which);
int mlp_num_inputs(int which);
int mlp_num_outputs(int which);
int mlp_num_targets(int which);
void launch_hist_record(agis_ctx* ctx, int slot);
void launch_hist_anchor(agis_ctx* ctx);
void launch_asi_sums(agis_ctx* ctx, int stride, double* part, double* out);
void launch_asi_apply(agis_ctx* ctx, double f);
void launch_features(agis_ctx* ctx, int which, float* X, float* scale);
void launch_mlp_forward(agis_ctx* ctx, int which, int64_t n, const float* X, float* Y);
void launch_mlp_grad(agis_ctx* ctx, int which, int64_t nb, const int64_t* idx, const float* X, const float* T,
                     float* part);
void launch_batch_idx(agis_ctx* ctx, int64_t nb, int64_t n, uint64_t seed, uint64_t step, int64_t* idx);
void launch_adam(agis_ctx* ctx, int which, float lr, int t);
void launch_round_weights(agis_ctx* ctx, int which);
void launch_apply_candidate(agis_ctx* ctx, const float* Cs, const float* Ca);
void launch_copy(agis_ctx* ctx, int64_t n, const double* src, double* dst);
void launch_chi2(agis_ctx* ctx, double* part, double* out);
// cg.hip
int64_t cg_size(const agis_ctx* ctx);
void launch_cg_gather(agis_ctx* ctx, double* r, double* z);
void launch_cg_step_state(agis_ctx* ctx, const double* v, double f);
void launch_cg_dot(agis_ctx* ctx, const double* a, const double* b, const double* c, double* out);
void launch_cg_dot2(agis_ctx* ctx, const double* a, const double* b1, const double* b2, double* out);
int64_t cg_quad_blocks(const agis_ctx* ctx);
void launch_cg_quad(agis_ctx* ctx, const double* p, double* part, double* out);
void launch_cg_direction(agis_ctx* ctx, double beta);
// robust.hip
void launch_source_update_robust(agis_ctx* ctx);
// plan of the robust kernels from the per-source offsets and the launch
// order (host copies); tells whether the HBM columns are needed
int robust_plan(agis_ctx* ctx, const std::vector<int64_t>& h_off, const std::vector<int32_t>& order,
                bool* need_columns);
void launch_excess_noise(agis_ctx* ctx);
void launch_freeze_sigma(agis_ctx* ctx);
void launch_ac_pass(agis_ctx* ctx);
void launch_band_solve(agis_ctx* ctx);
void launch_calib_solve(agis_ctx* ctx, double* rc = nullptr);   // rc: optional right-hand sides
// geo.hip
int load_geometry(agis_ctx* ctx, const int8_t* ccd, const float* mu, int32_t n_ccd, const int32_t* ac_cell,
                  int32_t n_ac_cells, int32_t small_days, int where);
void launch_geo_eta(agis_ctx* ctx);
void launch_geo_solve(agis_ctx* ctx);
void launch_geo_basic_angle(agis_ctx* ctx, double* out);   // out: device [n_cells / 2]
void launch_apply_attitude(agis_ctx* ctx);
void launch_global_solve(agis_ctx* ctx);
void launch_apply_add(agis_ctx* ctx, int64_t n, double* x, const double* dx);   // x += dx
void launch_apply_calibration(agis_ctx* ctx);
void launch_frame_fit(agis_ctx* ctx);
void launch_frame_apply(agis_ctx* ctx);
void launch_residuals(agis_ctx* ctx, double* R_input_order);
// statistics over n rows of width w (rms and max per column, col < 5);
// out[0..4] = rms, out[5..9] = max, out[10] = scalar sum of extra (or 0)
void launch_stats(agis_ctx* ctx, const double* x, int64_t n, int w, const double* extra, const int32_t* iextra,
                  double* out);

}  // namespace agis
