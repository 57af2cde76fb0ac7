// Large-scale geometric calibration (Sect. 3.4, eq:etazeta, the large-scale
// terms): per calibration cell (day and field of view) and CCD three
// coefficients of the shifted Legendre polynomials L*_0..2 in the
// across-scan pixel coordinate mu, x = (mu - 13.5) / 1966, in place of one
// offset per cell; optionally the across-scan term, three coefficients per
// AC cell (field of view and long interval) and CCD.
//
// The term enters the residual additively (eq:resAL, eq:resAC): R = eta_obs
// + sum_r c_r L*_r(x) - eta (zeta across scan).  The stored observed angles
// of both orders therefore carry it -- eta = eta_obs + term, refreshed
// whenever the coefficients change -- and every pass reads them unchanged,
// with the per-cell offsets held at zero.  The C block (Sect. 5.3, eq:normC with
// eq:pdC: dR/dc_r = L*_r(x)) is block-diagonal in groups of three
// coefficients (a cell and a CCD).  The records with a group are given a
// second order at load, by group and time within a group (a stable radix
// sort of the group indices); the A/C pass writes each record's W and W R
// at its place in that order, so that one block per group sums W L_r L_s and
// W R L_r over a contiguous range in a fixed order; one thread per
// constraint set then solves the set's 3x3 systems (the small modified
// Cholesky) and applies eq:calCon for its constraint, eq:cc1 (the AL
// constant terms of a day's two cells and all CCDs sum to zero) or eq:cc3
// (the AC constant terms of an AC cell's CCDs sum to zero): their mean is
// removed.
//
// The small-scale AL term (eq:etazeta's delta-eta with eq:cc2) adds one
// value per CCD, long interval k (a run of `days` days) and pixel column
// m = round(mu), 1966 a block.  It shares every record with the AL groups
// of its CCD and interval, so a block (CCD, interval) is solved as one
// system: the along-scan groups' records are ordered by column within a
// group as well; eight lanes per group and column sum W, W L_1, W L_2 and
// -W R over its records; one thread per block and column adds the block's
// cells; eight workgroups per block sum the reduced normal matrix over
// column ranges; one workgroup per block adds them, eliminates the diagonal
// small-scale part and the three eq:cc2 multipliers in closed form and
// solves the remaining system of the cells' 3 n_cells coefficients (at most
// 180) by the modified Cholesky in LDS, then the small-scale values by back
// substitution.  The eq:cc1 projection follows as without the term.
#include <hipcub/hipcub.hpp>

#include "agis_internal.h"
#include "model.h"

namespace agis {
namespace {

template <typename T>
int dalloc(agis_ctx* ctx, T** p, size_t n, const char* what) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(ctx, AGIS_E_OOM, std::string("device allocation failed: ") + what);
    }
    return AGIS_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

__device__ __forceinline__ double shifted_legendre(int r, double x) {
    return r == 0 ? 1.0 : (r == 1 ? 2.0 * x - 1.0 : 6.0 * x * x - 6.0 * x + 1.0);
}

__device__ __forceinline__ double geo_x(float mu) { return ((double)mu - 13.5) / 1966.0; }

constexpr int DG_COLS = 1966;       // pixel columns m = 14 .. 1979
constexpr int DG_SHIFT = 11;        // column bits of the group-order keys with the small-scale term

// The nearest pixel column m = round(mu) as 0 .. 1965 (1979.5 stays on the
// last column).
__device__ __forceinline__ int geo_column(float mu) {
    int m = (int)floor((double)mu + 0.5);
    return (m > 1979 ? 1979 : m) - 14;
}

// Group index and pixel coordinate of every record in time order from the
// input columns (t_perm: time index -> input index): an along-scan record's
// cell and CCD; with ac_cell an across-scan record's AC cell and CCD after
// the n_cells n_ccd AL groups; -1 for an across-scan record without it.
// Flags: 1 a CCD index out of range, 2 a coordinate not in [13.5, 1979.5],
// 4 an AC cell out of range.
__global__ void k_geo_index(int64_t n, const int32_t* __restrict__ t_perm, const int32_t* __restrict__ t_cellfov,
                            int32_t n_cells, const int8_t* __restrict__ ccd_in, const float* __restrict__ mu_in,
                            const int32_t* __restrict__ ac_cell_in, int32_t n_ac_cells, int32_t n_ccd,
                            int32_t* __restrict__ g_out, float* __restrict__ mu_out, int* __restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = t_perm[i];
        const int32_t cell = t_cellfov[i] >> 1;
        const float mu = mu_in[j];
        int32_t g = -1;
        int32_t base = -1;                       // the record's cell among the groups' cells
        if (cell < n_cells) {
            base = cell;
        } else if (ac_cell_in) {
            const int32_t ac = ac_cell_in[j];
            if (ac < 0 || ac >= n_ac_cells) atomicOr(flags, 4);
            else base = n_cells + ac;
        }
        if (base >= 0 || (cell >= n_cells && ac_cell_in)) {
            const int c = ccd_in[j];
            if (c < 0 || c >= n_ccd) atomicOr(flags, 1);
            else if (base >= 0) g = base * n_ccd + c;
            if (!(mu >= 13.5f && mu <= 1979.5f)) atomicOr(flags, 2);
        }
        g_out[i] = g;
        mu_out[i] = mu;
    }
}

template <typename T>
__global__ void k_geo_gather(int64_t n, const int32_t* __restrict__ from, const T* __restrict__ src,
                             T* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[from[i]];
}

// eta = eta_obs + sum_r c_r L*_r(x) of the record's group (nothing across
// scan), the sum taken from r = 0 up, plus along scan the small-scale value
// of the record's CCD, long interval and column when days > 0 (groups below
// n_al are along scan: cell * n_ccd + CCD; small: the first small-scale value).
__global__ void k_geo_eta(int64_t n, const double* __restrict__ eta0, const int32_t* __restrict__ g,
                          const float* __restrict__ mu, const double* __restrict__ geo, int32_t n_al, int32_t n_ccd,
                          int32_t days, int64_t small, double* __restrict__ eta) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t gi = g[i];
        double v = 0.0;
        if (gi >= 0) {
            const double x = geo_x(mu[i]);
            const double* c = geo + 3 * (int64_t)gi;
            v = c[0] * shifted_legendre(0, x);
            v += c[1] * shifted_legendre(1, x);
            v += c[2] * shifted_legendre(2, x);
            if (days > 0 && gi < n_al) {
                const int32_t cell = gi / n_ccd, ccd = gi - cell * n_ccd;
                const int64_t blk = (int64_t)((cell >> 1) / days) * n_ccd + ccd;
                v += geo[small + blk * DG_COLS + geo_column(mu[i])];
            }
        }
        eta[i] = eta0[i] + v;
    }
}

// Sort keys of the group order: the group, or n_groups without one (last);
// shifted left by `shift` bits with the record's pixel column below.
__global__ void k_geo_keys(int64_t n, const int32_t* __restrict__ g, const float* __restrict__ mu, int32_t n_groups,
                           int shift, uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = g[i] >= 0 ? ((uint32_t)g[i] << shift) | (shift ? (uint32_t)geo_column(mu[i]) : 0u)
                           : (uint32_t)n_groups << shift;
        idx[i] = (int32_t)i;
    }
}

// From the sorted keys and time indices: each time-order record's place in
// the group order (-1 for a record without a group) and the group order's
// coordinates.  end: the key of "no group".
__global__ void k_geo_order(int64_t n, const uint32_t* __restrict__ key, const int32_t* __restrict__ idx,
                            uint32_t end, const float* __restrict__ t_mu, int32_t* __restrict__ pos,
                            float* __restrict__ mu_g) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = idx[k];
        const bool in = key[k] < end;
        pos[i] = in ? (int32_t)k : -1;
        if (in) mu_g[k] = t_mu[i];
    }
}

// off[j] = the first place in the sorted keys with a key of at least j <<
// shift (j = 0..n_out - 1): with shift 0 the group ranges, with the column
// bits and j = group * 2^shift + column the column ranges.
__global__ void k_geo_offsets(int64_t n, const uint32_t* __restrict__ key, int64_t n_out, int shift,
                              int64_t* __restrict__ off) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_out; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t want = (uint64_t)j << shift;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((uint64_t)key[mid] < want) lo = mid + 1;
            else hi = mid;
        }
        off[j] = lo;
    }
}

// Column ranges of the along-scan groups: coff[g * 1967 + c] = the first
// place of group g's column c (c = 1966: the group's end).
__global__ void k_geo_col_offsets(int64_t n, const uint32_t* __restrict__ key, int64_t n_al,
                                  int32_t* __restrict__ coff) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_al * (DG_COLS + 1);
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = j / (DG_COLS + 1), c = j - g * (DG_COLS + 1);
        const uint64_t want = ((uint64_t)g << DG_SHIFT) + (uint64_t)c;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((uint64_t)key[mid] < want) lo = mid + 1;
            else hi = mid;
        }
        coff[j] = (int32_t)lo;
    }
}

constexpr int GEO_NT = 256;

// Normal equations of one group (block): its contiguous range of the group
// order, each thread summing its strided records, then a fixed-order block
// sum.  out: [group][9] = N00 N01 N02 N11 N12 N22 b0 b1 b2 with
// N = sum W L L', b = -sum W R L.
__global__ __launch_bounds__(GEO_NT) void k_geo_sums(int64_t n_groups, const int64_t* __restrict__ off,
                                                     const float* __restrict__ mu, const double* __restrict__ wr,
                                                     double* __restrict__ out) {
    __shared__ double red[(GEO_NT / 64) * 9];
    const int64_t gi = blockIdx.x;
    if (gi >= n_groups) return;
    const int64_t l0 = off[gi], l1 = off[gi + 1];
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t l = l0 + threadIdx.x; l < l1; l += GEO_NT) {
        const double W = wr[2 * l], WR = wr[2 * l + 1];
        const double x = geo_x(mu[l]);
        double L[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) L[r] = shifted_legendre(r, x);
        s[0] += L[0] * W * L[0];
        s[1] += L[0] * W * L[1];
        s[2] += L[0] * W * L[2];
        s[3] += L[1] * W * L[1];
        s[4] += L[1] * W * L[2];
        s[5] += L[2] * W * L[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) s[6 + r] -= L[r] * WR;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double v = wave_sum(s[e]);
        if (lane == 0) red[wv * 9 + e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < GEO_NT / 64; ++w) t += red[w * 9 + threadIdx.x];
        out[9 * gi + threadIdx.x] = t;
    }
}

// One thread per constraint set of per_set consecutive groups from group
// first: their 3x3 solves (unless solve is false: the updates are already in
// dgeo), then eq:calCon for its constraint (the set's mean constant term
// removed).  AL: a day's 2 n_ccd groups (eq:cc1); AC: an AC cell's n_ccd
// groups (eq:cc3).
__global__ void k_geo_solve(int64_t n_sets, int64_t first, int32_t per_set, bool solve,
                            const double* __restrict__ sums, double* __restrict__ dgeo) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_sets;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g0 = first + j * per_set, per_day = per_set;
        double mean = 0.0;
        for (int64_t k = 0; k < per_day; ++k) {
            double* d = dgeo + 3 * (g0 + k);
            if (solve) {
                const double* s = sums + 9 * (g0 + k);
                double U[9] = {s[0], s[1], s[2], s[1], s[3], s[4], s[2], s[4], s[5]};
                double x[3] = {s[6], s[7], s[8]};
                small_chol_solve<3>(U, x);
                d[0] = x[0];
                d[1] = x[1];
                d[2] = x[2];
            }
            mean += d[0];
        }
        mean /= (double)per_day;
        for (int64_t k = 0; k < per_day; ++k) dgeo[3 * (g0 + k)] -= mean;
    }
}

// Per along-scan group g and column c (DG_LPC lanes each, striding over
// the column's records of the group order, so that a wave's loads cover
// DG_LPC consecutive records of each of its columns; then a fixed-order
// butterfly over the lanes): cs = {sum W, sum W L_1, sum W L_2, -sum W R}
// at colsum[(g * 1966 + c) * 4].
constexpr int DG_LPC = 8;
__global__ void k_dg_colsums(int64_t n_al, const int32_t* __restrict__ coff, const float* __restrict__ mu,
                             const double* __restrict__ wr, double* __restrict__ colsum) {
    const int sub = threadIdx.x & (DG_LPC - 1);
    const int64_t per = (int64_t)blockDim.x / DG_LPC;
    for (int64_t j = blockIdx.x * per + threadIdx.x / DG_LPC; j - (threadIdx.x / DG_LPC) < n_al * DG_COLS;
         j += (int64_t)gridDim.x * per) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        const bool in = j < n_al * DG_COLS;
        if (in) {
            const int64_t g = j / DG_COLS, c = j - g * DG_COLS;
            const int64_t l0 = coff[g * (DG_COLS + 1) + c], l1 = coff[g * (DG_COLS + 1) + c + 1];
            for (int64_t l = l0 + sub; l < l1; l += DG_LPC) {
                const double W = wr[2 * l], WR = wr[2 * l + 1];
                const double x = geo_x(mu[l]);
                s0 += W;
                s1 += W * shifted_legendre(1, x);
                s2 += W * shifted_legendre(2, x);
                s3 -= WR;
            }
        }
#pragma unroll
        for (int m = DG_LPC / 2; m >= 1; m >>= 1) {
            s0 += __shfl_xor(s0, m, DG_LPC);
            s1 += __shfl_xor(s1, m, DG_LPC);
            s2 += __shfl_xor(s2, m, DG_LPC);
            s3 += __shfl_xor(s3, m, DG_LPC);
        }
        if (in && sub == 0) {
            double* o = colsum + 4 * j;
            o[0] = s0;
            o[1] = s1;
            o[2] = s2;
            o[3] = s3;
        }
    }
}

// Per block (long interval k, CCD n; blk = k n_ccd + n) and column: the
// diagonal D_m = sum W and the right-hand side -sum W R of the small-scale
// value, over the interval's cells in order, and the column's scale
// 1 / sqrt(D_m) (0 for a column without records): dcol[(blk * 1966 + c) * 4].
__global__ void k_dg_colred(int64_t n_blk, int32_t n_ccd, int32_t days, int64_t n_cells,
                            const double* __restrict__ colsum, double* __restrict__ dcol) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_blk * DG_COLS;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t blk = j / DG_COLS, c = j - blk * DG_COLS;
        const int64_t k = blk / n_ccd, nn = blk - k * n_ccd;
        const int64_t c0 = 2 * k * days, c1 = min<int64_t>(c0 + 2 * (int64_t)days, n_cells);
        double d = 0.0, r = 0.0;
        for (int64_t cell = c0; cell < c1; ++cell) {
            const double* s = colsum + 4 * ((cell * n_ccd + nn) * DG_COLS + c);
            d += s[0];
            r += s[3];
        }
        dcol[4 * j] = d;
        dcol[4 * j + 1] = r;
        dcol[4 * j + 2] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
        dcol[4 * j + 3] = 0.0;
    }
}

constexpr int DG_NT = 512;          // threads of the block solve
constexpr int DG_T = 6;             // side of a thread's tile of the accumulated matrix
constexpr int DG_CH = 32;           // columns staged in LDS at a time
constexpr int DG_NE_MAX = 180;      // cells' coefficients of a block: 60 cells, 30 days
constexpr int DG_NP_MAX = 186;      // with the three polynomials and the right-hand side, to a multiple of 6

__host__ __device__ constexpr int dg_np(int ne) { return ((ne + 4 + DG_T - 1) / DG_T) * DG_T; }
__host__ __device__ constexpr int64_t dg_packed(int np) { return (int64_t)np * (np + 1) / 2; }
// dynamic LDS of the block solve: the packed matrix, then the cells' right-hand
// side and activity (2 Ne values) and 15 small values
__host__ __device__ constexpr size_t dg_lds_bytes(int ne) {
    return (size_t)(dg_packed(dg_np(ne)) + 2 * ne + 16) * sizeof(double);
}
static_assert(dg_np(DG_NE_MAX) == DG_NP_MAX, "the padded size of the largest block");
static_assert((DG_NP_MAX / DG_T) * (DG_NP_MAX / DG_T + 1) / 2 <= DG_NT, "one tile of the lower triangle per thread");
static_assert(DG_NT / DG_NP_MAX >= 2, "at least two staged vectors at a time (the prefetch count assumes it)");
__device__ __forceinline__ int64_t pk(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }   // i >= j
constexpr int DG_SPAN = 256;                                    // columns of an accumulation part
constexpr int DG_PARTS = (DG_COLS + DG_SPAN - 1) / DG_SPAN;     // accumulation parts per block
constexpr int64_t DG_PACK = dg_packed(DG_NP_MAX);               // stride of a part's packed triangle

// The accumulation of the block solve, split over DG_PARTS workgroups per
// block: workgroup (blk, part) sums z_m z_m' over the columns part * DG_SPAN
// .. (part + 1) * DG_SPAN - 1 (z_m as in k_dg_block; 0 past the last column)
// into zpart[(blk * DG_PARTS + part) * DG_PACK], the packed lower triangle.
__global__ __launch_bounds__(DG_NT) void k_dg_accum(int32_t n_ccd, int32_t days, int64_t n_cells,
                                                    const double* __restrict__ colsum,
                                                    const double* __restrict__ dcol,
                                                    double* __restrict__ zpart) {
    const int64_t blk = blockIdx.x / DG_PARTS;
    const int part = (int)(blockIdx.x - blk * DG_PARTS), mb = part * DG_SPAN;
    const int64_t k = blk / n_ccd, nn = blk - k * n_ccd;
    const int64_t c0 = 2 * k * days, c1 = min<int64_t>(c0 + 2 * (int64_t)days, n_cells);
    const int nc = (int)(c1 - c0), ne = 3 * nc, np = dg_np(ne);
    const int tid = threadIdx.x;
    const double* dc = dcol + 4 * blk * DG_COLS;
    // --- Z = sum_m z_m z_m', a 6x6 tile of the lower triangle per thread
    const int ntile = np / DG_T;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= tid) ++ti;      // tile row of this thread
    const int tj = tid - ti * (ti + 1) / 2;
    const bool own = ti < ntile;
    double acc[DG_T * DG_T];
#pragma unroll
    for (int e = 0; e < DG_T * DG_T; ++e) acc[e] = 0.0;
    __shared__ double stage[DG_CH * DG_NP_MAX];      // DG_CH staged vectors
    // Staging: thread t fills entry i = t % np of the columns m0 + t / np,
    // m0 + t / np + rows, ... (rows = DG_NT / np vectors at a time), so that
    // its source is fixed: a cell's column sums (i < ne), a polynomial, or
    // the right-hand side; loads without branches on the data.
    const int rows = DG_NT / np, srow = tid / np, si = tid - srow * np;
    const bool stager = srow < rows;
    const int kind = si < ne ? 0 : (si < ne + 3 ? 1 : (si == ne + 3 ? 2 : 3));
    const double* src = kind == 0 ? colsum + 4 * ((c0 + si / 3) * n_ccd + nn) * DG_COLS + (si - 3 * (si / 3))
                                  : dc + 1;
    auto zval = [&](int m) -> double {               // z_m[si] for column m (0 past the last column)
        const int mc = m < DG_COLS ? m : DG_COLS - 1;
        const double s = m < DG_COLS ? dc[4 * mc + 2] : 0.0;
        const double x = ((double)(mc + 14) - 13.5) / 1966.0;
        const double v = kind == 1 ? shifted_legendre(si - ne, x) : (kind == 3 ? 0.0 : src[4 * mc]);
        return v * s;
    };
    constexpr int PF = (DG_CH + 1) / 2;               // vectors per stager: rows >= 2 (np <= 186)
    double pf[PF];                                    // the next stage, loaded during the current one
#pragma unroll
    for (int q = 0; q < PF; ++q) pf[q] = stager && srow + q * rows < DG_CH ? zval(mb + srow + q * rows) : 0.0;
    for (int m0 = mb; m0 < mb + DG_SPAN; m0 += DG_CH) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (stager && srow + q * rows < DG_CH) stage[(srow + q * rows) * np + si] = pf[q];
        __syncthreads();
        if (m0 + DG_CH < mb + DG_SPAN) {
#pragma unroll
            for (int q = 0; q < PF; ++q)
                pf[q] = stager && srow + q * rows < DG_CH ? zval(m0 + DG_CH + srow + q * rows) : 0.0;
        }
        if (own) {
#pragma unroll 2
            for (int mm = 0; mm < DG_CH; ++mm) {
                const double* z = stage + mm * np;
                double a[DG_T], b[DG_T];
#pragma unroll
                for (int q = 0; q < DG_T; ++q) {
                    a[q] = z[DG_T * ti + q];
                    b[q] = z[DG_T * tj + q];
                }
#pragma unroll
                for (int p = 0; p < DG_T; ++p)
#pragma unroll
                    for (int q = 0; q < DG_T; ++q) acc[p * DG_T + q] += a[p] * b[q];
            }
        }
    }
    if (own) {
        double* zp = zpart + ((int64_t)blk * DG_PARTS + part) * DG_PACK;
#pragma unroll
        for (int p = 0; p < DG_T; ++p)
#pragma unroll
            for (int q = 0; q < DG_T; ++q) {
                const int i = DG_T * ti + p, j = DG_T * tj + q;
                if (i >= j) zp[pk(i, j)] = acc[p * DG_T + q];
            }
    }
}

// The C update of one block (long interval k, CCD n; one workgroup each):
// with z_m = [B_m, L*_0..2(x_m), b_m] / sqrt(D_m) over the active columns
// (D_m > 0; B_m: the column's sums W L_r of each cell of the block, b_m: -sum
// W R), Z = sum_m z_m z_m' (lower triangle, packed, in LDS; the sum of
// k_dg_accum's partial sums over column ranges) holds B'D^-1 B,
// G = B'D^-1 C, H = C'D^-1 C, B'D^-1 b and C'D^-1 b.  Eliminating the
// small-scale values d = D^-1 (b - B e - C nu) and the eq:cc2 multipliers
// nu = H^-1 (C'D^-1 b - G'e) leaves, for the cells' coefficients e,
//     (E - B'D^-1 B + G H^-1 G') e = b_e - B'D^-1 b + G H^-1 C'D^-1 b,
// E and b_e the groups' 3x3 sums (k_geo_sums); a cell without records keeps
// e = 0.  That system goes through the modified Cholesky (a pivot that is
// not positive gives a zero column and a zero unknown) and two triangular
// solves, then nu and d follow.  Writes the cells' three coefficients and the
// block's 1966 small-scale values of dgeo (0 for a column without records).
__global__ __launch_bounds__(DG_NT) void k_dg_block(int32_t n_ccd, int32_t days, int64_t n_cells,
                                                    const int64_t* __restrict__ off,
                                                    const double* __restrict__ colsum,
                                                    const double* __restrict__ dcol,
                                                    const double* __restrict__ zpart,
                                                    const double* __restrict__ sums, int64_t small,
                                                    double* __restrict__ dgeo) {
    extern __shared__ double lds[];
    const int64_t blk = blockIdx.x;
    const int64_t k = blk / n_ccd, nn = blk - k * n_ccd;
    const int64_t c0 = 2 * k * days, c1 = min<int64_t>(c0 + 2 * (int64_t)days, n_cells);
    const int nc = (int)(c1 - c0), ne = 3 * nc, np = dg_np(ne);
    const int tid = threadIdx.x;
    double* Z = lds;                                  // packed lower triangle, np x np
    double* ex = lds + dg_packed(np);                 // the cells' right-hand side, then solution [ne]
    double* act = ex + ne;                            // 1: the cell of row i has records [ne]
    double* hs = act + ne;                            // H^-1 [9], w = H^-1 C'D^-1 b [3], nu [3]
    const double* dc = dcol + 4 * blk * DG_COLS;
    // --- Z = sum_m z_m z_m' from the partial sums of k_dg_accum, in order
    for (int64_t e = tid; e < dg_packed(np); e += DG_NT) {
        double v = 0.0;
        for (int part = 0; part < DG_PARTS; ++part) v += zpart[((int64_t)blk * DG_PARTS + part) * DG_PACK + e];
        Z[e] = v;
    }
    for (int i = tid; i < ne; i += DG_NT) {
        const int64_t g = (c0 + i / 3) * n_ccd + nn;
        act[i] = off[g + 1] > off[g] ? 1.0 : 0.0;
    }
    __syncthreads();
    // --- H^-1 (cofactors of the 3x3 SPD matrix) and w = H^-1 C'D^-1 b
    if (tid == 0) {
        const double h00 = Z[pk(ne, ne)], h10 = Z[pk(ne + 1, ne)], h11 = Z[pk(ne + 1, ne + 1)];
        const double h20 = Z[pk(ne + 2, ne)], h21 = Z[pk(ne + 2, ne + 1)], h22 = Z[pk(ne + 2, ne + 2)];
        const double a00 = h11 * h22 - h21 * h21, a01 = h20 * h21 - h10 * h22, a02 = h10 * h21 - h20 * h11;
        const double det = h00 * a00 + h10 * a01 + h20 * a02;
        const double inv = det != 0.0 ? 1.0 / det : 0.0;
        const double a11 = h00 * h22 - h20 * h20, a12 = h10 * h20 - h00 * h21, a22 = h00 * h11 - h10 * h10;
        const double Hi[9] = {a00 * inv, a01 * inv, a02 * inv, a01 * inv, a11 * inv,
                              a12 * inv, a02 * inv, a12 * inv, a22 * inv};
        for (int e = 0; e < 9; ++e) hs[e] = Hi[e];
        for (int s = 0; s < 3; ++s) {
            double v = 0.0;
            for (int t = 0; t < 3; ++t) v += Hi[3 * s + t] * Z[pk(ne + 3, ne + t)];
            hs[9 + s] = v;
        }
    }
    __syncthreads();
    // --- the reduced system in place: A = E - Z + G H^-1 G', right-hand side in ex
    for (int e = tid; e < ne * ne; e += DG_NT) {
        const int i = e / ne, j = e - i * ne;
        if (j > i) continue;
        double v;
        if (act[i] == 0.0 || act[j] == 0.0) {
            v = i == j ? 1.0 : 0.0;
        } else {
            double Ev = 0.0;
            if (i / 3 == j / 3) {
                const int a = j - 3 * (j / 3), b = i - 3 * (i / 3);           // a <= b
                const int idx = a == 0 ? b : (a == 1 ? 2 + b : 5);
                Ev = sums[9 * ((c0 + i / 3) * n_ccd + nn) + idx];
            }
            double gg = 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                double t = 0.0;
#pragma unroll
                for (int u = 0; u < 3; ++u) t += hs[3 * s + u] * Z[pk(ne + u, j)];
                gg += Z[pk(ne + s, i)] * t;
            }
            v = Ev - Z[pk(i, j)] + gg;
        }
        Z[pk(i, j)] = v;
    }
    for (int i = tid; i < ne; i += DG_NT) {
        double v = 0.0;
        if (act[i] != 0.0) {
            const int cell = i / 3, r = i - 3 * cell;
            v = sums[9 * ((c0 + cell) * n_ccd + nn) + 6 + r] - Z[pk(ne + 3, i)];
#pragma unroll
            for (int s = 0; s < 3; ++s) v += Z[pk(ne + s, i)] * hs[9 + s];
        }
        ex[i] = v;
    }
    __syncthreads();
    // --- modified Cholesky A = L L' (right-looking over A's lower triangle):
    // step p leaves column p as it is and updates the trailing entries by
    // A_ij -= A_ip (A_jp / A_pp) when the pivot A_pp is positive (else column
    // p is zero); afterwards each column is divided by the square root of
    // its pivot, which gives L (a column with a pivot that is not positive
    // becomes zero).  One barrier per step.
    for (int p = 0; p < ne; ++p) {
        const double piv = Z[pk(p, p)];
        if (piv > 0.0) {
            const double ip = 1.0 / piv;
            const int rem = ne - p - 1, n_tri = rem * (rem + 1) / 2;
            for (int t = tid; t < n_tri; t += DG_NT) {
                // trailing entry t of the packed lower triangle: row a, column b <= a
                int a = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
                if ((a + 1) * (a + 2) / 2 <= t) ++a;
                if (a * (a + 1) / 2 > t) --a;
                const int i = p + 1 + a, j = p + 1 + (t - a * (a + 1) / 2);
                Z[pk(i, j)] -= Z[pk(i, p)] * (Z[pk(j, p)] * ip);
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < ne * ne; e += DG_NT) {
        const int i = e / ne, j = e - i * ne;
        if (j >= i) continue;
        const double piv = Z[pk(j, j)];
        Z[pk(i, j)] = piv > 0.0 ? Z[pk(i, j)] / sqrt(piv) : 0.0;
    }
    __syncthreads();
    for (int p = tid; p < ne; p += DG_NT) {
        const double piv = Z[pk(p, p)];
        Z[pk(p, p)] = piv > 0.0 ? sqrt(piv) : 0.0;
    }
    __syncthreads();
    // --- L y = rhs, then L' e = y (a zero pivot gives a zero unknown): one
    // wavefront, row i in lane i % 64, slot i / 64, of registers; the pivot
    // row's value broadcast by a shuffle
    if (tid < 64) {
        double xr[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) xr[s] = tid + 64 * s < ne ? ex[tid + 64 * s] : 0.0;
        for (int p = 0; p < ne; ++p) {
            const int slot = p >> 6;
            const double mine = slot == 0 ? xr[0] : (slot == 1 ? xr[1] : xr[2]);
            const double xp = __shfl(mine, p & 63, 64);
            const double d = Z[pk(p, p)];
            const double y = d > 0.0 ? xp / d : 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int i = tid + 64 * s;
                if (i == p) xr[s] = y;
                else if (i > p && i < ne) xr[s] -= Z[pk(i, p)] * y;
            }
        }
        for (int p = ne - 1; p >= 0; --p) {
            const int slot = p >> 6;
            const double mine = slot == 0 ? xr[0] : (slot == 1 ? xr[1] : xr[2]);
            const double yp = __shfl(mine, p & 63, 64);
            const double d = Z[pk(p, p)];
            const double x = d > 0.0 ? yp / d : 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int i = tid + 64 * s;
                if (i == p) xr[s] = x;
                else if (i < p) xr[s] -= Z[pk(p, i)] * x;
            }
        }
#pragma unroll
        for (int s = 0; s < 3; ++s)
            if (tid + 64 * s < ne) ex[tid + 64 * s] = xr[s];
    }
    __syncthreads();
    // --- nu = H^-1 (C'D^-1 b - G'e)
    if (tid == 0) {
        double q[3];
        for (int s = 0; s < 3; ++s) {
            double v = Z[pk(ne + 3, ne + s)];
            for (int i = 0; i < ne; ++i) v -= Z[pk(ne + s, i)] * ex[i];
            q[s] = v;
        }
        for (int s = 0; s < 3; ++s) hs[12 + s] = hs[3 * s] * q[0] + hs[3 * s + 1] * q[1] + hs[3 * s + 2] * q[2];
    }
    __syncthreads();
    // --- the cells' coefficients and the small-scale values
    for (int i = tid; i < ne; i += DG_NT) dgeo[3 * ((c0 + i / 3) * n_ccd + nn) + (i - 3 * (i / 3))] = ex[i];
    for (int m = tid; m < DG_COLS; m += DG_NT) {
        const double D = dc[4 * m];
        double v = 0.0;
        if (D > 0.0) {
            const double x = ((double)(m + 14) - 13.5) / 1966.0;
            // B_m e over the cells, each cell's column sums one 32-byte load,
            // four partial sums
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int cell = 0; cell < nc; ++cell) {
                const double4 b = *reinterpret_cast<const double4*>(
                    colsum + 4 * (((c0 + cell) * n_ccd + nn) * DG_COLS + m));
                acc[cell & 3] += b.x * ex[3 * cell] + b.y * ex[3 * cell + 1] + b.z * ex[3 * cell + 2];
            }
            v = dc[4 * m + 1] - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
#pragma unroll
            for (int s = 0; s < 3; ++s) v -= shifted_legendre(s, x) * hs[12 + s];
            v /= D;
        }
        dgeo[small + blk * DG_COLS + m] = v;
    }
}

// The basic-angle offset of each short interval (day) j (Sect. 3.4,
// eq:DeltaGamma): the mean over the n_ccd AF CCDs of the preceding field of
// view's AL constant term minus the following one's, (1/n_ccd) sum_n sum_f
// f c_0(f, n, j), f = +1 preceding (cell 2j), -1 following (cell 2j + 1);
// the CCDs summed in order.
__global__ void k_geo_basic_angle(int64_t n_days, int32_t n_ccd, const double* __restrict__ geo,
                                  double* __restrict__ out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_days;
         j += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t n = 0; n < n_ccd; ++n)
            s += geo[3 * ((2 * j) * n_ccd + n)] - geo[3 * ((2 * j + 1) * n_ccd + n)];
        out[j] = s / (double)n_ccd;
    }
}

inline unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

#define HIPCHK(expr)                                            \
    do {                                                        \
        int rc_ = hip_check(ctx, (expr), #expr);                \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

#define ALLOC(p, n, what)                                       \
    do {                                                        \
        int rc_ = dalloc(ctx, &(p), (size_t)(n), what);         \
        if (rc_ != AGIS_OK) return rc_;                         \
    } while (0)

void launch_geo_eta(agis_ctx* ctx) {
    if (ctx->geo_ccds <= 0 || ctx->n_obs == 0) return;
    const int32_t n_al = (int32_t)(ctx->n_cells * ctx->geo_ccds);
    const int64_t small = 3 * ctx->n_groups;
    k_geo_eta<<<grid_for(ctx->n_obs), 256, 0, ctx->stream>>>(ctx->n_obs, ctx->t_eta0, ctx->t_geo_g, ctx->t_geo_mu,
                                                             ctx->geo, n_al, ctx->geo_ccds, ctx->geo_small_days,
                                                             small, ctx->t_eta);
    k_geo_eta<<<grid_for(ctx->n_obs), 256, 0, ctx->stream>>>(ctx->n_obs, ctx->s_eta0, ctx->s_geo_g, ctx->s_geo_mu,
                                                             ctx->geo, n_al, ctx->geo_ccds, ctx->geo_small_days,
                                                             small, ctx->s_eta);
}

void launch_geo_basic_angle(agis_ctx* ctx, double* out) {
    const int64_t n_days = ctx->n_cells / 2;
    if (ctx->geo_ccds <= 0 || n_days == 0) return;
    k_geo_basic_angle<<<grid_for(n_days), 256, 0, ctx->stream>>>(n_days, ctx->geo_ccds, ctx->geo, out);
}

void launch_geo_solve(agis_ctx* ctx) {
    if (ctx->geo_ccds <= 0 || ctx->n_groups == 0) return;
    k_geo_sums<<<(unsigned)ctx->n_groups, GEO_NT, 0, ctx->stream>>>(ctx->n_groups, ctx->geo_off, ctx->geo_mu_g,
                                                                    ctx->geo_wr, ctx->geo_sums);
    const int64_t n_days = ctx->n_cells / 2;
    const bool small = ctx->geo_small_days > 0;
    if (small) {
        // the AL groups with the small-scale values, by block (eq:cc2 inside)
        const int64_t n_al = ctx->n_cells * ctx->geo_ccds, n_blk = ctx->n_small / DG_COLS;
        k_dg_colsums<<<grid_for(n_al * DG_COLS * DG_LPC), 256, 0, ctx->stream>>>(n_al, ctx->geo_coff, ctx->geo_mu_g,
                                                                                ctx->geo_wr, ctx->geo_colsum);
        k_dg_colred<<<grid_for(n_blk * DG_COLS), 256, 0, ctx->stream>>>(n_blk, ctx->geo_ccds, ctx->geo_small_days,
                                                                       ctx->n_cells, ctx->geo_colsum, ctx->geo_dcol);
        k_dg_accum<<<(unsigned)(n_blk * DG_PARTS), DG_NT, 0, ctx->stream>>>(
            ctx->geo_ccds, ctx->geo_small_days, ctx->n_cells, ctx->geo_colsum, ctx->geo_dcol, ctx->geo_zpart);
        k_dg_block<<<(unsigned)n_blk, DG_NT, dg_lds_bytes(3 * 2 * ctx->geo_small_days), ctx->stream>>>(
            ctx->geo_ccds, ctx->geo_small_days, ctx->n_cells, ctx->geo_off, ctx->geo_colsum, ctx->geo_dcol,
            ctx->geo_zpart, ctx->geo_sums, 3 * ctx->n_groups, ctx->dgeo);
    }
    k_geo_solve<<<grid_for(n_days), 256, 0, ctx->stream>>>(n_days, 0, 2 * ctx->geo_ccds, !small, ctx->geo_sums,
                                                           ctx->dgeo);
    if (ctx->geo_ac_cells > 0)
        k_geo_solve<<<grid_for(ctx->geo_ac_cells), 256, 0, ctx->stream>>>(
            ctx->geo_ac_cells, ctx->n_cells * ctx->geo_ccds, ctx->geo_ccds, true, ctx->geo_sums, ctx->dgeo);
}

// The group order of the records with a group (time order within a group,
// or with the small-scale term column then time order): geo_pos, geo_mu_g,
// geo_off (and geo_coff) from the time-order groups t_geo_g.
static int build_group_order(agis_ctx* ctx) {
    const int64_t n = ctx->n_obs, ng = ctx->n_groups;
    const int shift = ctx->geo_small_days > 0 ? DG_SHIFT : 0;
    hipStream_t st = ctx->stream;
    uint32_t *k_in = nullptr, *k_out = nullptr;
    int32_t *v_in = nullptr, *v_out = nullptr;
    uint8_t* temp = nullptr;
    auto done = [&](int rc) {
        dfree(k_in);
        dfree(k_out);
        dfree(v_in);
        dfree(v_out);
        dfree(temp);
        return rc;
    };
    int rc;
    if ((rc = dalloc(ctx, &k_in, (size_t)n, "group order keys")) || (rc = dalloc(ctx, &k_out, (size_t)n, "group order keys")) ||
        (rc = dalloc(ctx, &v_in, (size_t)n, "group order")) || (rc = dalloc(ctx, &v_out, (size_t)n, "group order")))
        return done(rc);
    const int end_bit = 32 - __builtin_clz((unsigned)ng << shift);       // keys 0..ng << shift
    size_t tb = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k_in, k_out, v_in, v_out, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return done(hip_check(ctx, e, "group order sort"));
    if ((rc = dalloc(ctx, &temp, tb, "group order sort"))) return done(rc);
    k_geo_keys<<<grid_for(n), 256, 0, st>>>(n, ctx->t_geo_g, ctx->t_geo_mu, (int32_t)ng, shift, k_in, v_in);
    e = hipcub::DeviceRadixSort::SortPairs(temp, tb, k_in, k_out, v_in, v_out, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return done(hip_check(ctx, e, "group order sort"));
    k_geo_order<<<grid_for(n), 256, 0, st>>>(n, k_out, v_out, (uint32_t)ng << shift, ctx->t_geo_mu, ctx->geo_pos,
                                             ctx->geo_mu_g);
    k_geo_offsets<<<grid_for(ng + 1), 256, 0, st>>>(n, k_out, ng + 1, shift, ctx->geo_off);
    if (shift)
        k_geo_col_offsets<<<grid_for(ctx->n_cells * ctx->geo_ccds * (DG_COLS + 1)), 256, 0, st>>>(
            n, k_out, ctx->n_cells * ctx->geo_ccds, ctx->geo_coff);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);       // before the temporaries go
    return done(e == hipSuccess ? AGIS_OK : hip_check(ctx, e, "group order"));
}

int load_geometry(agis_ctx* ctx, const int8_t* ccd, const float* mu, int32_t n_ccd, const int32_t* ac_cell,
                  int32_t n_ac_cells, int32_t small_days, int where) {
    const int64_t n = ctx->n_obs;
    hipStream_t st = ctx->stream;
    const int8_t* ccd_d = ccd;
    const float* mu_d = mu;
    const int32_t* ac_d = n_ac_cells > 0 ? ac_cell : nullptr;
    int8_t* ccd_tmp = nullptr;
    float* mu_tmp = nullptr;
    int32_t* ac_tmp = nullptr;
    auto release = [&]() {
        if (ccd_tmp) (void)hipFree(ccd_tmp);
        if (mu_tmp) (void)hipFree(mu_tmp);
        if (ac_tmp) (void)hipFree(ac_tmp);
    };
    if (where == AGIS_HOST && n > 0) {
        int rc = dalloc(ctx, &ccd_tmp, (size_t)n, "geometry ccd");
        if (rc == AGIS_OK) rc = dalloc(ctx, &mu_tmp, (size_t)n, "geometry mu");
        if (rc == AGIS_OK && ac_d) rc = dalloc(ctx, &ac_tmp, (size_t)n, "geometry AC cells");
        if (rc != AGIS_OK) {
            release();
            return rc;
        }
        hipError_t e = hipMemcpyAsync(ccd_tmp, ccd, n * sizeof(int8_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(mu_tmp, mu, n * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && ac_d) e = hipMemcpyAsync(ac_tmp, ac_cell, n * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            release();
            return hip_check(ctx, e, "geometry upload");
        }
        ccd_d = ccd_tmp;
        mu_d = mu_tmp;
        if (ac_d) ac_d = ac_tmp;
    }
    const int32_t n_ac = ac_d ? n_ac_cells : 0;
    const int64_t ng = (ctx->n_cells + n_ac) * n_ccd;
    if (ng >= INT32_MAX || n > INT32_MAX) {
        release();
        return set_error(ctx, AGIS_E_INVALID_ARG, "agis_load_geometry: more than 2^31 - 1 records or groups");
    }
    // the small-scale term: blocks of 2 small_days cells, the group-order
    // keys with 11 column bits, the block solve's LDS
    const int64_t n_al = ctx->n_cells * n_ccd;
    const int64_t n_k = small_days > 0 ? (ctx->n_cells / 2 + small_days - 1) / small_days : 0;
    const int64_t n_small = n_k * n_ccd * DG_COLS;
    if (small_days > 0) {
        int dev = 0, lds_max = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const size_t lds = dg_lds_bytes(6 * small_days);
        std::string m;
        if (6 * small_days > DG_NE_MAX) m = "small-scale long interval above 30 days";
        else if (((ng + 1) << DG_SHIFT) > (int64_t)UINT32_MAX) m = "more than 2^21 - 1 groups with the small-scale term";
        else if ((int64_t)lds > (int64_t)lds_max) m = "the small-scale block solve does not fit the device's LDS";
        if (!m.empty()) {
            release();
            return set_error(ctx, AGIS_E_INVALID_ARG, "agis_load_geometry: " + m);
        }
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dg_block),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            release();
            return hip_check(ctx, e, "small-scale block solve LDS");
        }
    }
    auto fail = [&](int rc) {
        release();
        return rc;
    };
    int rc = AGIS_OK;
#define GALLOC(p, cnt, what)                                                 \
    if (!(p) && (rc = dalloc(ctx, &(p), (size_t)std::max<int64_t>(cnt, 1), what)) != AGIS_OK) return fail(rc)
    GALLOC(ctx->t_geo_g, n, "geometry groups");
    GALLOC(ctx->s_geo_g, n, "geometry groups");
    GALLOC(ctx->t_geo_mu, n, "geometry mu");
    GALLOC(ctx->s_geo_mu, n, "geometry mu");
    GALLOC(ctx->t_eta0, n, "observed eta");
    GALLOC(ctx->s_eta0, n, "observed eta");
    GALLOC(ctx->geo_wr, 2 * n, "geometry weights");
    GALLOC(ctx->geo_pos, n, "group order");
    GALLOC(ctx->geo_mu_g, n, "group order mu");
    GALLOC(ctx->geo_flags, 1, "geometry flags");
#undef GALLOC
    const int64_t n_coef = 3 * ng + n_small;
    if (ctx->geo_ccds != n_ccd || ctx->geo_ac_cells != n_ac || ctx->geo_small_days != small_days || !ctx->geo) {
        dfree(ctx->geo);
        dfree(ctx->dgeo);
        dfree(ctx->geo_sums);
        dfree(ctx->geo_off);
        dfree(ctx->geo_coff);
        dfree(ctx->geo_colsum);
        dfree(ctx->geo_dcol);
        dfree(ctx->geo_zpart);
        if ((rc = dalloc(ctx, &ctx->geo, (size_t)std::max<int64_t>(n_coef, 1), "geometric calibration")) ||
            (rc = dalloc(ctx, &ctx->dgeo, (size_t)std::max<int64_t>(n_coef, 1), "geometric update")) ||
            (rc = dalloc(ctx, &ctx->geo_sums, (size_t)std::max<int64_t>(9 * ng, 1), "geometric sums")) ||
            (rc = dalloc(ctx, &ctx->geo_off, (size_t)(ng + 1), "group offsets")))
            return fail(rc);
        if (small_days > 0 &&
            ((rc = dalloc(ctx, &ctx->geo_coff, (size_t)(n_al * (DG_COLS + 1)), "column offsets")) ||
             (rc = dalloc(ctx, &ctx->geo_colsum, (size_t)(4 * n_al * DG_COLS), "column sums")) ||
             (rc = dalloc(ctx, &ctx->geo_dcol, (size_t)(4 * n_small), "small-scale diagonal")) ||
             (rc = dalloc(ctx, &ctx->geo_zpart, (size_t)(n_small / DG_COLS * DG_PARTS * DG_PACK),
                          "small-scale partial sums"))))
            return fail(rc);
    }
    hipError_t e = hipMemsetAsync(ctx->geo_flags, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->geo, 0, std::max<int64_t>(n_coef, 1) * sizeof(double), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->dgeo, 0, std::max<int64_t>(n_coef, 1) * sizeof(double), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->geo_off, 0, (ng + 1) * sizeof(int64_t), st);
    if (e != hipSuccess) return fail(hip_check(ctx, e, "geometry clear"));
    if (n > 0) {
        k_geo_index<<<grid_for(n), 256, 0, st>>>(n, ctx->t_perm, ctx->t_cellfov, (int32_t)ctx->n_cells, ccd_d, mu_d,
                                                  ac_d, n_ac, n_ccd, ctx->t_geo_g, ctx->t_geo_mu, ctx->geo_flags);
        k_geo_gather<int32_t><<<grid_for(n), 256, 0, st>>>(n, ctx->s_from_t, ctx->t_geo_g, ctx->s_geo_g);
        k_geo_gather<float><<<grid_for(n), 256, 0, st>>>(n, ctx->s_from_t, ctx->t_geo_mu, ctx->s_geo_mu);
    }
    e = hipGetLastError();
    int flags = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, ctx->geo_flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess) return hip_check(ctx, e, "geometry load");
    if (flags) {
        // the group columns now hold the rejected input: back to the cell
        // offsets (held at zero) and the observed angles as loaded
        if (ctx->geo_ccds > 0 && n > 0) {
            HIPCHK(hipMemcpyAsync(ctx->t_eta, ctx->t_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(ctx->s_eta, ctx->s_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        ctx->geo_ccds = 0;
        ctx->geo_ac_cells = 0;
        ctx->geo_small_days = 0;
        ctx->n_small = 0;
        ctx->n_groups = 0;
        std::string m = "agis_load_geometry:";
        if (flags & 1) m += " ccd index outside [0, n_ccd);";
        if (flags & 2) m += " across-scan pixel coordinate outside [13.5, 1979.5];";
        if (flags & 4) m += " AC calibration cell outside [0, n_ac_cells);";
        return set_error(ctx, AGIS_E_INVALID_ARG, m);
    }
    // the observed angles as loaded (the first load of the geometry keeps
    // them; a later one keeps the copies it already holds)
    if (ctx->geo_ccds == 0 && n > 0) {
        HIPCHK(hipMemcpyAsync(ctx->t_eta0, ctx->t_eta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->s_eta0, ctx->s_eta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    ctx->geo_ccds = n_ccd;
    ctx->geo_ac_cells = n_ac;
    ctx->geo_small_days = small_days;
    ctx->n_small = n_small;
    ctx->n_groups = ng;
    if (n > 0 && (rc = build_group_order(ctx)) != AGIS_OK) {
        // back to the cell offsets and the observed angles as loaded
        (void)hipMemcpyAsync(ctx->t_eta, ctx->t_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(ctx->s_eta, ctx->s_eta0, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        (void)hipStreamSynchronize(st);
        ctx->geo_ccds = 0;
        ctx->geo_ac_cells = 0;
        ctx->geo_small_days = 0;
        ctx->n_small = 0;
        ctx->n_groups = 0;
        return rc;
    }
    // the per-cell offsets are replaced by the geometric terms
    HIPCHK(hipMemsetAsync(ctx->c, 0, (ctx->n_cells + 1) * sizeof(double), st));
    launch_geo_eta(ctx);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return AGIS_OK;
}

#undef HIPCHK
#undef ALLOC

}  // namespace agis
