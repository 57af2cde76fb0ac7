// The three kernels that carry the iteration's cost.
//
//   k_source_update<G>  S block (Sect. 5.1).  G lanes per source stream the
//                       source's observations (by-source store), evaluate the
//                       model and the design row (Sect. 5.1.3) and accumulate
//                       the 15 + 5 sums of eq:normS in registers; a butterfly
//                       over the G lanes reduces them; one lane per source
//                       runs Algorithms C1-C3 on the 5x5 system and applies
//                       the update.
//   k_ac_pass           A/C accumulation (Sect. 5.2.1, 5.2.4, 5.3).  One
//                       wavefront per knot interval streams the time-ordered
//                       store at (s^(k+1), a^(k), c^(k)) and sums, on the FP64
//                       matrix cores, the 10 block pairs x 10 unique entries
//                       of eq:normAmod, its 16 right-hand-side entries and the
//                       per-fov calibration sums of eq:normC.
//   k_band_solve        A solve (Sect. 5.2.2, App. C): one 16-lane row of a
//                       wavefront per segment; right-looking modified band
//                       Cholesky (Algorithm C1 with C2 folded in) over a
//                       register window of 16 rows x 16 band offsets, rows
//                       entering from the per-interval sums in an LDS ring;
//                       then C3; the segment keeps its selected coefficients.
//
// Each lane walks its item's observations with stride G and loads the next
// observation's columns while the current one is evaluated.  No global
// atomics; all sums have a fixed order.
#include <type_traits>

#include "agis_internal.h"
#include "source_block.h"

namespace agis {

namespace {

// pair index of (n, m), 0 <= n <= m <= 3 (also the entry index of (r, c))
__host__ __device__ __forceinline__ int tri4(int n, int m) { return n * 4 - (n * (n - 1)) / 2 + (m - n); }


// ------------------------------------------------------------------ S block
// Compensated (Kahan) single-precision running sum: s + (-c) carries the sum.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// AC: the observations may include across-scan ones (cell/fov code from
// k.ac_cf0 on); the along-scan-only instance is the plain pass.  SigT: the
// type of the sigma column (float: the input; double: the frozen sigma_eff
// of the hybrid scheme).
template <int G, bool MIXED, bool AC, typename SigT, bool DEFL = false>
__global__ __launch_bounds__(256, 2) void k_source_update(DevConsts k, int64_t n_src, const int64_t* __restrict__ off,
                                                       const double* __restrict__ ot, const double* __restrict__ oeta,
                                                       const SigT* __restrict__ osig,
                                                       const int32_t* __restrict__ ocell,
                                                       const int32_t* __restrict__ oell,
                                                       const double* __restrict__ knots,
                                                       const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                       const double* __restrict__ c, double* __restrict__ s,
                                                       SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                       double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                       double* __restrict__ svar, const int32_t* __restrict__ order,
                                                       double* __restrict__ rhs) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    // group k takes the k-th source of the launch order
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = kg < n_src;
    const int64_t i = valid ? order[kg] : 0;
    double alpha = 0.0, delta = 0.0, plx = 0.0, pma = 0.0, pmd = 0.0;
    int64_t l0 = 0, l1 = 0;
    if (valid) {
        const double* si = s + 5 * i;
        alpha = si[0];
        delta = si[1];
        plx = si[2];
        pma = si[3];
        pmd = si[4];
        l0 = off[i];
        l1 = off[i + 1];
    }
    double sa, ca, sd, cd;
    sincos(alpha, &sa, &ca);
    sincos(delta, &sd, &cd);
    const double p[3] = {-sa, ca, 0.0};
    const double q[3] = {-sd * ca, -sd * sa, cd};
    const double r[3] = {cd * ca, cd * sa, sd};
    double mu[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) mu[cc] = p[cc] * pma + q[cc] * pmd;

    double acc[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) acc[e] = 0.0;
    // mixed precision: the 15 normal-matrix sums from single-precision
    // partials with compensation; the right-hand side and h'Wh stay FP64,
    // so the iteration's fixed point is the FP64 one (the FP32 matrix only
    // changes the path to it)
    float fs[MIXED ? 15 : 1], fc[MIXED ? 15 : 1];
#pragma unroll
    for (int e = 0; e < (MIXED ? 15 : 1); ++e) fs[e] = fc[e] = 0.0f;
    int64_t l = l0 + gl;
    // Current observation: columns, and the gathered attitude coefficients,
    // interval table entry and calibration of its cell.  The next
    // observation's columns load at the top of an iteration, its gathers
    // after the current observation has been evaluated.
    double t_c = 0.0, e_c = 0.0, cal_c = 0.0;
    SigT s_c = 1;
    int32_t ell_c = 3;
    bool ac_c = false;
    double a_c[16];
    KnotTab kt_c = {0.0, 1.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 16; ++e) a_c[e] = 0.0;
    if (l < l1) {
        t_c = ot[l];
        e_c = oeta[l];
        s_c = osig[l];
        ell_c = oell[l];
        const int32_t cf = ocell[l];
        cal_c = c[cf >> 1];
        ac_c = AC && cf >= k.ac_cf0;
        const double* a4 = a + 4 * (ell_c - 3);
#pragma unroll
        for (int e = 0; e < 16; ++e) a_c[e] = a4[e];
        kt_c = ktab[ell_c - 3];
    }
    for (; l < l1; l += G) {
        const int64_t ln = l + G;
        const bool more = ln < l1;
        double t_n = 0.0, e_n = 0.0;
        SigT s_n = 1;
        int32_t c_n = 0, ell_n = 3;
        if (more) {
            t_n = ot[ln];
            e_n = oeta[ln];
            s_n = osig[ln];
            c_n = ocell[ln];
            ell_n = oell[ln];
        }
        ObsEval o;
        observe<DEFL>(k, t_c, e_c, cal_c, r, mu, plx, a_c, knots + (ell_c - 2), kt_c, o, ac_c);
        double A[5];
        source_partials(o, p, q, r, A, ac_c);
        const double sg = (double)s_c;
        const double W = rcp_nr(sg * sg);
        if constexpr (MIXED) {
            float Af[5];
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) Af[rr] = (float)A[rr];
            const float Wf = (float)W;
            int e = 0;
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) {
                const float wa = Wf * Af[rr];
#pragma unroll
                for (int cc = rr; cc < 5; ++cc) {
                    kahan_add(fs[e], fc[e], wa * Af[cc]);
                    ++e;
                }
            }
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) acc[15 + rr] += W * A[rr] * o.R;
            acc[20] += W * o.R * o.R;
        } else {
            int e = 0;
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) {
                const double wa = W * A[rr];
#pragma unroll
                for (int cc = rr; cc < 5; ++cc) acc[e++] += wa * A[cc];
            }
#pragma unroll
            for (int rr = 0; rr < 5; ++rr) acc[15 + rr] += W * A[rr] * o.R;
            acc[20] += W * o.R * o.R;
        }
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        ell_c = ell_n;
        if (more) {
            cal_c = c[c_n >> 1];
            ac_c = AC && c_n >= k.ac_cf0;
            const double* a4 = a + 4 * (ell_n - 3);
#pragma unroll
            for (int e2 = 0; e2 < 16; ++e2) a_c[e2] = a4[e2];
            kt_c = ktab[ell_n - 3];
        }
    }
    if constexpr (MIXED) {
#pragma unroll
        for (int e = 0; e < 15; ++e) acc[e] = (double)fs[e] - (double)fc[e];
    }
#pragma unroll
    for (int e = 0; e < 21; ++e) acc[e] = group_sum<G>(acc[e]);
    if (!valid || gl != 0) return;
    source_finish(acc, i, alpha, delta, plx, pma, pmd, cd, s, prep, ds, qsrc, sdef, svar, rhs);
}

// ------------------------------------------------------------- A/C pass
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int AC_WAVES = 1;             // wavefronts per block, one knot interval each (2 and 4 measured 4% and 7% slower)
constexpr int AC_XS = 33;               // LDS row stride (doubles) of the transposition buffer

// A/C accumulation as a matrix product on the FP64 matrix cores.  Every
// observation of knot interval j gives two 16-vectors
//   a = (B_n B_m for the 10 pairs n <= m, B_0..B_3, [fov +1], [fov -1])
//   b = (10 unique entries of W (g g' + 4 lambda^2 q q'),
//        -W (g R - 2 lambda^2 q D) (4), W, W R)
// and the interval's sums are blocks of C = sum over observations of a b'
// (16 x 16): pairs x entries (eq:normAmod), B_n x right-hand side, and
// fov x (W, W R) for eq:normC.  One wavefront takes 64 observations at a
// time (one per lane), writes (a, b) to LDS and feeds them to 16
// v_mfma_f64_16x16x4 steps, four observations each.
//
// Mixed precision (MIXED): the model stays FP64; a and b are formed in FP32
// from single-precision partials, each 64-observation chunk is summed by
// v_mfma_f32_16x16x4 and the chunk sums enter compensated (Kahan) FP32
// running sums, converted to FP64 for the band solve.
// AC: across-scan observations present (cell/fov code from k.ac_cf0 on):
// their rows carry the AC attitude partials and no calibration entries.
template <bool MIXED, bool AC, typename SigT, bool DEFL = false>
__global__ __launch_bounds__(64 * AC_WAVES) void k_ac_pass(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                           const double* __restrict__ ot,
                                                           const double* __restrict__ oeta,
                                                           const SigT* __restrict__ osig,
                                                           const int32_t* __restrict__ ocellfov,
                                                           const int32_t* __restrict__ osrc,
                                                           const SrcPrep* __restrict__ prep,
                                                           const double* __restrict__ knots,
                                                           const KnotTab* __restrict__ ktab,
                                                           const double* __restrict__ a,
                                                           const double* __restrict__ c,
                                                           const double* __restrict__ eps_a2, int eps_bucket,
                                                           int robust, double* __restrict__ iv_sums,
                                                           double* __restrict__ iv_cal, double* __restrict__ wr_out,
                                                           const int32_t* __restrict__ wr_pos) {
    using XT = typename std::conditional<MIXED, float, double>::type;
    __shared__ XT xb[AC_WAVES][64][AC_XS];
    __shared__ double sh_a[AC_WAVES][16];
    __shared__ double sh_k[AC_WAVES][6];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * AC_WAVES + wv;
    const bool valid = j < K;
    if (lane < 22) {
        double v = 0.0;
        if (valid) v = lane < 16 ? a[4 * j + lane] : knots[j + 1 + (lane - 16)];
        if (lane < 16) sh_a[wv][lane] = v;
        else sh_k[wv][lane - 16] = v;
    }
    __syncthreads();
    const double lam2 = k.lam2;
    const int64_t l0 = valid ? iv_off[j] : 0, l1 = valid ? iv_off[j + 1] : 0;
    const KnotTab kt = valid ? ktab[j] : KnotTab{0.0, 1.0, 0.0, 0.0};
    // robust: sigma~^2 = sigma^2 + eps_a^2 of the record's component in the
    // interval's bucket (eq:W)
    XT (*xw)[AC_XS] = xb[wv];
    const int ri = lane & 15, rk = lane >> 4;
    double4_t C = {0.0, 0.0, 0.0, 0.0};
    float4_t Cs = {0.0f, 0.0f, 0.0f, 0.0f}, Cc = {0.0f, 0.0f, 0.0f, 0.0f};
    // mixed precision: the right-hand sides (B_n times the 4 attitude
    // right-hand sides, and W, WR per field of view) are summed per lane in
    // FP64 and reduced over the wavefront at the end, so the fixed point of
    // the iteration is the FP64 one
    double rb[MIXED ? 16 : 1], cb[MIXED ? 4 : 1];
#pragma unroll
    for (int e = 0; e < (MIXED ? 16 : 1); ++e) rb[e] = 0.0;
#pragma unroll
    for (int e = 0; e < (MIXED ? 4 : 1); ++e) cb[e] = 0.0;
    // lanes past the end evaluate the interval's last observation again with
    // weight zero
    int64_t base = l0;
    double t_c = 0.0, e_c = 0.0;
    SigT s_c = 1;
    int32_t cf_c = 0;
    bool h_c = false;
    SrcPrep sp_c = {};
    if (base < l1) {
        h_c = base + lane < l1;
        const int64_t le = h_c ? base + lane : l1 - 1;
        t_c = ot[le];
        e_c = oeta[le];
        s_c = osig[le];
        cf_c = ocellfov[le];
        sp_c = prep[osrc[le]];
    }
    for (; base < l1; base += 64) {
        const int64_t bn = base + 64;
        double t_n = 0.0, e_n = 0.0;
        SigT s_n = 1;
        int32_t cf_n = 0, src_n = 0;
        bool h_n = false;
        if (bn < l1) {
            h_n = bn + lane < l1;
            const int64_t le = h_n ? bn + lane : l1 - 1;
            t_n = ot[le];
            e_n = oeta[le];
            s_n = osig[le];
            cf_n = ocellfov[le];
            src_n = osrc[le];
        }
        {
            const bool ac = AC && cf_c >= k.ac_cf0;
            ObsEval o;
            observe<DEFL>(k, t_c, e_c, c[cf_c >> 1], sp_c.r, sp_c.mu, sp_c.plx, sh_a[wv], sh_k[wv], kt, o, ac);
            double g[4];
            attitude_partial(o, g, ac);
            const double sg = (double)s_c;
            double W;
            if (robust) {
                // robust mode 2: plus the source's excess noise eps_i^2 (eq:W)
                const double s2 = sg * sg + eps_a2[eps_slot(k, cf_c, j, eps_bucket)] + (robust == 2 ? sp_c.pad : 0.0);
                W = h_c ? down_weight(o.R / sqrt(s2)) / s2 : 0.0;
            } else {
                W = h_c ? rcp_nr(sg * sg) : 0.0;
            }
            // geometric calibration: each along-scan record's W and W R for
            // its C block, at its place in the group order
            if (wr_out && h_c) {
                const int32_t p = wr_pos[base + lane];
                if (p >= 0) {
                    wr_out[2 * (int64_t)p] = W;
                    wr_out[2 * (int64_t)p + 1] = W * o.R;
                }
            }
            XT* row = xw[lane];
            const int f = cf_c & 1;
            if constexpr (MIXED) {
                float B[4], gf[4], qf[4];
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    B[n] = (float)o.B[n];
                    gf[n] = (float)g[n];
                    qf[n] = (float)o.qraw[n];
                }
                const float Wf = (float)W, Rf = (float)o.R, Df = (float)o.D, l2 = (float)lam2;
                int e = 0;
#pragma unroll
                for (int n = 0; n < 4; ++n)
#pragma unroll
                    for (int m = n; m < 4; ++m) row[e++] = B[n] * B[m];
#pragma unroll
                for (int n = 0; n < 4; ++n) row[10 + n] = B[n];
                row[14] = (f == 0 && !ac) ? 1.0f : 0.0f;
                row[15] = (f == 1 && !ac) ? 1.0f : 0.0f;
                e = 0;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int cc = rr; cc < 4; ++cc) row[16 + e++] = Wf * (gf[rr] * gf[cc] + 4.0f * l2 * qf[rr] * qf[cc]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) row[26 + rr] = -Wf * (gf[rr] * Rf - 2.0f * l2 * qf[rr] * Df);
                row[30] = Wf;
                row[31] = Wf * Rf;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const double rhs = -W * (g[rr] * o.R - 2.0 * lam2 * o.qraw[rr] * o.D);
#pragma unroll
                    for (int n = 0; n < 4; ++n) rb[4 * n + rr] += o.B[n] * rhs;
                }
                if (!ac) {
                    cb[2 * f] += W;
                    cb[2 * f + 1] += W * o.R;
                }
            } else {
                int e = 0;
#pragma unroll
                for (int n = 0; n < 4; ++n)
#pragma unroll
                    for (int m = n; m < 4; ++m) row[e++] = o.B[n] * o.B[m];
#pragma unroll
                for (int n = 0; n < 4; ++n) row[10 + n] = o.B[n];
                row[14] = (f == 0 && !ac) ? 1.0 : 0.0;
                row[15] = (f == 1 && !ac) ? 1.0 : 0.0;
                e = 0;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int cc = rr; cc < 4; ++cc)
                        row[16 + e++] = W * (g[rr] * g[cc] + 4.0 * lam2 * o.qraw[rr] * o.qraw[cc]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) row[26 + rr] = -W * (g[rr] * o.R - 2.0 * lam2 * o.qraw[rr] * o.D);
                row[30] = W;
                row[31] = W * o.R;
            }
        }
        SrcPrep sp_n = {};
        if (bn < l1) sp_n = prep[src_n];
        // the rows just written are read back below by other lanes: a
        // workgroup barrier (the block is one wavefront, so it reduces to
        // waiting for the LDS stores) orders the stores before the reads
        __syncthreads();
        // groups of four observations past the interval's end hold padding
        // rows of weight zero: their matrix-core steps would add zeros
        const int64_t n_here = l1 - base < 64 ? l1 - base : 64;
        const int steps = (int)((n_here + 3) >> 2);
        if constexpr (MIXED) {
            float4_t Ck = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                if (kk >= steps) break;
                const float av = xw[4 * kk + rk][ri];
                const float bv = xw[4 * kk + rk][16 + ri];
                Ck = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, Ck, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float sv = Cs[v], cv = Cc[v];
                kahan_add(sv, cv, Ck[v]);
                Cs[v] = sv;
                Cc[v] = cv;
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                if (kk >= steps) break;
                const double av = xw[4 * kk + rk][ri];
                const double bv = xw[4 * kk + rk][16 + ri];
                C = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, C, 0, 0, 0);
            }
        }
        // the next chunk's stores overwrite these rows: every lane's reads
        // above come first
        __syncthreads();
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        cf_c = cf_n;
        h_c = h_n;
        sp_c = sp_n;
    }
    if (!valid) return;
    if constexpr (MIXED) {
#pragma unroll
        for (int v = 0; v < 4; ++v) C[v] = (double)Cs[v] - (double)Cc[v];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
            for (int e = 0; e < 16; ++e) rb[e] += __shfl_xor(rb[e], m, 64);
#pragma unroll
            for (int e = 0; e < 4; ++e) cb[e] += __shfl_xor(cb[e], m, 64);
        }
    }
    // lane l holds C[4 v + l / 16][l % 16] (FP64 product) or
    // C[4 (l / 16) + v][l % 16] (FP32 product), v = 0..3
    double* out = iv_sums + j * IV_SUMS;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = MIXED ? 4 * rk + v : 4 * v + rk, jj = ri;
        if (i < 10 && jj < 10) out[i * 10 + jj] = C[v];
        else if (!MIXED && i >= 10 && i < 14 && jj >= 10 && jj < 14) out[100 + (i - 10) * 4 + (jj - 10)] = C[v];
        else if (!MIXED && i >= 14 && jj >= 14) iv_cal[j * IV_CAL + (i - 14) * 2 + (jj - 14)] = C[v];
    }
    if constexpr (MIXED) {
        // every lane holds the reduced FP64 sums; lane e writes entry e
#pragma unroll
        for (int e = 0; e < 16; ++e)
            if (lane == e) out[100 + e] = rb[e];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (lane == 16 + e) iv_cal[j * IV_CAL + e] = cb[e];
    }
}

// ------------------------------------------------------------ band solve
// Intervals held in LDS per segment.  The row read at step i (row i + 17)
// needs the intervals (i+17)/4 - 3 .. (i+17)/4, and interval b + 5 enters at
// the end of step 4b + 2, after that step's read, into the slot of interval
// b, which no later row needs; the start needs intervals 0..4.  Five slots
// keep four segments per block within 18.6 KB of LDS (eight blocks per CU).
constexpr int RING = 5;
constexpr int RING_W = IV_SUMS;         // doubles per interval

// Entry (i, kk) (segment-relative scalar indices, i <= kk <= i + 15) of the
// segment's band matrix from the ring of per-interval sums.
__device__ __forceinline__ double ring_entry(const double (*ring)[RING_W], int64_t nb, int64_t i, int64_t kk) {
    const int64_t bi = i >> 2, bk = kk >> 2;
    const int r = (int)(i & 3), cc = (int)(kk & 3);
    const int e = r < cc ? tri4(r, cc) : tri4(cc, r);
    const int64_t jlo = bk - 3 > 0 ? bk - 3 : 0;
    const int64_t jhi = bi < nb - 4 ? bi : nb - 4;
    double s = 0.0;
    for (int64_t j = jlo, sl = jlo % RING; j <= jhi; ++j, sl = sl + 1 == RING ? 0 : sl + 1)
        s += ring[sl][tri4((int)(bi - j), (int)(bk - j)) * 10 + e];
    return s;
}

__device__ __forceinline__ double ring_rhs(const double (*ring)[RING_W], int64_t nb, int64_t i) {
    const int64_t bi = i >> 2;
    const int r = (int)(i & 3);
    const int64_t jlo = bi - 3 > 0 ? bi - 3 : 0;
    const int64_t jhi = bi < nb - 4 ? bi : nb - 4;
    double s = 0.0;
    for (int64_t j = jlo, sl = jlo % RING; j <= jhi; ++j, sl = sl + 1 == RING ? 0 : sl + 1)
        s += ring[sl][100 + (bi - j) * 4 + r];
    return s;
}

// Value of v in another lane of the 16-lane row (DPP, both 32-bit halves):
// CTRL 0x150 + n broadcasts lane n of the row, 0x100 + n reads lane + n,
// 0x110 + n reads lane - n, 0x120 + n rotates by n; lanes with no source
// read 0.
template <int CTRL>
__device__ __forceinline__ double row_dpp(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Right-looking update of the window rows c = C..15 by pivot row i:
// lane d, row c: entry (i+c, i+c+d) -= U(i, i+c) U(i, i+c+d).
template <int C>
__device__ __forceinline__ void band_trailing(double (&W)[16], double U) {
    if constexpr (C < 16) {
        W[C] -= row_dpp<0x150 + C>(U) * row_dpp<0x100 + C>(U);
        band_trailing<C + 1>(W, U);
    }
}

constexpr int BAND_SEGS = 4;            // segments per block (one wavefront), one per 16-lane row
constexpr int PFL = (RING_W + 15) / 16; // doubles per lane to fetch one interval

// Modified band Cholesky of the attitude segments (Algorithms C1-C3 with
// half bandwidth 15, Sect. 5.2.2).  Each 16-lane row of the wavefront solves
// one segment: lane d holds band offset d of the 16 window rows i..i+15 in
// registers (W[c] = entry (i+c, i+c+d)) and the right-hand side of row i+d.
// Step i takes the pivot from lane 0, forms U(i, i+d) in lane d, updates the
// window through row broadcasts and shifts, retires row i and lets row i+16
// enter from the per-interval sums (an LDS ring, each interval prefetched
// two coefficient blocks ahead).  A zero or negative pivot gives a zero
// factor row and counts one defect.  C3 then runs back up the segment with
// x(i+d) in lane d and a row reduction per step.
__global__ __launch_bounds__(16 * BAND_SEGS) void k_band_solve(int64_t nseg, const SegDesc* __restrict__ segs,
                                                   const double* __restrict__ iv_sums, double* __restrict__ ufac,
                                                   double* __restrict__ yfac, double* __restrict__ da,
                                                   int32_t* __restrict__ seg_def) {
    __shared__ double ring_all[BAND_SEGS][RING][RING_W];
    const int d = threadIdx.x & 15;
    const int sl = threadIdx.x >> 4;
    const int64_t sgi = (int64_t)blockIdx.x * BAND_SEGS + sl;
    const bool valid = sgi < nseg;
    double (*ring)[RING_W] = ring_all[sl];
    SegDesc sd = {0, -1, 0, -1, 0};
    if (valid) sd = segs[sgi];
    const int64_t nb = sd.n_hi - sd.n_lo + 1;
    const int64_t nu = valid ? 4 * nb : 0;
    const int64_t n_iv = valid ? nb - 3 : 0;
    int64_t nu_max = 0;
    for (int s2 = 0; s2 < BAND_SEGS; ++s2) {
        const int64_t g = (int64_t)blockIdx.x * BAND_SEGS + s2;
        if (g < nseg) {
            const SegDesc o = segs[g];
            const int64_t n2 = 4 * (o.n_hi - o.n_lo + 1);
            nu_max = n2 > nu_max ? n2 : nu_max;
        }
    }
    const double* sums = iv_sums + (valid ? sd.n_lo : 0) * IV_SUMS;
    double* U = ufac + sd.u_off * 16;
    double* Y = yfac + sd.u_off;
    // intervals 0..4 into the ring, interval 5 into registers
    for (int jj = 0; jj < 5; ++jj)
        if (jj < n_iv)
            for (int e = d; e < RING_W; e += 16) ring[jj][e] = sums[(int64_t)jj * IV_SUMS + e];
    double pfA[PFL], pfB[PFL];
#pragma unroll
    for (int u = 0; u < PFL; ++u) {
        const int e = d + 16 * u;
        pfA[u] = (5 < n_iv && e < RING_W) ? sums[5 * IV_SUMS + e] : 0.0;
        pfB[u] = 0.0;
    }
    __syncthreads();
    double W[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) W[c] = (c + d < nu) ? ring_entry(ring, nb, c, c + d) : 0.0;
    double R = d < nu ? ring_rhs(ring, nb, d) : 0.0;
    // row i + 16 (entering after step i) is read from the ring one step early
    double nW = (16 + d < nu) ? ring_entry(ring, nb, 16, 16 + d) : 0.0;
    double nR = (d == 15 && 16 < nu) ? ring_rhs(ring, nb, 16) : 0.0;
    int defect = 0;
    for (int64_t i = 0; i < nu_max; ++i) {
        const bool act = i < nu;
        const int64_t b = i >> 2;
        if ((i & 3) == 0 && b + 6 < n_iv) {
#pragma unroll
            for (int u = 0; u < PFL; ++u) {
                const int e = d + 16 * u;
                pfB[u] = e < RING_W ? sums[(b + 6) * IV_SUMS + e] : 0.0;
            }
        }
        const double piv = row_dpp<0x150>(W[0]);
        const bool ok = piv > 0.0;
        const double inv = ok ? rsqrt_nr(piv) : 0.0;
        const double Ud = d == 0 ? piv * inv : W[0] * inv;
        const double y = row_dpp<0x150>(R) * inv;
        band_trailing<1>(W, Ud);
        R -= Ud * y;
        R = row_dpp<0x101>(R);
        if (d == 15) R = nR;
#pragma unroll
        for (int c = 0; c < 15; ++c) W[c] = W[c + 1];
        W[15] = nW;
        if (act) {
            U[i * 16 + d] = Ud;
            if (d == 0) {
                Y[i] = y;
                defect += ok ? 0 : 1;
            }
        }
        const int64_t r = i + 17;
        nW = (r + d < nu) ? ring_entry(ring, nb, r, r + d) : 0.0;
        nR = (d == 15 && r < nu) ? ring_rhs(ring, nb, r) : 0.0;
        if ((i & 3) == 2) {
            // interval b + 5 (first read for row 4b + 20, at step 4b + 3)
            // enters the ring in the slot of interval b, which no row read
            // from step 4b + 3 on refers to
            if (b + 5 < n_iv) {
#pragma unroll
                for (int u = 0; u < PFL; ++u) {
                    const int e = d + 16 * u;
                    if (e < RING_W) ring[(int)(b + 5) % RING][e] = pfA[u];
                }
            }
#pragma unroll
            for (int u = 0; u < PFL; ++u) pfA[u] = pfB[u];
            __syncthreads();
        }
    }
    __syncthreads();   // factor rows and forward-substituted y visible to all lanes
    // Algorithm C3 from the last row up: lane d holds x(i+d), d >= 1.  Rows
    // are read 16 at a time, one chunk ahead of their use.
    double x = 0.0;
    double cU[16], cu[16], cy[16];
    auto load_rows = [&](int64_t t0, double* lU, double* lu, double* ly) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t i = nu - 1 - (t0 + k);
            lU[k] = lu[k] = ly[k] = 0.0;
            if (i >= 0) {
                lU[k] = U[i * 16 + d];
                lu[k] = U[i * 16];
                ly[k] = Y[i];
            }
        }
    };
    load_rows(0, cU, cu, cy);
    for (int64_t t0 = 0; t0 < nu_max; t0 += 16) {
        double nU[16], nu_[16], ny[16];
        load_rows(t0 + 16, nU, nu_, ny);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t i = nu - 1 - (t0 + k);
            double p = d >= 1 ? cU[k] * x : 0.0;
            p += row_dpp<0x128>(p);
            p += row_dpp<0x124>(p);
            p += row_dpp<0x122>(p);
            p += row_dpp<0x121>(p);
            const double xi = cu[k] > 0.0 ? (cy[k] - p) * rcp_nr(cu[k]) : 0.0;
            if (i >= 0 && d == 0) {
                const int64_t n = sd.n_lo + (i >> 2);
                if (n >= sd.keep_lo && n <= sd.keep_hi) da[4 * n + (i & 3)] = xi;
            }
            x = row_dpp<0x111>(d == 0 ? xi : x);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            cU[k] = nU[k];
            cu[k] = nu_[k];
            cy[k] = ny[k];
        }
    }
    if (valid && d == 0) seg_def[sgi] = defect;
}

inline int groups_grid(int64_t n_items, int items_per_block) {
    return (int)((n_items + items_per_block - 1) / items_per_block);
}

}  // namespace

#define AGIS_S_KERNEL(G, T)                                                                                    \
    (ctx->cfg.precision == AGIS_MIXED                                                                          \
         ? (ctx->has_ac ? k_source_update<G, true, true, T> : k_source_update<G, true, false, T>)               \
         : (ctx->has_ac ? k_source_update<G, false, true, T> : k_source_update<G, false, false, T>))
#define AGIS_S_ARGS(SIG)                                                                                       \
    ctx->k, ctx->n_src, ctx->src_off, ctx->s_t, ctx->s_eta, SIG, ctx->s_cell, ctx->s_ell, ctx->knots, ctx->ktab,   \
        ctx->a, ctx->c, ctx->s, ctx->prep, ctx->ds, ctx->qsrc, ctx->sdef, ctx->svar, ctx->src_order, ctx->rhs_s_out
#define AGIS_S_LAUNCH(G)                                                                                       \
    if (ctx->k.defl > 0.0)                                                                                     \
        (ctx->has_ac ? k_source_update<G, false, true, float, true> : k_source_update<G, false, false, float, true>) \
            <<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(AGIS_S_ARGS(ctx->s_sig));            \
    else if (ctx->frozen)                                                                                      \
        AGIS_S_KERNEL(G, double)<<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(                  \
            AGIS_S_ARGS(ctx->s_sig_eff));                                                                      \
    else                                                                                                       \
        AGIS_S_KERNEL(G, float)<<<groups_grid(ctx->n_src, 256 / G), 256, 0, ctx->stream>>>(AGIS_S_ARGS(ctx->s_sig))

void launch_source_update(agis_ctx* ctx) {
    if (ctx->n_src == 0) return;
    switch (ctx->s_group) {
        case 8: AGIS_S_LAUNCH(8); break;
        case 16: AGIS_S_LAUNCH(16); break;
        case 32: AGIS_S_LAUNCH(32); break;
        default: AGIS_S_LAUNCH(64); break;
    }
}

template <typename T>
static void ac_pass_with(agis_ctx* ctx, const T* sig) {
    auto kern = ctx->cfg.precision == AGIS_MIXED
                    ? (ctx->has_ac ? k_ac_pass<true, true, T> : k_ac_pass<true, false, T>)
                    : (ctx->has_ac ? k_ac_pass<false, true, T> : k_ac_pass<false, false, T>);
    if constexpr (std::is_same<T, float>::value) {
        // the model with the Sun's light deflection (FP64 only, as the
        // global block requires)
        if (ctx->k.defl > 0.0) kern = ctx->has_ac ? k_ac_pass<false, true, float, true> : k_ac_pass<false, false, float, true>;
    }
    kern<<<(unsigned)((ctx->K + AC_WAVES - 1) / AC_WAVES), 64 * AC_WAVES, 0, ctx->stream>>>(
        ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, sig, ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots,
        ctx->ktab, ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, robust_now(ctx), ctx->iv_sums, ctx->iv_cal,
        ctx->geo_ccds > 0 ? ctx->geo_wr : nullptr, ctx->geo_pos);
}

void launch_ac_pass(agis_ctx* ctx) {
    if (ctx->K == 0) return;
    if (ctx->frozen)
        ac_pass_with(ctx, ctx->t_sig_eff);
    else
        ac_pass_with(ctx, ctx->t_sig);
}

void launch_band_solve(agis_ctx* ctx) {
    const int64_t nseg = (int64_t)ctx->h_segs.size();
    if (nseg == 0) return;
    k_band_solve<<<(unsigned)((nseg + BAND_SEGS - 1) / BAND_SEGS), 16 * BAND_SEGS, 0, ctx->stream>>>(
        nseg, ctx->segs, ctx->iv_sums, ctx->ufac, ctx->yfac, ctx->da, ctx->seg_def);
}

}  // namespace agis
