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
// number of keys in the lower digits (every lane of the calling wavefront
// receives both; any wavefront of the block may call it).
__device__ __forceinline__ void radix_digit(const uint32_t* hist, int64_t k, int& digit_out, uint32_t& below_out) {
    const int lane = threadIdx.x & 63;
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

// Every element selected (the sets without a filter).
struct AllOf {
    __device__ bool operator()(int64_t) const { return true; }
};

// Elements whose cell/fov code belongs to one excess-noise component (0
// along scan, 1 across scan preceding, 2 following field of view) or, with
// kind_only, to one kind of record (0 along scan, 1 across scan).  Without
// codes (cf null) every element is along scan.
struct OfComponent {
    const int32_t* cf;
    int32_t ac_cf0;
    int comp;
    bool kind_only;
    __device__ bool operator()(int64_t i) const {
        if (!cf) return comp == 0;
        const int32_t c = cf[i];
        const int k = c >= ac_cf0 ? 1 + (c & 1) : 0;
        return kind_only ? (k > 0) == (comp > 0) : k == comp;
    }
};

// k-th smallest (0-based) of the elements i of v[0..n) with sel(i), by the
// whole 64-thread block, reading v on every pass (any n).
template <class Sel>
__device__ double block_select(const double* __restrict__ v, int64_t n, int64_t k, uint32_t* hist, Sel sel) {
    const int lane = threadIdx.x;
    uint64_t prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = lane; b < 256; b += 64) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = lane; i < n; i += 64) {
            if (!sel(i)) continue;
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

// p-quantile of the m selected elements (sel) of v[0..n) by linear
// interpolation between the order statistics at (m - 1) p (type 7); 0 for
// m = 0.
template <class Sel>
__device__ double block_quantile7(const double* __restrict__ v, int64_t n, int64_t m, double p, uint32_t* hist,
                                  Sel sel) {
    if (m <= 0) return 0.0;
    const double h = (double)(m - 1) * p;
    const int64_t j = (int64_t)floor(h);
    const double xj = block_select(v, n, j, hist, sel);
    if (j + 1 >= m) return xj;
    const double xj1 = block_select(v, n, j + 1, hist, sel);
    return xj + (h - (double)j) * (xj1 - xj);
}

// Number of the elements i of [0, n) with sel(i), summed over the 64-thread
// block (every thread receives it).
template <class Sel>
__device__ int64_t block_count(int64_t n, Sel sel) {
    int64_t c = 0;
    for (int64_t i = threadIdx.x; i < n; i += 64) c += sel(i) ? 1 : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    return c;
}

// Keys held in registers: key r of lane l is element l + 64 r (n <= 64 KR).
constexpr int KR = 32;

// Elements not selected (sel) get the largest key, above every finite
// value: they sort after the m selected ones, which the ranks address.
template <class Sel>
__device__ __forceinline__ void load_keys(const double* __restrict__ v, int64_t n, uint64_t (&kr)[KR], Sel sel) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int64_t i = lane + 64 * r;
        kr[r] = (i < n && sel(i)) ? order_key(v[i]) : ~0ull;
    }
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

// Type-7 p-quantile of the m selected keys among the n register-held ones
// (the others hold the largest key): the order statistic j by selection,
// j + 1 as the same key if more than j + 1 keys are <= it, else as the
// smallest key above it.
__device__ double reg_quantile7(const uint64_t (&kr)[KR], int64_t n, int64_t m, double p, uint32_t* hist) {
    if (m <= 0) return 0.0;
    const int lane = threadIdx.x;
    const double h = (double)(m - 1) * p;
    const int64_t j = (int64_t)floor(h);
    const uint64_t kj = reg_select(kr, n, j, hist);
    const double xj = key_value(kj);
    if (j + 1 >= m) return xj;
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

// Adds the digits dg of the lanes with in set to the histogram h: where
// every such lane of the wavefront has the same digit, one lane adds their
// count.
__device__ __forceinline__ void count_digits(uint32_t* h, uint32_t dg, bool in) {
    if (!in) return;
    const int lane = threadIdx.x & 63;
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
    const uint64_t am = __ballot(true);
    const uint64_t same = __ballot(dg == d0);
    if (same == am) {
        if (lane == __ffsll((unsigned long long)am) - 1) atomicAdd(&h[d0], (uint32_t)__popcll(am));
    } else {
        atomicAdd(&h[dg], 1u);
    }
}

// The 64 keys of a wavefront sorted ascending over its lanes (bitonic
// network; every lane of the wavefront takes part).
__device__ __forceinline__ uint64_t wave_sort64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)v, j, 64), hi = __shfl_xor((uint32_t)(v >> 32), j, 64);
            const uint64_t o = ((uint64_t)hi << 32) | lo;
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
        }
    }
    return v;
}

// Rank k among the c <= 64 register-held keys under prefix (mask): the keys
// gathered in lane order into cand (LDS, 64 keys), sorted over the
// wavefront, the k-th taken.  One wavefront.
__device__ uint64_t reg_finish_select(const uint64_t (&kr)[KR], int64_t n, int nr, uint64_t mask, uint64_t prefix,
                                      int64_t k, uint64_t* cand) {
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t base = 0;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const bool in = r < nr && lane + 64 * r < n && (kr[r] & mask) == prefix;
        const uint64_t b = __ballot(in);
        if (in) cand[base + __popcll(b & below)] = kr[r];
        base += (uint32_t)__popcll(b);
    }
    __syncthreads();
    uint64_t v = lane < (int)base ? cand[lane] : ~0ull;
    __syncthreads();
    v = wave_sort64(v);
    const uint32_t lo = __shfl((uint32_t)v, (int)k, 64), hi = __shfl((uint32_t)(v >> 32), (int)k, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Type-7 quantiles at pa and pb of the m selected keys among the n
// register-held ones (the others hold the largest key), both order
// statistics found in one set of radix passes: each pass counts the digits
// of the keys under either prefix into a histogram of its own (hist: 512
// counts); once at most 64 keys share a statistic's prefix, they are
// gathered and sorted over the wavefront and the statistic is read off
// (cand: 64 keys in LDS).  Then one sweep finds, for each, whether the next
// order statistic is the same key or the smallest key above it.
__device__ void reg_quantile7_pair(const uint64_t (&kr)[KR], int64_t n, int64_t m, double pa, double pb,
                                   uint32_t* hist, uint64_t* cand, double& qa, double& qb) {
    if (m <= 0) {
        qa = qb = 0.0;
        return;
    }
    const int lane = threadIdx.x;
    const int nr = (int)((n + 63) / 64);
    const double ha_ = (double)(m - 1) * pa, hb_ = (double)(m - 1) * pb;
    const int64_t ja = (int64_t)floor(ha_), jb = (int64_t)floor(hb_);
    int64_t ka = ja, kb = jb;
    uint64_t prea = 0, preb = 0, mask = 0;
    bool done_a = false, done_b = false;
    uint32_t* hista = hist;
    uint32_t* histb = hist + 256;
    for (int shift = 56; shift >= 0 && !(done_a && done_b); shift -= 8) {
        for (int b = lane; b < 512; b += 64) hist[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            if (r < nr && lane + 64 * r < n) {
                const uint64_t key = kr[r];
                const uint32_t dg = (uint32_t)(key >> shift) & 255u;
                count_digits(hista, dg, !done_a && (key & mask) == prea);
                count_digits(histb, dg, !done_b && (key & mask) == preb);
            }
        }
        __syncthreads();
        uint32_t ca = 65u, cb = 65u;
        if (!done_a) {
            int d;
            uint32_t bel;
            radix_digit(hista, ka, d, bel);
            prea |= (uint64_t)d << shift;
            ka -= (int64_t)bel;
            ca = hista[d];
        }
        if (!done_b) {
            int d;
            uint32_t bel;
            radix_digit(histb, kb, d, bel);
            preb |= (uint64_t)d << shift;
            kb -= (int64_t)bel;
            cb = histb[d];
        }
        mask |= 0xFFull << shift;
        __syncthreads();
        if (shift > 0 && !done_a && ca <= 64u) {
            prea = reg_finish_select(kr, n, nr, mask, prea, ka, cand);
            done_a = true;
        }
        if (shift > 0 && !done_b && cb <= 64u) {
            preb = reg_finish_select(kr, n, nr, mask, preb, kb, cand);
            done_b = true;
        }
    }
    uint32_t cla = 0, clb = 0;
    uint64_t mna = ~0ull, mnb = ~0ull;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        if (lane + 64 * r < n) {
            const uint64_t key = kr[r];
            cla += key <= prea ? 1u : 0u;
            clb += key <= preb ? 1u : 0u;
            if (key > prea && key < mna) mna = key;
            if (key > preb && key < mnb) mnb = key;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cla += __shfl_xor(cla, o, 64);
        clb += __shfl_xor(clb, o, 64);
        uint32_t lo = __shfl_xor((uint32_t)mna, o, 64), hi = __shfl_xor((uint32_t)(mna >> 32), o, 64);
        uint64_t other = ((uint64_t)hi << 32) | lo;
        mna = other < mna ? other : mna;
        lo = __shfl_xor((uint32_t)mnb, o, 64);
        hi = __shfl_xor((uint32_t)(mnb >> 32), o, 64);
        other = ((uint64_t)hi << 32) | lo;
        mnb = other < mnb ? other : mnb;
    }
    const double xa = key_value(prea), xb = key_value(preb);
    qa = ja + 1 >= m ? xa : xa + (ha_ - (double)ja) * (key_value((int64_t)cla >= ja + 2 ? prea : mna) - xa);
    qb = jb + 1 >= m ? xb : xb + (hb_ - (double)jb) * (key_value((int64_t)clb >= jb + 2 ? preb : mnb) - xb);
}

// ------------------------------------------------------------- S, pass 0
template <int G, bool DEFL = false>
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
    int64_t l = off[i] + gl;
    // Current observation with its gathers (attitude coefficients, interval
    // table entry, calibration, excess noise); the next observation's
    // columns load at the top of an iteration, its gathers after the
    // current one has been evaluated.
    double t_c = 0.0, e_c = 0.0, cal_c = 0.0, ea_c = 0.0;
    float s_c = 1.0f;
    int32_t ell_c = 3, cf_c = 0;
    double a_c[16];
    KnotTab kt_c = {0.0, 1.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 16; ++e) a_c[e] = 0.0;
    if (l < l1) {
        t_c = ot[l];
        e_c = oeta[l];
        s_c = osig[l];
        ell_c = oell[l];
        cf_c = ocell[l];
        cal_c = c[cf_c >> 1];
        ea_c = eps_a2[eps_slot(k, cf_c, ell_c - 3, eps_bucket)];
        const double* a4 = a + 4 * (ell_c - 3);
#pragma unroll
        for (int e = 0; e < 16; ++e) a_c[e] = a4[e];
        kt_c = ktab[ell_c - 3];
    }
    for (; l < l1; l += G) {
        const int64_t ln = l + G;
        const bool more = ln < l1;
        double t_n = 0.0, e_n = 0.0;
        float s_n = 1.0f;
        int32_t cf_n = 0, ell_n = 3;
        if (more) {
            t_n = ot[ln];
            e_n = oeta[ln];
            s_n = osig[ln];
            cf_n = ocell[ln];
            ell_n = oell[ln];
        }
        const bool ac = cf_c >= k.ac_cf0;
        ObsEval o;
        observe<DEFL>(k, t_c, e_c, cal_c, r, mu, plx, a_c, knots + (ell_c - 2), kt_c, o, ac);
        double A[5];
        source_partials(o, p, q, r, A, ac);
        const double sg = (double)s_c;
#pragma unroll
        for (int e = 0; e < 3; ++e) col[e * n_obs + l] = A[e];
        col[3 * n_obs + l] = o.tau;              // A[3] = A[0] tau, A[4] = A[1] tau
        col[4 * n_obs + l] = o.R;
        col[5 * n_obs + l] = sg * sg + ea_c;
        if (more) {
            const double* a4 = a + 4 * (ell_n - 3);
#pragma unroll
            for (int e = 0; e < 16; ++e) a_c[e] = a4[e];
            kt_c = ktab[ell_n - 3];
            cal_c = c[cf_n >> 1];
            ea_c = eps_a2[eps_slot(k, cf_n, ell_n - 3, eps_bucket)];
        }
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        cf_c = cf_n;
        ell_c = ell_n;
    }
}

// ------------------------------------------------ S, initial downweights
// REG: keys of sets up to reg_limit in registers (fewer wavefronts per SIMD,
// pays for large sets), the two order statistics selected one after the
// other (REG 1) or in one set of radix passes (REG 2); otherwise (REG 0)
// re-read on every pass (small sets).
// varsigma of one kind of a source's records: half the intersextile range
// of the selected (sel) h of the n; m of them are selected.
template <int REG, class Sel>
__device__ double half_intersextile(const double* __restrict__ h, int64_t n, int64_t m, int64_t reg_limit,
                                    uint32_t* hist, uint64_t* cand, Sel sel) {
    double q5, q1;
    if (REG && n <= reg_limit) {
        uint64_t kr[KR];
        load_keys(h, n, kr, sel);
        if (REG == 2) {
            reg_quantile7_pair(kr, n, m, 5.0 / 6.0, 1.0 / 6.0, hist, cand, q5, q1);
        } else {
            q5 = reg_quantile7(kr, n, m, 5.0 / 6.0, hist);
            q1 = reg_quantile7(kr, n, m, 1.0 / 6.0, hist);
        }
    } else {
        q5 = block_quantile7(h, n, m, 5.0 / 6.0, hist, sel);
        q1 = block_quantile7(h, n, m, 1.0 / 6.0, hist, sel);
    }
    return 0.5 * (q5 - q1);
}

// vs[2 i + kind]: varsigma_i of the along-scan (kind 0) and the across-scan
// (kind 1) records of source i, whose residual scales differ by the ratio of
// their formal errors.  cell: the records' cell/fov codes in source order,
// or null where every record is along scan (AC false; vs[2 i + 1] = 0 then).
template <int REG, bool AC>
__global__ __launch_bounds__(64) void k_s_sigma(int64_t n_src, const int64_t* __restrict__ off,
                                                const double* __restrict__ h, double* __restrict__ vs,
                                                int64_t reg_limit, const int32_t* __restrict__ order,
                                                const int32_t* __restrict__ cell, int32_t ac_cf0) {
    __shared__ uint32_t hist[512];
    __shared__ uint64_t cand[64];
    if ((int64_t)blockIdx.x >= n_src) return;
    const int64_t i = order[blockIdx.x];         // the largest sets first
    const int64_t l0 = off[i], n = off[i + 1] - l0;
    if (!AC) {
        const double v = half_intersextile<REG>(h + l0, n, n, reg_limit, hist, cand, AllOf{});
        if (threadIdx.x == 0) {
            vs[2 * i] = v;
            vs[2 * i + 1] = 0.0;
        }
        return;
    }
    const int32_t* cf = cell + l0;
    const int64_t m_ac = block_count(n, OfComponent{cf, ac_cf0, 1, true});
    for (int kind = 0; kind < 2; ++kind) {
        const int64_t m = kind ? m_ac : n - m_ac;
        const double v = m > 0 ? half_intersextile<REG>(h + l0, n, m, reg_limit, hist, cand,
                                                          OfComponent{cf, ac_cf0, kind, true})
                               : 0.0;
        if (threadIdx.x == 0) vs[2 * i + kind] = v;
    }
}

// Initial downweight of a record (eq:wl's first round): w(h / varsigma) of
// the record's kind; 1 where that varsigma is 0.
__device__ __forceinline__ double first_weight(double h, double vs0, double vs1, const int32_t* __restrict__ cell,
                                               int32_t ac_cf0, int64_t l) {
    const double v = (cell && cell[l] >= ac_cf0) ? vs1 : vs0;
    return v > 0.0 ? down_weight(h / v) : 1.0;
}

// ------------------------------------------------- S, inner iteration
constexpr int INNER_SOLVES = 4;

// The accumulation of one record into the 21 sums of a round: its weight
// w(h / varsigma) of its kind in the first round, w(R / sigma~) from the
// previous round's d after it (eq:dw, eq:wl, eq:W).
__device__ __forceinline__ void irls_row(double (&acc)[21], const double (&A)[5], double h, double s2, int it,
                                         const double (&d)[5], double vs0, double vs1, bool ac_row) {
    double wl;
    if (it == 0) {
        const double v = ac_row ? vs1 : vs0;
        wl = v > 0.0 ? down_weight(h / v) : 1.0;
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

// RC > 0: each lane keeps its first RC records (alpha*, delta, parallax
// entries, tau, h, sigma~^2 and the kind) in registers from the first round
// on, so the later rounds re-read only the records beyond them from the
// columns.  The sums take the records in the same order either way.
constexpr int IRLS_RC = 8;

template <int G, int RC = 0>
__global__ __launch_bounds__(256) void k_s_irls(int64_t n_src, const int64_t* __restrict__ off,
                                                const double* __restrict__ col, int64_t n_obs,
                                                const double* __restrict__ vs, double* __restrict__ s,
                                                SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                double* __restrict__ svar, const int32_t* __restrict__ order,
                                                const int32_t* __restrict__ cell, int32_t ac_cf0) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int leader = (threadIdx.x & 63) & ~(G - 1);
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = kg < n_src;
    const int64_t i = valid ? order[kg] : 0;
    const int64_t l0 = valid ? off[i] : 0, l1 = valid ? off[i + 1] : 0;
    const double vs0 = valid ? vs[2 * i] : 0.0, vs1 = valid ? vs[2 * i + 1] : 0.0;
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double acc[21];
    constexpr int NC = RC > 0 ? RC : 1;
    double cA[NC][4], cH[NC], cS[NC];            // the lane's first RC records
    uint32_t cAC = 0;                            // bit q: record q is across scan
    for (int it = 0; it < INNER_SOLVES; ++it) {
#pragma unroll
        for (int e = 0; e < 21; ++e) acc[e] = 0.0;
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int64_t l = l0 + gl + (int64_t)q * G;
            if (l < l1) {
                if (it == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) cA[q][e] = col[e * n_obs + l];
                    cH[q] = col[4 * n_obs + l];
                    cS[q] = col[5 * n_obs + l];
                    if (cell && cell[l] >= ac_cf0) cAC |= 1u << q;
                }
                const double A[5] = {cA[q][0], cA[q][1], cA[q][2], cA[q][0] * cA[q][3], cA[q][1] * cA[q][3]};
                irls_row(acc, A, cH[q], cS[q], it, d, vs0, vs1, (cAC >> q) & 1u);
            }
        }
        for (int64_t l = l0 + gl + (int64_t)RC * G; l < l1; l += G) {
            double A[5];
#pragma unroll
            for (int e = 0; e < 3; ++e) A[e] = col[e * n_obs + l];
            const double tau = col[3 * n_obs + l];
            A[3] = A[0] * tau;                   // as the design row forms them
            A[4] = A[1] * tau;
            irls_row(acc, A, col[4 * n_obs + l], col[5 * n_obs + l], it, d, vs0, vs1, cell && cell[l] >= ac_cf0);
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
                                                    double* __restrict__ eps2_out, double* __restrict__ D_out,
                                                    const int32_t* __restrict__ cell, int32_t ac_cf0) {
    constexpr int GPB = 256 / G;
    const int gl = threadIdx.x % G;
    const int leader = (threadIdx.x & 63) & ~(G - 1);
    const int64_t kg = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const bool valid = kg < n_src;
    const int64_t i = valid ? order[kg] : 0;
    const int64_t l0 = valid ? off[i] : 0, l1 = valid ? off[i + 1] : 0;
    const double vs0 = valid ? vs[2 * i] : 0.0, vs1 = valid ? vs[2 * i + 1] : 0.0;
    double dw[5] = {0.0, 0.0, 0.0, 0.0, 0.0};      // solution the round's weights come from
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};       // current solution
    double y = 0.0, D = 0.0;
    double acc[21];
    // w_l of the round (it) from dw and the previous round's eps_i^2 (yw)
    auto weight_of = [&](int it, int64_t l, const double* A, double h, double s2, double yw) {
        if (it == 0) return first_weight(h, vs0, vs1, cell, ac_cf0, l);
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
                const double wl = weight_of(it, l, A, h, s2, yw);
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
                const double wl = weight_of(it, l, A, h, s2, yw);
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
template <bool DEFL>
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
        const int32_t cf = ocellfov[l];
        ObsEval o;
        observe<DEFL>(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o, cf >= k.ac_cf0);
        const double sg = (double)osig[l];
        v[l] = o.R * o.R - sg * sg - (robust == 2 ? sp.pad : 0.0);       // e09 with eps_i^2 (mode 2)
    }
}

// Frozen weights: the robust weight of the A/C pass, W = w(R / sigma~) /
// sigma~^2 with sigma~^2 = sigma^2 + eps_a^2 of the record's component and
// bucket (eq:dw, eq:W), at the current parameters, stored as sigma_eff = 1 /
// sqrt(W) in FP64 (W = 0, or sigma_eff beyond it: the largest finite float).
// FP64 because the weight of an outlier, exp(-|z| / 3), moves by ~1e-7
// relative for a rounding-level change of its residual: in FP32 that is a
// whole ulp, and a source whose solution hangs on one such record would
// move with it.
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
                                                     double* __restrict__ sig_eff) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    if (j >= K) return;
    double a4[16], kn[6];
    for (int e = 0; e < 16; ++e) a4[e] = a[4 * j + e];
    for (int e = 0; e < 6; ++e) kn[e] = knots[j + 1 + e];
    const KnotTab kt = ktab[j];
    for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
        const SrcPrep sp = prep[osrc[l]];
        const int32_t cf = ocellfov[l];
        ObsEval o;
        observe(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, a4, kn, kt, o, cf >= k.ac_cf0);
        const double sg = (double)osig[l];
        const double s2 = sg * sg + eps_a2[eps_slot(k, cf, j, eps_bucket)] + (robust == 2 ? sp.pad : 0.0);
        const double W = down_weight(o.R / sqrt(s2)) / s2;
        double se = W > 0.0 ? 1.0 / sqrt(W) : (double)FLT_MAX;
        if (!(se <= (double)FLT_MAX)) se = (double)FLT_MAX;
        sig_eff[l] = se;
    }
}

__global__ void k_gather_f64(int64_t n, const int32_t* __restrict__ from, const double* __restrict__ src,
                             double* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[from[i]];
}

// 68th percentile of the selected values among the n of v, m selected.
template <bool REG, class Sel>
__device__ double percentile68(const double* __restrict__ v, int64_t n, int64_t m, int64_t reg_limit, uint32_t* hist,
                               Sel sel) {
    if (REG && n <= reg_limit) {
        uint64_t kr[KR];
        load_keys(v, n, kr, sel);
        return reg_quantile7(kr, n, m, 0.68, hist);
    }
    return block_quantile7(v, n, m, 0.68, hist, sel);
}

// eq e09 per component and bucket: block c n_buckets + b takes component c
// of bucket b.  cellfov: the records' cell/fov codes in time order, or null
// where every record is along scan (one block per bucket then, which also
// clears the across-scan components).
template <bool REG>
__global__ __launch_bounds__(64) void k_bucket_eps(int64_t n_buckets, int64_t K, int eps_bucket,
                                                   const int64_t* __restrict__ iv_off, const double* __restrict__ v,
                                                   double* __restrict__ eps_a2, int64_t reg_limit,
                                                   const int32_t* __restrict__ cellfov, int32_t ac_cf0) {
    __shared__ uint32_t hist[256];
    const int comp = (int)(blockIdx.x / n_buckets);
    const int64_t b = blockIdx.x - comp * n_buckets;
    if (comp >= 3) return;
    const int64_t j0 = b * eps_bucket;
    const int64_t j1 = j0 + eps_bucket < K ? j0 + eps_bucket : K;
    const int64_t l0 = iv_off[j0], n = iv_off[j1] - l0;
    double q;
    if (!cellfov) {
        q = percentile68<REG>(v + l0, n, n, reg_limit, hist, AllOf{});
        if (threadIdx.x == 0) eps_a2[n_buckets + b] = eps_a2[2 * n_buckets + b] = 0.0;
    } else {
        const OfComponent sel{cellfov + l0, ac_cf0, comp, false};
        q = percentile68<REG>(v + l0, n, block_count(n, sel), reg_limit, hist, sel);
    }
    if (threadIdx.x == 0) eps_a2[comp * n_buckets + b] = q > 0.0 ? q : 0.0;
}

// ------------------------------------------- S block per source in LDS
// The robust source update with a source's observations held on chip: one
// block of NT threads per source fills six LDS columns (alpha*, delta and
// parallax entries of the design row, tau, h and sigma~^2; cap values each)
// -- by evaluating the model and the design row of each observation, or
// (FROM_COL) by reading the HBM columns k_s_rows wrote -- finds varsigma from
// the h column by a block-wide radix selection, and runs the four solves of
// the inner iteration from LDS.  Same arithmetic per observation as k_s_rows
// / k_s_sigma / k_s_irls; the sums are taken in another order.  Sources with
// more than the largest cap observations keep the HBM-column kernels.

// Sum over the NT threads of the block of v[0..NV), every thread receiving
// the sums (fixed order: a butterfly in each wavefront, then the wavefronts in
// order).  red: LDS of (NT / 64) x NV doubles; out: LDS of NV doubles.
template <int NT, int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* red, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = wave_sum(v[e]);
    if (lane == 0)
#pragma unroll
        for (int e = 0; e < NV; ++e) red[wv * NV + e] = v[e];
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[w * NV + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = out[e];
    __syncthreads();
}

// k-th smallest (0-based, k < n) of the selected doubles among x[0..n) in
// LDS, as its order key, by 8-bit radix passes of the whole block; once at
// most 64 keys share the prefix, they are gathered into cand (64 keys in
// LDS), sorted over the first wavefront and the k-th is read off.  hist: 256
// counts in LDS; bc: four ints in LDS (a pass's result, the gather count).
template <int NT, class Sel>
__device__ uint64_t block_select_lds(const double* __restrict__ x, int n, int k, uint32_t* hist, int* bc,
                                     uint64_t* cand, Sel sel) {
    uint64_t prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += NT) hist[b] = 0u;
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += NT) {
            const uint64_t key = order_key(x[j]);
            if ((key & mask) == prefix && sel(j)) {
                // where every active lane of the wavefront has the same digit,
                // one lane adds their count (the leading digits of values of
                // one sign and magnitude would otherwise serialise)
                const uint32_t dg = (uint32_t)(key >> shift) & 255u;
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                const uint64_t am = __ballot(true);
                const uint64_t same = __ballot(dg == d0);
                if (same == am) {
                    if ((int)(threadIdx.x & 63) == __ffsll((unsigned long long)am) - 1)
                        atomicAdd(&hist[d0], (uint32_t)__popcll(am));
                } else {
                    atomicAdd(&hist[dg], 1u);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            int digit;
            uint32_t below;
            radix_digit(hist, k, digit, below);
            if (threadIdx.x == 0) {
                bc[0] = digit;
                bc[1] = (int)below;
                bc[2] = (int)hist[digit];
                bc[3] = 0;
            }
        }
        __syncthreads();
        prefix |= (uint64_t)bc[0] << shift;
        mask |= 0xFFull << shift;
        k -= bc[1];
        const int c = bc[2];
        __syncthreads();
        if (shift > 0 && c <= 64) {
            // gather (in any order: the sort makes the result independent of it)
            for (int j = threadIdx.x; j < n; j += NT) {
                const uint64_t key = order_key(x[j]);
                if ((key & mask) == prefix && sel(j)) cand[atomicAdd(&bc[3], 1)] = key;
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                uint64_t v = (int)threadIdx.x < c ? cand[threadIdx.x] : ~0ull;
                v = wave_sort64(v);
                const uint32_t lo = __shfl((uint32_t)v, k, 64), hi = __shfl((uint32_t)(v >> 32), k, 64);
                if (threadIdx.x == 0) {
                    bc[0] = (int)lo;
                    bc[1] = (int)hi;
                }
            }
            __syncthreads();
            const uint64_t key = ((uint64_t)(uint32_t)bc[1] << 32) | (uint32_t)bc[0];
            __syncthreads();
            return key;
        }
    }
    return prefix;
}

// Type-7 p-quantile of the m selected (sel) elements of x[0..n) in LDS (0
// for m = 0): the order statistic j = floor((m - 1) p) by selection; j + 1
// is the same key when more than j + 1 selected keys are <= it, else the
// smallest selected key above it.  m is the same in every thread.
template <int NT, class Sel>
__device__ double block_quantile7_lds(const double* __restrict__ x, int n, int m, double p, uint32_t* hist, int* bc,
                                      uint64_t* cand,
                                      double* red, double* out, Sel sel) {
    if (m <= 0) return 0.0;
    const double h = (double)(m - 1) * p;
    const int j = (int)floor(h);
    const uint64_t kj = block_select_lds<NT>(x, n, j, hist, bc, cand, sel);
    const double xj = key_value(kj);
    if (j + 1 >= m) return xj;
    // count of selected keys <= kj, and the smallest selected key above it
    double cnt[1] = {0.0};
    uint64_t kmin = ~0ull;
    for (int i = threadIdx.x; i < n; i += NT) {
        if (!sel(i)) continue;
        const uint64_t key = order_key(x[i]);
        if (key <= kj) cnt[0] += 1.0;
        else if (key < kmin) kmin = key;
    }
    // minimum over the block of kmin: per wavefront by shuffles, then in LDS
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)kmin, o, 64), hi = __shfl_xor((uint32_t)(kmin >> 32), o, 64);
        const uint64_t other = ((uint64_t)hi << 32) | lo;
        kmin = other < kmin ? other : kmin;
    }
    uint64_t* kred = reinterpret_cast<uint64_t*>(red);
    // the block's count (exact: integers well below 2^53)
    block_sums<NT, 1>(cnt, red + 2 * (NT / 64), out);
    if ((threadIdx.x & 63) == 0) kred[threadIdx.x >> 6] = kmin;
    __syncthreads();
    uint64_t km = kred[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) km = kred[w] < km ? kred[w] : km;
    __syncthreads();
    const uint64_t kj1 = cnt[0] >= (double)(j + 2) ? kj : km;
    return xj + (h - (double)j) * (key_value(kj1) - xj);
}

// Elements whose byte tag in LDS equals one value.
struct TagIs {
    const uint8_t* tag;
    uint8_t want;
    __device__ bool operator()(int64_t i) const { return tag[i] == want; }
};

template <int NT, bool FROM_COL>
__global__ __launch_bounds__(NT) void k_s_robust(DevConsts k, int64_t n_src, int cap,
                                                 const int64_t* __restrict__ off, const double* __restrict__ ot,
                                                 const double* __restrict__ oeta, const float* __restrict__ osig,
                                                 const int32_t* __restrict__ ocell, const int32_t* __restrict__ oell,
                                                 const double* __restrict__ knots, const KnotTab* __restrict__ ktab,
                                                 const double* __restrict__ a, const double* __restrict__ c,
                                                 const double* __restrict__ eps_a2, int eps_bucket,
                                                 double* __restrict__ s, SrcPrep* __restrict__ prep,
                                                 double* __restrict__ ds, double* __restrict__ qsrc,
                                                 int32_t* __restrict__ sdef, double* __restrict__ svar,
                                                 const int32_t* __restrict__ order, double* __restrict__ vs_out,
                                                 const double* __restrict__ col, int64_t n_obs) {
    extern __shared__ double colm[];            // six columns of cap values, then cap kind bytes
    __shared__ uint32_t hist[256];
    __shared__ double red[(NT / 64) * 24];
    __shared__ double out[24];
    __shared__ int bc[4];
    __shared__ uint64_t cand[64];
    if ((int64_t)blockIdx.x >= n_src) return;
    uint8_t* cKind = reinterpret_cast<uint8_t*>(colm + 6 * cap);   // 1: across scan
    const int64_t i = order[blockIdx.x];
    const int64_t l0 = off[i];
    const int n = (int)(off[i + 1] - l0);       // <= cap (the launcher's class)
    double* cA0 = colm;
    double* cA1 = colm + cap;
    double* cA2 = colm + 2 * cap;
    double* cTau = colm + 3 * cap;
    double* cH = colm + 4 * cap;
    double* cS2 = colm + 5 * cap;
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
    // pass 0: model and design row of every observation, into LDS
    double n_ac[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += NT) {
        const int64_t l = l0 + j;
        const int32_t cf = ocell[l];
        const bool ac = cf >= k.ac_cf0;
        cKind[j] = ac ? 1 : 0;
        n_ac[0] += ac ? 1.0 : 0.0;
        if (FROM_COL) {
            cA0[j] = col[l];
            cA1[j] = col[n_obs + l];
            cA2[j] = col[2 * n_obs + l];
            cTau[j] = col[3 * n_obs + l];
            cH[j] = col[4 * n_obs + l];
            cS2[j] = col[5 * n_obs + l];
            continue;
        }
        const int32_t ell = oell[l];
        const double sg = (double)osig[l];
        ObsEval o;
        observe(k, ot[l], oeta[l], c[cf >> 1], r, mu, plx, a + 4 * (ell - 3), knots + (ell - 2), ktab[ell - 3], o,
                ac);
        double A[5];
        source_partials(o, p, q, r, A, ac);
        cA0[j] = A[0];
        cA1[j] = A[1];
        cA2[j] = A[2];
        cTau[j] = o.tau;                         // A[3] = A[0] tau, A[4] = A[1] tau
        cH[j] = o.R;
        cS2[j] = sg * sg + eps_a2[eps_slot(k, cf, ell - 3, eps_bucket)];
    }
    block_sums<NT, 1>(n_ac, red, out);          // also the barrier after the columns
    // varsigma per kind of record: half the intersextile range of its h
    double vk[2];
    for (int kind = 0; kind < 2; ++kind) {
        const int m = kind ? (int)n_ac[0] : n - (int)n_ac[0];
        const TagIs sel{cKind, (uint8_t)kind};
        const double q5 = block_quantile7_lds<NT>(cH, n, m, 5.0 / 6.0, hist, bc, cand, red, out, sel);
        const double q1 = block_quantile7_lds<NT>(cH, n, m, 1.0 / 6.0, hist, bc, cand, red, out, sel);
        vk[kind] = 0.5 * (q5 - q1);
    }
    if (threadIdx.x == 0) {
        vs_out[2 * i] = vk[0];
        vs_out[2 * i + 1] = vk[1];
    }
    // the inner iteration
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double acc[21];
    for (int it = 0; it < INNER_SOLVES; ++it) {
#pragma unroll
        for (int e = 0; e < 21; ++e) acc[e] = 0.0;
        for (int j = threadIdx.x; j < n; j += NT) {
            double A[5];
            A[0] = cA0[j];
            A[1] = cA1[j];
            A[2] = cA2[j];
            const double tau = cTau[j];
            A[3] = A[0] * tau;
            A[4] = A[1] * tau;
            const double h = cH[j], s2 = cS2[j];
            double wl;
            if (it == 0) {
                const double v = cKind[j] ? vk[1] : vk[0];
                wl = v > 0.0 ? down_weight(h / v) : 1.0;
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
        block_sums<NT, 21>(acc, red, out);
        if (it + 1 < INNER_SOLVES) {
            // one thread solves; every thread takes d
            if (threadIdx.x == 0) {
                double U[25], x[5];
                int e = 0;
                for (int rr = 0; rr < 5; ++rr)
                    for (int cc = rr; cc < 5; ++cc) U[rr * 5 + cc] = acc[e++];
                for (int rr = 0; rr < 5; ++rr) x[rr] = acc[15 + rr];
                small_chol_factor<5>(U);
                small_chol_subst<5>(U, x);
                for (int rr = 0; rr < 5; ++rr) out[rr] = x[rr];
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 5; ++e) d[e] = out[e];
            __syncthreads();
        }
    }
    if (threadIdx.x != 0) return;
    source_finish(acc, i, alpha, delta, plx, pma, pmd, cos(delta), s, prep, ds, qsrc, sdef, svar);
}

// ------------------------------------------ S, rows held in registers
// The robust S block with each source's rows on chip in registers: a block
// of W wavefronts per source, lane l of wavefront w holding the source's
// rows 64 rows w + l + 64 q, q < rows <= SR_M, in FP64 (the design row's
// alpha*, delta and parallax entries and tau, h, sigma~^2: 12 registers a
// row).  The model pass evaluates each observation once; varsigma per kind
// of record is selected from the register-held h across the block's
// wavefronts (exact order statistics, as on the other paths); the four
// rounds of the inner iteration sum over the registers.  Nothing goes
// through HBM but the model's inputs.  (FP32 copies of the design row for
// the first three rounds were tried: the 5x5 systems amplify their rounding
// to ~0.1 uas in the solutions that set the next round's weights.)
constexpr int SR_M = 4;
constexpr int SR_WMAX = 8;

// Sum over the block's W wavefronts of NV values per lane: a butterfly in
// each wavefront (every lane gets the same total), then the wavefronts'
// totals added in wavefront order by every thread.  red: W * NV doubles.
template <int W, int NV>
__device__ __forceinline__ void blk_sum(double (&v)[NV], double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        double x = v[e];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        v[e] = x;
    }
    if (W == 1) return;
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < NV; ++e) red[wv * NV + e] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        double t = red[e];
        for (int w = 1; w < W; ++w) t += red[w * NV + e];
        v[e] = t;
    }
    __syncthreads();
}

// Integer sum over the block (xi: W ints).
template <int W>
__device__ __forceinline__ int blk_count(int v, int* xi) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (W == 1) return v;
    if (lane == 0) xi[wv] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < W; ++w) t += xi[w];
    __syncthreads();
    return t;
}

// Rank k among the <= 64 keys of the block under prefix (mask): each
// wavefront writes its keys after those of the wavefronts before it into
// cand, and every wavefront sorts the same 64 slots and reads the k-th.
// nw: the rows this wavefront holds.
template <int W, int NK>
__device__ __forceinline__ uint64_t blk_finish_select(const uint64_t (&kr)[NK], int nw, uint64_t mask, uint64_t prefix, int64_t k,
                                      uint64_t* cand, int* xi) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < NK; ++q) cnt += (uint32_t)__popcll(__ballot(lane + 64 * q < nw && (kr[q] & mask) == prefix));
    uint32_t base = 0, total = cnt;
    if (W > 1) {
        if (lane == 0) xi[wv] = (int)cnt;
        __syncthreads();
        total = 0;
        for (int w = 0; w < W; ++w) {
            if (w < wv) base += (uint32_t)xi[w];
            total += (uint32_t)xi[w];
        }
    }
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        const bool in = lane + 64 * q < nw && (kr[q] & mask) == prefix;
        const uint64_t b = __ballot(in);
        if (in) cand[base + __popcll(b & below)] = kr[q];
        base += (uint32_t)__popcll(b);
    }
    __syncthreads();
    uint64_t v = lane < (int)total ? cand[lane] : ~0ull;
    __syncthreads();
    v = wave_sort64(v);
    const uint32_t lo = __shfl((uint32_t)v, (int)k, 64), hi = __shfl((uint32_t)(v >> 32), (int)k, 64);
    return ((uint64_t)hi << 32) | lo;
}

// reg_quantile7_pair over the keys of all W wavefronts of the block: the
// histograms are shared, every thread reads the same counts, so every
// wavefront takes the same digits; the closing counts and minima are
// combined over the wavefronts in a fixed order.  hist: 512 counts; cand:
// 64 keys; xi: 2 W ints; xk: 2 W keys.
template <int W, int NK>
__device__ __forceinline__ void blk_quantile7_pair(const uint64_t (&kr)[NK], int nw, int64_t m, double pa, double pb,
                                   uint32_t* hist, uint64_t* cand, int* xi, uint64_t* xk, double& qa, double& qb) {
    if (m <= 0) {
        qa = qb = 0.0;
        return;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double ha_ = (double)(m - 1) * pa, hb_ = (double)(m - 1) * pb;
    const int64_t ja = (int64_t)floor(ha_), jb = (int64_t)floor(hb_);
    int64_t ka = ja, kb = jb;
    uint64_t prea = 0, preb = 0, mask = 0;
    bool done_a = false, done_b = false;
    uint32_t* hista = hist;
    uint32_t* histb = hist + 256;
    for (int shift = 56; shift >= 0 && !(done_a && done_b); shift -= 8) {
        for (int b = threadIdx.x; b < 512; b += 64 * W) hist[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            if (lane + 64 * q < nw) {
                const uint64_t key = kr[q];
                const uint32_t dg = (uint32_t)(key >> shift) & 255u;
                count_digits(hista, dg, !done_a && (key & mask) == prea);
                count_digits(histb, dg, !done_b && (key & mask) == preb);
            }
        }
        __syncthreads();
        uint32_t ca = 65u, cb = 65u;
        if (!done_a) {
            int d;
            uint32_t bel;
            radix_digit(hista, ka, d, bel);
            prea |= (uint64_t)d << shift;
            ka -= (int64_t)bel;
            ca = hista[d];
        }
        if (!done_b) {
            int d;
            uint32_t bel;
            radix_digit(histb, kb, d, bel);
            preb |= (uint64_t)d << shift;
            kb -= (int64_t)bel;
            cb = histb[d];
        }
        mask |= 0xFFull << shift;
        __syncthreads();
        if (shift > 0 && !done_a && ca <= 64u) {
            prea = blk_finish_select<W>(kr, nw, mask, prea, ka, cand, xi);
            done_a = true;
        }
        if (shift > 0 && !done_b && cb <= 64u) {
            preb = blk_finish_select<W>(kr, nw, mask, preb, kb, cand, xi);
            done_b = true;
        }
    }
    uint32_t cla = 0, clb = 0;
    uint64_t mna = ~0ull, mnb = ~0ull;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        if (lane + 64 * q < nw) {
            const uint64_t key = kr[q];
            cla += key <= prea ? 1u : 0u;
            clb += key <= preb ? 1u : 0u;
            if (key > prea && key < mna) mna = key;
            if (key > preb && key < mnb) mnb = key;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cla += __shfl_xor(cla, o, 64);
        clb += __shfl_xor(clb, o, 64);
        uint32_t lo = __shfl_xor((uint32_t)mna, o, 64), hi = __shfl_xor((uint32_t)(mna >> 32), o, 64);
        uint64_t other = ((uint64_t)hi << 32) | lo;
        mna = other < mna ? other : mna;
        lo = __shfl_xor((uint32_t)mnb, o, 64);
        hi = __shfl_xor((uint32_t)(mnb >> 32), o, 64);
        other = ((uint64_t)hi << 32) | lo;
        mnb = other < mnb ? other : mnb;
    }
    if (W > 1) {
        if (lane == 0) {
            xi[2 * wv] = (int)cla;
            xi[2 * wv + 1] = (int)clb;
            xk[2 * wv] = mna;
            xk[2 * wv + 1] = mnb;
        }
        __syncthreads();
        cla = clb = 0;
        mna = mnb = ~0ull;
        for (int w = 0; w < W; ++w) {
            cla += (uint32_t)xi[2 * w];
            clb += (uint32_t)xi[2 * w + 1];
            mna = xk[2 * w] < mna ? xk[2 * w] : mna;
            mnb = xk[2 * w + 1] < mnb ? xk[2 * w + 1] : mnb;
        }
        __syncthreads();
    }
    const double xa = key_value(prea), xb = key_value(preb);
    qa = ja + 1 >= m ? xa : xa + (ha_ - (double)ja) * (key_value((int64_t)cla >= ja + 2 ? prea : mna) - xa);
    qb = jb + 1 >= m ? xb : xb + (hb_ - (double)jb) * (key_value((int64_t)clb >= jb + 2 ? preb : mnb) - xb);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_s_regs(DevConsts k, int64_t n_src, const int64_t* __restrict__ off,
                                                   const double* __restrict__ ot, const double* __restrict__ oeta,
                                                   const float* __restrict__ osig, const int32_t* __restrict__ ocell,
                                                   const int32_t* __restrict__ oell,
                                                   const double* __restrict__ knots,
                                                   const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                   const double* __restrict__ c, const double* __restrict__ eps_a2,
                                                   int eps_bucket, double* __restrict__ s,
                                                   SrcPrep* __restrict__ prep, double* __restrict__ ds,
                                                   double* __restrict__ qsrc, int32_t* __restrict__ sdef,
                                                   double* __restrict__ svar, const int32_t* __restrict__ order,
                                                   double* __restrict__ vs_out, int rows) {
    __shared__ uint32_t hist[512];
    __shared__ uint64_t cand[64];
    __shared__ double red[W * 21];
    __shared__ int xi[2 * W];
    __shared__ uint64_t xk[2 * W];
    if ((int64_t)blockIdx.x >= n_src) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = order[blockIdx.x];
    const int64_t l0 = off[i];
    const int n = (int)(off[i + 1] - l0);        // <= 64 rows W (the launcher's class)
    const int nw = min(max(n - 64 * rows * wv, 0), 64 * rows);
    const int64_t lw = l0 + 64 * rows * wv;      // this wavefront's first observation
    double p[3], q[3], r[3], mu[3], plx;
    {
        const double* si = s + 5 * i;
        double sa, ca, sd, cd;
        sincos(si[0], &sa, &ca);
        sincos(si[1], &sd, &cd);
        p[0] = -sa;
        p[1] = ca;
        p[2] = 0.0;
        q[0] = -sd * ca;
        q[1] = -sd * sa;
        q[2] = cd;
        r[0] = cd * ca;
        r[1] = cd * sa;
        r[2] = sd;
        plx = si[2];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) mu[cc] = p[cc] * si[3] + q[cc] * si[4];
    }
    // the rows: design row (alpha*, delta, parallax entries and tau), h,
    // sigma~^2; bit qq of acm: row qq is across scan
    double af[SR_M][4], s2v[SR_M], hv[SR_M];
    uint32_t acm = 0;
#pragma unroll
    for (int qq = 0; qq < SR_M; ++qq) {
        af[qq][0] = af[qq][1] = af[qq][2] = af[qq][3] = 0.0;
        s2v[qq] = 1.0;
        hv[qq] = 0.0;
    }
    // model pass: the current row with its gathers; the next row's columns
    // load at the top of a step, its gathers after the current row has been
    // evaluated (lanes past the end repeat the wavefront's last row)
    double t_c = 0.0, e_c = 0.0, cal_c = 0.0, ea_c = 0.0;
    float s_c = 1.0f;
    int32_t ell_c = 3, cf_c = 0;
    double a_c[16];
    KnotTab kt_c = {0.0, 1.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 16; ++e) a_c[e] = 0.0;
    if (nw > 0) {
        const int64_t le = lw + (lane < nw ? lane : nw - 1);
        t_c = ot[le];
        e_c = oeta[le];
        s_c = osig[le];
        ell_c = oell[le];
        cf_c = ocell[le];
        cal_c = c[cf_c >> 1];
        ea_c = eps_a2[eps_slot(k, cf_c, ell_c - 3, eps_bucket)];
        const double* a4 = a + 4 * (ell_c - 3);
#pragma unroll
        for (int e = 0; e < 16; ++e) a_c[e] = a4[e];
        kt_c = ktab[ell_c - 3];
    }
    for (int qs = 0; qs < SR_M && 64 * qs < nw; ++qs) {
        const int rn = 64 * (qs + 1) + lane;
        const bool more = 64 * (qs + 1) < nw;    // the wavefront has a next step
        double t_n = 0.0, e_n = 0.0;
        float s_n = 1.0f;
        int32_t cf_n = 0, ell_n = 3;
        if (more) {
            const int64_t le = lw + (rn < nw ? rn : nw - 1);
            t_n = ot[le];
            e_n = oeta[le];
            s_n = osig[le];
            cf_n = ocell[le];
            ell_n = oell[le];
        }
        const bool ac = cf_c >= k.ac_cf0;
        ObsEval o;
        observe(k, t_c, e_c, cal_c, r, mu, plx, a_c, knots + (ell_c - 2), kt_c, o, ac);
        double A[5];
        source_partials(o, p, q, r, A, ac);
        const double sg = (double)s_c;
        const double s2 = sg * sg + ea_c;
        if (ac && 64 * qs + lane < nw) acm |= 1u << qs;
#pragma unroll
        for (int qq = 0; qq < SR_M; ++qq) {
            if (qq == qs) {
                af[qq][0] = A[0];
                af[qq][1] = A[1];
                af[qq][2] = A[2];
                af[qq][3] = o.tau;               // A[3] = A[0] tau, A[4] = A[1] tau
                hv[qq] = o.R;
                s2v[qq] = s2;
            }
        }
        if (more) {
            const double* a4 = a + 4 * (ell_n - 3);
#pragma unroll
            for (int e = 0; e < 16; ++e) a_c[e] = a4[e];
            kt_c = ktab[ell_n - 3];
            cal_c = c[cf_n >> 1];
            ea_c = eps_a2[eps_slot(k, cf_n, ell_n - 3, eps_bucket)];
        }
        t_c = t_n;
        e_c = e_n;
        s_c = s_n;
        cf_c = cf_n;
        ell_c = ell_n;
    }
    // varsigma per kind of record: half the intersextile range of its h
    const int n_ac = blk_count<W>(__popc(acm), xi);
    double vk0 = 0.0, vk1 = 0.0;
    for (int kind = 0; kind < 2; ++kind) {
        const int64_t m = kind ? n_ac : n - n_ac;
        if (m <= 0) continue;
        uint64_t kr[SR_M];
#pragma unroll
        for (int qq = 0; qq < SR_M; ++qq)
            kr[qq] = (lane + 64 * qq < nw && (int)((acm >> qq) & 1u) == kind) ? order_key(hv[qq]) : ~0ull;
        double q5, q1;
        blk_quantile7_pair<W>(kr, nw, m, 5.0 / 6.0, 1.0 / 6.0, hist, cand, xi, xk, q5, q1);
        if (kind == 0) vk0 = 0.5 * (q5 - q1);
        else vk1 = 0.5 * (q5 - q1);
    }
    if (threadIdx.x == 0) {
        vs_out[2 * i] = vk0;
        vs_out[2 * i + 1] = vk1;
    }
    // the inner iteration
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double acc[21];
    for (int it = 0; it < INNER_SOLVES; ++it) {
        const bool last = it + 1 == INNER_SOLVES;
#pragma unroll
        for (int e = 0; e < 21; ++e) acc[e] = 0.0;
#pragma unroll
        for (int qq = 0; qq < SR_M; ++qq) {
            if (lane + 64 * qq < nw) {
                double A[5];
                const double h = hv[qq], s2 = s2v[qq];
                A[0] = af[qq][0];
                A[1] = af[qq][1];
                A[2] = af[qq][2];
                A[3] = A[0] * af[qq][3];         // as the design row forms them
                A[4] = A[1] * af[qq][3];
                double wl;
                if (it == 0) {
                    const double v = ((acm >> qq) & 1u) ? vk1 : vk0;
                    wl = v > 0.0 ? down_weight(h / v) : 1.0;
                } else {
                    double R = h;
#pragma unroll
                    for (int e = 0; e < 5; ++e) R -= A[e] * d[e];
                    wl = down_weight(R / sqrt(s2));
                }
                const double Wt = wl / s2;
                int e = 0;
#pragma unroll
                for (int rr = 0; rr < 5; ++rr) {
                    const double wa = A[rr] * Wt;
#pragma unroll
                    for (int cc = rr; cc < 5; ++cc) acc[e++] += wa * A[cc];
                }
#pragma unroll
                for (int rr = 0; rr < 5; ++rr) acc[15 + rr] += A[rr] * Wt * h;
                acc[20] += Wt * h * h;
            }
        }
        blk_sum<W, 21>(acc, red);
        if (!last) {
            // lane 0 of each wavefront solves (the same numbers in each);
            // every lane takes d
            double x[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (lane == 0) {
                double U[25];
                int e = 0;
                for (int rr = 0; rr < 5; ++rr)
                    for (int cc = rr; cc < 5; ++cc) U[rr * 5 + cc] = acc[e++];
                for (int rr = 0; rr < 5; ++rr) x[rr] = acc[15 + rr];
                small_chol_factor<5>(U);
                small_chol_subst<5>(U, x);
            }
#pragma unroll
            for (int e = 0; e < 5; ++e) d[e] = __shfl(x[e], 0, 64);
        }
    }
    if (threadIdx.x != 0) return;
    const double* si = s + 5 * i;
    source_finish(acc, i, si[0], si[1], si[2], si[3], si[4], cos(si[1]), s, prep, ds, qsrc, sdef, svar);
}

// Excess attitude noise in one kernel: one block of NT threads per bucket of
// eps_bucket knot intervals evaluates R^2 - sigma^2 (- eps_i^2 in robust mode
// 2) of the bucket's observations into LDS, with the attitude component each
// measures, and takes the 68th percentile of each component's values there
// (eq e09): k_ac_resid and k_bucket_eps without the HBM round trip.  The
// threads stream the bucket's observations as one range (an interval holds
// a few hundred, so a pass per interval would leave many threads idle); the
// bucket's attitude coefficients, knots, interval tables and offsets sit in
// LDS, and each observation finds its interval there by bisection.
template <int NT, bool DEFL = false>
__global__ __launch_bounds__(NT) void k_eps_fused(DevConsts k, int64_t n_buckets, int64_t K, int eps_bucket, int cap,
                                                  const int64_t* __restrict__ iv_off, const double* __restrict__ ot,
                                                  const double* __restrict__ oeta, const float* __restrict__ osig,
                                                  const int32_t* __restrict__ ocellfov,
                                                  const int32_t* __restrict__ osrc, const SrcPrep* __restrict__ prep,
                                                  const double* __restrict__ knots,
                                                  const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                  const double* __restrict__ c, int robust,
                                                  double* __restrict__ eps_a2) {
    // dynamic LDS: the bucket's values (cap doubles), its eps_bucket + 3
    // attitude coefficients (4 doubles each), eps_bucket + 6 knots,
    // eps_bucket interval tables and eps_bucket + 1 offsets, then cap
    // component bytes
    extern __shared__ double vals[];
    __shared__ uint32_t hist[256];
    __shared__ double red[(NT / 64) * 24];
    __shared__ double out[24];
    __shared__ int bc[4];
    __shared__ uint64_t cand[64];
    const int64_t b = blockIdx.x;
    if (b >= n_buckets) return;
    double* sa = vals + cap;
    double* sk = sa + 4 * (eps_bucket + 3);
    KnotTab* st = reinterpret_cast<KnotTab*>(sk + eps_bucket + 6);
    int64_t* so = reinterpret_cast<int64_t*>(st + eps_bucket);
    uint8_t* comp = reinterpret_cast<uint8_t*>(so + eps_bucket + 1);
    const int64_t j0 = b * eps_bucket;
    const int64_t j1 = j0 + eps_bucket < K ? j0 + eps_bucket : K;
    const int nj = (int)(j1 - j0);
    for (int e = threadIdx.x; e < 4 * (nj + 3); e += NT) sa[e] = a[4 * j0 + e];
    for (int e = threadIdx.x; e < nj + 6; e += NT) sk[e] = knots[j0 + 1 + e];
    for (int e = threadIdx.x; e < nj; e += NT) st[e] = ktab[j0 + e];
    for (int e = threadIdx.x; e <= nj; e += NT) so[e] = iv_off[j0 + e];
    __syncthreads();
    const int64_t lb = so[0];
    const int n = (int)(so[nj] - lb);
    double cnt[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += NT) {
        const int64_t l = lb + i;
        // the interval: the largest jj with so[jj] <= l
        int lo = 0, hi = nj - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (so[mid] <= l) lo = mid;
            else hi = mid - 1;
        }
        const SrcPrep sp = prep[osrc[l]];
        const int32_t cf = ocellfov[l];
        const bool ac = cf >= k.ac_cf0;
        ObsEval o;
        observe<DEFL>(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, sa + 4 * lo, sk + lo, st[lo], o, ac);
        const double sg = (double)osig[l];
        vals[i] = o.R * o.R - sg * sg - (robust == 2 ? sp.pad : 0.0);
        const int cm = ac ? 1 + (cf & 1) : 0;
        comp[i] = (uint8_t)cm;
        cnt[0] += cm == 0 ? 1.0 : 0.0;
        cnt[1] += cm == 1 ? 1.0 : 0.0;
        cnt[2] += cm == 2 ? 1.0 : 0.0;
    }
    block_sums<NT, 3>(cnt, red, out);           // also the barrier after the values
    for (int cm = 0; cm < 3; ++cm) {
        const double qv = block_quantile7_lds<NT>(vals, n, (int)cnt[cm], 0.68, hist, bc, cand, red, out,
                                                  TagIs{comp, (uint8_t)cm});
        if (threadIdx.x == 0) eps_a2[cm * n_buckets + b] = qv > 0.0 ? qv : 0.0;
    }
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

// Dynamic LDS of k_s_robust (six columns and a byte per record) and of
// k_eps_fused (a value and a byte per record) for cap records.
inline size_t s_lds_bytes(int64_t cap) { return (size_t)cap * (6 * sizeof(double) + 1); }
inline size_t eps_lds_bytes(int64_t cap, int64_t eps_bucket) {
    return (size_t)cap * (sizeof(double) + 1) +
           (size_t)(4 * (eps_bucket + 3) + (eps_bucket + 6) + 4 * eps_bucket + (eps_bucket + 1)) * sizeof(double);
}

}  // namespace

#define AGIS_ROWS_LAUNCH(G)                                                                                      \
    (ctx->k.defl > 0.0 ? k_s_rows<G, true> : k_s_rows<G, false>)<<<groups_grid(n_src, 256 / G), 256, 0, ctx->stream>>>( \
        ctx->k, n_src, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots,        \
        ctx->ktab, ctx->a, ctx->c, ctx->s, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->rcol, ctx->n_obs, order)
#define AGIS_IRLS_LAUNCH(G)                                                                                      \
    if (ctx->cfg.robust == 2)                                                                                    \
        k_s_irls_eps<G><<<groups_grid(n_src, 256 / G), 256, 0, ctx->stream>>>(                                   \
            n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc,           \
            ctx->sdef, ctx->svar, order, ctx->src_eps2, ctx->src_D, ac_cells, ctx->k.ac_cf0);                    \
    else                                                                                                         \
        k_s_irls<G><<<groups_grid(n_src, 256 / G), 256, 0, ctx->stream>>>(                                       \
            n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc,           \
            ctx->sdef, ctx->svar, order, ac_cells, ctx->k.ac_cf0)

// The HBM-column kernels over launch positions [k0, k0 + n) of the
// count-ordered source list: the rows (model and design row per
// observation into the columns), then varsigma and the inner iteration.
static void source_rows(agis_ctx* ctx, int64_t k0, int64_t n) {
    if (n <= 0) return;
    const int32_t* order = ctx->src_order + k0;
    const int64_t n_src = n;
    switch (ctx->s_group) {
        case 8: AGIS_ROWS_LAUNCH(8); break;
        case 16: AGIS_ROWS_LAUNCH(16); break;
        case 32: AGIS_ROWS_LAUNCH(32); break;
        default: AGIS_ROWS_LAUNCH(64); break;
    }
}

static void source_solve_columns(agis_ctx* ctx, int64_t k0, int64_t n) {
    if (n <= 0) return;
    const int32_t* order = ctx->src_order + k0;
    const int64_t n_src = n;
    const int32_t* ac_cells = ctx->has_ac ? ctx->s_cell : nullptr;   // kinds of record matter with AC records
    const bool reg = select_in_registers(ctx, ctx->n_obs, ctx->n_src);
    const bool pair = ctx->select_pair;
    (ac_cells ? (reg ? (pair ? k_s_sigma<2, true> : k_s_sigma<1, true>) : k_s_sigma<0, true>)
              : (reg ? (pair ? k_s_sigma<2, false> : k_s_sigma<1, false>) : k_s_sigma<0, false>))
        <<<(unsigned)n_src, 64, 0, ctx->stream>>>(n_src, ctx->src_off, ctx->rcol + 4 * ctx->n_obs, ctx->vs,
                                                  select_reg_limit(ctx), order, ac_cells, ctx->k.ac_cf0);
    if (ctx->cfg.robust == 1 && ctx->irls_cache > 0) {
        // the lanes' first records cached in registers across the rounds
#define AGIS_IRLS_CACHED(G)                                                                                      \
    k_s_irls<G, IRLS_RC><<<groups_grid(n_src, 256 / G), 256, 0, ctx->stream>>>(                                  \
        n_src, ctx->src_off, ctx->rcol, ctx->n_obs, ctx->vs, ctx->s, ctx->prep, ctx->ds, ctx->qsrc, ctx->sdef,    \
        ctx->svar, order, ac_cells, ctx->k.ac_cf0)
        if (ctx->irls_cache == 1) AGIS_IRLS_CACHED(32);
        else AGIS_IRLS_CACHED(64);
#undef AGIS_IRLS_CACHED
        return;
    }
    switch (ctx->s_group) {
        case 8: AGIS_IRLS_LAUNCH(8); break;
        case 16: AGIS_IRLS_LAUNCH(16); break;
        case 32: AGIS_IRLS_LAUNCH(32); break;
        default: AGIS_IRLS_LAUNCH(64); break;
    }
}

// Per-source LDS kernels for the robust S block (robust mode 1 only; the
// excess source noise of mode 2 keeps the HBM-column kernels).
static bool s_lds(const agis_ctx* ctx) {
    return ctx->robust_s_mode >= 1 && ctx->cfg.robust == 1 && !(ctx->k.defl > 0.0);   // on-chip paths: plain model
}
static bool s_from_columns(const agis_ctx* ctx) { return ctx->robust_s_mode == 1; }
static bool s_regs(const agis_ctx* ctx) { return ctx->robust_s_mode == 3; }
static int sreg_rows(const agis_ctx* ctx) { return std::min(std::max(ctx->sreg_rows, 1), SR_M); }
static bool eps_one_kernel(const agis_ctx* ctx) { return ctx->robust_fused_eps && ctx->cfg.robust >= 1; }

void launch_source_update_robust(agis_ctx* ctx) {
    if (ctx->n_src == 0) return;
    if (!s_lds(ctx)) {
        source_rows(ctx, 0, ctx->n_src);
        source_solve_columns(ctx, 0, ctx->n_src);
        return;
    }
    const bool from_col = s_from_columns(ctx);
    // the sources beyond the largest LDS class: the HBM-column kernels
    source_rows(ctx, 0, from_col ? ctx->n_src : ctx->s_fallback);
    source_solve_columns(ctx, 0, ctx->s_fallback);
    if (s_regs(ctx)) {
        for (const SClass& cl : ctx->s_classes) {
            const int64_t n = cl.k1 - cl.k0;
#define AGIS_SREG_LAUNCH(W)                                                                                      \
    k_s_regs<W><<<(unsigned)n, 64 * W, 0, ctx->stream>>>(                                                        \
        ctx->k, n, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots, ctx->ktab,  \
        ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->s, ctx->prep, ctx->ds, ctx->qsrc, ctx->sdef,        \
        ctx->svar, ctx->src_order + cl.k0, ctx->vs, sreg_rows(ctx))
            switch (cl.nt / 64) {
                case 1: AGIS_SREG_LAUNCH(1); break;
                case 2: AGIS_SREG_LAUNCH(2); break;
                case 3: AGIS_SREG_LAUNCH(3); break;
                case 4: AGIS_SREG_LAUNCH(4); break;
                case 5: AGIS_SREG_LAUNCH(5); break;
                case 6: AGIS_SREG_LAUNCH(6); break;
                case 7: AGIS_SREG_LAUNCH(7); break;
                default: AGIS_SREG_LAUNCH(8); break;
            }
#undef AGIS_SREG_LAUNCH
        }
        return;
    }
    for (const SClass& cl : ctx->s_classes) {
        const int64_t n = cl.k1 - cl.k0;
        const size_t lds = s_lds_bytes(cl.cap);
#define AGIS_SROB_LAUNCH(NT, FC)                                                                                 \
    k_s_robust<NT, FC><<<(unsigned)n, NT, lds, ctx->stream>>>(                                                  \
        ctx->k, n, cl.cap, ctx->src_off, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell, ctx->knots,    \
        ctx->ktab, ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->s, ctx->prep, ctx->ds, ctx->qsrc,        \
        ctx->sdef, ctx->svar, ctx->src_order + cl.k0, ctx->vs, ctx->rcol, ctx->n_obs)
        if (from_col) {
            if (cl.nt == 64) AGIS_SROB_LAUNCH(64, true);
            else if (cl.nt == 128) AGIS_SROB_LAUNCH(128, true);
            else AGIS_SROB_LAUNCH(256, true);
        } else {
            if (cl.nt == 64) AGIS_SROB_LAUNCH(64, false);
            else if (cl.nt == 128) AGIS_SROB_LAUNCH(128, false);
            else AGIS_SROB_LAUNCH(256, false);
        }
#undef AGIS_SROB_LAUNCH
    }
}

#define HIPCHK(expr)                                            \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_check(ctx, e_, #expr); \
    } while (0)

// Observation-count classes of the one-kernel S path and its thread counts,
// largest first; a class holds the counts above the next one's cap.
static const int kSCaps[] = {3072, 2560, 2048, 1536, 1024, 768, 512, 384, 256, 128, 64, 32};
static int s_threads(int cap) { return cap > 1024 ? 256 : (cap > 256 ? 128 : 64); }
constexpr int EPS_NT = 256;

int robust_plan(agis_ctx* ctx, const std::vector<int64_t>& h_off, const std::vector<int32_t>& order,
                bool* need_columns) {
    ctx->s_classes.clear();
    ctx->s_fallback = 0;
    ctx->eps_fused = false;
    ctx->eps_cap = 0;
    *need_columns = true;
    // dynamic LDS a block may use beside the kernels' own (a few KB)
    int max_lds = 0;
    HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    const int64_t dyn_max = (int64_t)max_lds - 4096;
    const int64_t n_src = (int64_t)order.size();
    // classes: walk the count-ordered list from the smallest counts up
    int64_t k1 = s_lds(ctx) ? n_src : 0;
    if (s_regs(ctx)) {
        // register path: W wavefronts for up to 64 rows W rows
        for (int W = 1; W <= SR_WMAX && k1 > 0; ++W) {
            const int cap = 64 * sreg_rows(ctx) * W;
            int64_t k0 = k1;
            while (k0 > 0) {
                const int32_t i = order[k0 - 1];
                const int64_t cnt = h_off[i + 1] - h_off[i];
                if (cnt > cap || cnt > ctx->robust_max_cap) break;
                --k0;
            }
            if (k0 < k1) ctx->s_classes.push_back(SClass{k0, k1, cap, 64 * W});
            k1 = k0;
        }
        ctx->s_fallback = k1;
        std::reverse(ctx->s_classes.begin(), ctx->s_classes.end());
        k1 = 0;                          // no LDS classes
    }
    for (int ci = (int)(sizeof kSCaps / sizeof kSCaps[0]) - 1; ci >= 0 && k1 > 0; --ci) {
        const int cap = kSCaps[ci];
        if ((int64_t)s_lds_bytes(cap) > dyn_max || cap > ctx->robust_max_cap) break;
        int64_t k0 = k1;
        while (k0 > 0) {
            const int32_t i = order[k0 - 1];
            if (h_off[i + 1] - h_off[i] > cap) break;
            --k0;
        }
        if (k0 < k1) ctx->s_classes.push_back(SClass{k0, k1, cap, s_threads(cap)});
        k1 = k0;
    }
    if (!s_regs(ctx)) {
        ctx->s_fallback = k1;
        // largest classes first (the count order)
        std::reverse(ctx->s_classes.begin(), ctx->s_classes.end());
    }
    int used_max[3] = {0, 0, 0};
    for (const SClass& cl : ctx->s_classes) {
        if (s_regs(ctx)) break;
        const int slot = cl.nt == 64 ? 0 : (cl.nt == 128 ? 1 : 2);
        used_max[slot] = std::max(used_max[slot], (int)s_lds_bytes(cl.cap));
    }
    const bool fc = s_from_columns(ctx);
    const void* fn[3] = {fc ? reinterpret_cast<const void*>(&k_s_robust<64, true>)
                            : reinterpret_cast<const void*>(&k_s_robust<64, false>),
                         fc ? reinterpret_cast<const void*>(&k_s_robust<128, true>)
                            : reinterpret_cast<const void*>(&k_s_robust<128, false>),
                         fc ? reinterpret_cast<const void*>(&k_s_robust<256, true>)
                            : reinterpret_cast<const void*>(&k_s_robust<256, false>)};
    for (int slot = 0; slot < 3; ++slot)
        if (used_max[slot]) HIPCHK(hipFuncSetAttribute(fn[slot], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       used_max[slot]));
    // the excess-noise buckets: the largest bucket's values must fit
    if (!eps_one_kernel(ctx)) {
        ctx->eps_fused = false;
    } else if (ctx->K > 0 && ctx->n_buckets > 0) {
        std::vector<int64_t> iv(ctx->K + 1);
        HIPCHK(hipMemcpy(iv.data(), ctx->iv_off, (ctx->K + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        int64_t mx = 0;
        for (int64_t b = 0; b < ctx->n_buckets; ++b) {
            const int64_t j0 = b * ctx->cfg.eps_bucket, j1 = std::min<int64_t>(j0 + ctx->cfg.eps_bucket, ctx->K);
            mx = std::max(mx, iv[j1] - iv[j0]);
        }
        ctx->eps_cap = std::max<int64_t>(mx, 1);
        if ((int64_t)eps_lds_bytes(ctx->eps_cap, ctx->cfg.eps_bucket) <= dyn_max) {
            HIPCHK(hipFuncSetAttribute(ctx->k.defl > 0.0 ? reinterpret_cast<const void*>(&k_eps_fused<EPS_NT, true>)
                                                         : reinterpret_cast<const void*>(&k_eps_fused<EPS_NT, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)eps_lds_bytes(ctx->eps_cap, ctx->cfg.eps_bucket)));
            ctx->eps_fused = true;
        }
    } else {
        ctx->eps_fused = true;
    }
    *need_columns = !s_lds(ctx) || fc || ctx->s_fallback > 0 || !ctx->eps_fused;
    return AGIS_OK;
}
#undef HIPCHK

void launch_freeze_sigma(agis_ctx* ctx) {
    if (ctx->K > 0)
        k_freeze_sigma<<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(
            ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig, ctx->t_cellfov, ctx->t_src, ctx->prep,
            ctx->knots, ctx->ktab, ctx->a, ctx->c, ctx->eps_a2, ctx->cfg.eps_bucket, ctx->cfg.robust, ctx->t_sig_eff);
    if (ctx->n_obs > 0) {
        const int64_t b = std::min<int64_t>((ctx->n_obs + 255) / 256, 65536);
        k_gather_f64<<<(unsigned)b, 256, 0, ctx->stream>>>(ctx->n_obs, ctx->s_from_t, ctx->t_sig_eff,
                                                           ctx->s_sig_eff);
    }
}

void launch_excess_noise(agis_ctx* ctx) {
    if (ctx->K == 0 || ctx->n_buckets == 0) return;
    if (eps_one_kernel(ctx) && ctx->eps_fused) {
        (ctx->k.defl > 0.0 ? k_eps_fused<EPS_NT, true> : k_eps_fused<EPS_NT, false>)
            <<<(unsigned)ctx->n_buckets, EPS_NT, eps_lds_bytes(ctx->eps_cap, ctx->cfg.eps_bucket), ctx->stream>>>(
            ctx->k, ctx->n_buckets, ctx->K, ctx->cfg.eps_bucket, (int)ctx->eps_cap, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig,
            ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots, ctx->ktab, ctx->a, ctx->c, ctx->cfg.robust,
            ctx->eps_a2);
        return;
    }
    (ctx->k.defl > 0.0 ? k_ac_resid<true> : k_ac_resid<false>)<<<(unsigned)ctx->K, 64, 0, ctx->stream>>>(
                                                         ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta, ctx->t_sig,
                                                         ctx->t_cellfov, ctx->t_src, ctx->prep, ctx->knots, ctx->ktab,
                                                         ctx->a, ctx->c, ctx->cfg.robust, ctx->rcol);
    const int32_t* cellfov = ctx->has_ac ? ctx->t_cellfov : nullptr;
    (select_in_registers(ctx, ctx->n_obs, ctx->n_buckets) ? k_bucket_eps<true> : k_bucket_eps<false>)
        <<<(unsigned)((cellfov ? 3 : 1) * ctx->n_buckets), 64, 0, ctx->stream>>>(
            ctx->n_buckets, ctx->K, ctx->cfg.eps_bucket, ctx->iv_off, ctx->rcol, ctx->eps_a2, select_reg_limit(ctx),
            cellfov, ctx->k.ac_cf0);
}

}  // namespace agis
