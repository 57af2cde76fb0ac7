// Observation store: validation and the two device orders of the
// observation records (Sect. 3.5) streamed by the update blocks.
//   by (source, time): the S block reads each source's observations
//                      contiguously (eq:normS sums over l in i);
//   by time:           the A and C blocks read each knot interval's
//                      observations contiguously (eq:normA sums over L_n).
// Runs once per problem; sorting uses rocPRIM's radix sort through hipCUB.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>

#include "agis_internal.h"

namespace agis {

namespace {

template <typename T>
int dalloc(agis_ctx* ctx, T** p, size_t n, const char* what) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(ctx, AGIS_E_OOM, std::string("device allocation failed for ") + what);
    }
    return AGIS_OK;
}

// Error bits raised by the validation kernel.
enum : int {
    BAD_SRC = 1,
    BAD_CELL = 2,
    BAD_FOV = 4,
    BAD_T = 8,
    BAD_SIGMA = 16,
    BAD_ETA = 32,
    HAS_AC = 128        // not an error: some observation is across scan (cell -1)
};

__global__ void k_validate(int64_t n, const double* __restrict__ t, const double* __restrict__ eta,
                           const float* __restrict__ sig, const int32_t* __restrict__ src,
                           const int8_t* __restrict__ fov, const int32_t* __restrict__ cell, int64_t n_src,
                           int64_t n_cells, double t_lo, double t_hi, int* __restrict__ flags) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (src[i] < 0 || src[i] >= n_src) bad |= BAD_SRC;
        if (cell[i] == -1) bad |= HAS_AC;
        else if (cell[i] < 0 || cell[i] >= n_cells) bad |= BAD_CELL;
        if (fov[i] != 1 && fov[i] != -1) bad |= BAD_FOV;
        const double ti = t[i];
        if (!(ti >= t_lo && ti <= t_hi)) bad |= BAD_T;
        const float s = sig[i];
        if (!(s > 0.0f) || !isfinite(s)) bad |= BAD_SIGMA;
        if (!isfinite(eta[i])) bad |= BAD_ETA;
    }
    // ingest-time validation only: one flag word for the whole launch
    if (bad) atomicOr(flags, bad);
}

__global__ void k_iota(int64_t n, int32_t* __restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

// Gather the input columns into time order.  An across-scan observation
// (cell -1) takes the pseudo-cell n_cells, whose calibration entry stays
// zero, so that every pass may read c[cellfov >> 1].
__global__ void k_gather_time(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ eta,
                              const float* __restrict__ sig, const int32_t* __restrict__ src,
                              const int8_t* __restrict__ fov, const int32_t* __restrict__ cell, int32_t n_cells,
                              double* __restrict__ o_eta, float* __restrict__ o_sig, int32_t* __restrict__ o_src,
                              int32_t* __restrict__ o_cellfov) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = perm[i];
        o_eta[i] = eta[j];
        o_sig[i] = sig[j];
        o_src[i] = src[j];
        o_cellfov[i] = (cell[j] < 0 ? n_cells : cell[j]) * 2 + (fov[j] < 0 ? 1 : 0);
    }
}

// Left index of t: largest l in [3, N-1] with tau_l <= t (t = tau_N -> N-1).
__device__ __forceinline__ int32_t left_index(const double* __restrict__ knots, int64_t N, double t) {
    int64_t lo = 3, hi = N - 1;
    if (t >= knots[N]) return (int32_t)(N - 1);
    if (t <= knots[3]) return 3;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (knots[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return (int32_t)lo;
}

// Gather the time-ordered columns into (source, time) order and compute
// the left index of every observation.
__global__ void k_gather_source(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ t_t,
                                const double* __restrict__ t_eta, const float* __restrict__ t_sig,
                                const int32_t* __restrict__ t_cellfov, const double* __restrict__ knots, int64_t N,
                                double* __restrict__ o_t, double* __restrict__ o_eta, float* __restrict__ o_sig,
                                int32_t* __restrict__ o_cell, int32_t* __restrict__ o_ell) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = perm[i];
        const double ti = t_t[j];
        o_t[i] = ti;
        o_eta[i] = t_eta[j];
        o_sig[i] = t_sig[j];
        o_cell[i] = t_cellfov[j];
        o_ell[i] = left_index(knots, N, ti);
    }
}

// off[i] = first position whose key >= i (keys sorted), i in [0, m].
__global__ void k_offsets_int(int64_t n, const int32_t* __restrict__ keys, int64_t m, int64_t* __restrict__ off) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        off[i] = lo;
    }
}

// Knot-interval offsets: interval j (left index j + 3) starts at the first
// observation with t >= tau_{j+3}; the last interval ends at n (it also holds
// t = tau_N).
__global__ void k_offsets_time(int64_t n, const double* __restrict__ t, const double* __restrict__ knots, int64_t K,
                               int64_t* __restrict__ off) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= K; j += (int64_t)gridDim.x * blockDim.x) {
        if (j == 0) {
            off[0] = 0;
            continue;
        }
        if (j == K) {
            off[K] = n;
            continue;
        }
        const double tau = knots[j + 3];
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (t[mid] < tau) lo = mid + 1;
            else hi = mid;
        }
        off[j] = lo;
    }
}

// Calibration cell of each field of view within each knot interval (across-
// scan observations, pseudo-cell n_cells, have none); flags intervals whose
// observations of one field of view span several cells.
__global__ void k_interval_cells(int64_t K, const int64_t* __restrict__ off, const int32_t* __restrict__ cellfov,
                                 int32_t n_cells, int32_t* __restrict__ iv_cell, int* __restrict__ flags) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < K; j += (int64_t)gridDim.x * blockDim.x) {
        int32_t cp = -1, cf = -1;
        int bad = 0;
        for (int64_t l = off[j]; l < off[j + 1]; ++l) {
            const int32_t cv = cellfov[l];
            const int32_t cell = cv >> 1;
            if (cell >= n_cells) continue;
            if (cv & 1) {
                if (cf < 0) cf = cell;
                else if (cf != cell) bad = 1;
            } else {
                if (cp < 0) cp = cell;
                else if (cp != cell) bad = 1;
            }
        }
        iv_cell[2 * j] = cp;
        iv_cell[2 * j + 1] = cf;
        if (bad) atomicOr(flags, 64);
    }
}

void grid1d(int64_t n, int& blocks, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    blocks = (int)b;
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

int build_store(agis_ctx* ctx, const agis_obs_soa_t* obs, int where) {
    const int64_t n = obs->n;
    hipStream_t st = ctx->stream;
    // device copies of the inputs (or the caller's device pointers)
    double *t_in = nullptr, *eta_in = nullptr;
    float* sig_in = nullptr;
    int32_t *src_in = nullptr, *cell_in = nullptr;
    int8_t* fov_in = nullptr;
    std::vector<void*> tmp;
    struct Guard {
        std::vector<void*>* v;
        ~Guard() {
            for (void* p : *v) (void)hipFree(p);
        }
    } guard{&tmp};
    if (where == AGIS_HOST) {
        ALLOC(t_in, n, "t");
        tmp.push_back(t_in);
        ALLOC(eta_in, n, "eta_obs");
        tmp.push_back(eta_in);
        ALLOC(sig_in, n, "sigma");
        tmp.push_back(sig_in);
        ALLOC(src_in, n, "src");
        tmp.push_back(src_in);
        ALLOC(fov_in, n, "fov");
        tmp.push_back(fov_in);
        ALLOC(cell_in, n, "cell");
        tmp.push_back(cell_in);
        HIPCHK(hipMemcpyAsync(t_in, obs->t, n * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(eta_in, obs->eta_obs, n * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sig_in, obs->sigma, n * sizeof(float), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(src_in, obs->src, n * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(fov_in, obs->fov, n * sizeof(int8_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(cell_in, obs->cell, n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    } else {
        t_in = const_cast<double*>(obs->t);
        eta_in = const_cast<double*>(obs->eta_obs);
        sig_in = const_cast<float*>(obs->sigma);
        src_in = const_cast<int32_t*>(obs->src);
        fov_in = const_cast<int8_t*>(obs->fov);
        cell_in = const_cast<int32_t*>(obs->cell);
    }
    int* flags = nullptr;
    ALLOC(flags, 1, "flags");
    tmp.push_back(flags);
    HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), st));
    int blocks;
    grid1d(n, blocks);
    k_validate<<<blocks, 256, 0, st>>>(n, t_in, eta_in, sig_in, src_in, fov_in, cell_in, ctx->n_src, ctx->n_cells,
                                       ctx->h_knots[3], ctx->h_knots[ctx->N], flags);
    HIPCHK(hipGetLastError());
    int hflags = 0;
    HIPCHK(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->has_ac = (hflags & HAS_AC) != 0;
    hflags &= ~HAS_AC;
    if (hflags) {
        std::string m = "invalid observations:";
        if (hflags & BAD_SRC) m += " src outside [0, n_src);";
        if (hflags & BAD_CELL) m += " cell outside [0, n_cells) and not -1;";
        if (hflags & BAD_FOV) m += " fov not +1/-1;";
        if (hflags & BAD_T) m += " t outside [tau_3, tau_N];";
        if (hflags & BAD_SIGMA) m += " sigma not positive and finite;";
        if (hflags & BAD_ETA) m += " eta_obs not finite;";
        return set_error(ctx, (hflags & (BAD_SIGMA | BAD_ETA)) ? AGIS_E_NUMERIC : AGIS_E_RANGE, m);
    }

    // ---- time order (stable radix sort of t with the input index) ----
    int32_t *iota = nullptr, *perm_t = nullptr;
    ALLOC(iota, n, "iota");
    tmp.push_back(iota);
    ALLOC(ctx->t_perm, n, "t_perm");
    perm_t = ctx->t_perm;
    ALLOC(ctx->t_t, n, "t_t");
    k_iota<<<blocks, 256, 0, st>>>(n, iota);
    HIPCHK(hipGetLastError());
    size_t tb = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, t_in, ctx->t_t, iota, perm_t, (int)n, 0, 64, st));
    size_t tb2 = 0;
    int32_t* keys_src = nullptr;  // time-ordered source keys, sorted below
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, keys_src, keys_src, iota, iota, (int)n, 0, 32, st));
    void* temp = nullptr;
    const size_t tbytes = std::max(tb, tb2);
    {
        int rc = dalloc(ctx, (char**)&temp, tbytes, "sort workspace");
        if (rc != AGIS_OK) return rc;
    }
    tmp.push_back(temp);
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(temp, tb, t_in, ctx->t_t, iota, perm_t, (int)n, 0, 64, st));
    ALLOC(ctx->t_eta, n, "t_eta");
    ALLOC(ctx->t_sig, n, "t_sig");
    ALLOC(ctx->t_src, n, "t_src");
    ALLOC(ctx->t_cellfov, n, "t_cellfov");
    k_gather_time<<<blocks, 256, 0, st>>>(n, perm_t, eta_in, sig_in, src_in, fov_in, cell_in, (int32_t)ctx->n_cells,
                                          ctx->t_eta,
                                          ctx->t_sig, ctx->t_src, ctx->t_cellfov);
    HIPCHK(hipGetLastError());

    // ---- (source, time) order: stable sort of the time order by source ----
    int32_t* src_sorted = nullptr;
    ALLOC(src_sorted, n, "src_sorted");
    tmp.push_back(src_sorted);
    ALLOC(ctx->s_from_t, n, "s_from_t");          // kept: gathers time-ordered columns into source order
    int32_t* perm_s = ctx->s_from_t;
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < ctx->n_src) ++bits;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(temp, tb2, ctx->t_src, src_sorted, iota, perm_s, (int)n, 0, bits, st));
    ALLOC(ctx->s_t, n, "s_t");
    ALLOC(ctx->s_eta, n, "s_eta");
    ALLOC(ctx->s_sig, n, "s_sig");
    ALLOC(ctx->s_cell, n, "s_cell");
    ALLOC(ctx->s_ell, n, "s_ell");
    k_gather_source<<<blocks, 256, 0, st>>>(n, perm_s, ctx->t_t, ctx->t_eta, ctx->t_sig, ctx->t_cellfov, ctx->knots,
                                            ctx->N, ctx->s_t, ctx->s_eta, ctx->s_sig, ctx->s_cell, ctx->s_ell);
    HIPCHK(hipGetLastError());
    ALLOC(ctx->src_off, ctx->n_src + 1, "src_off");
    int b2;
    grid1d(ctx->n_src + 1, b2);
    k_offsets_int<<<b2, 256, 0, st>>>(n, src_sorted, ctx->n_src, ctx->src_off);
    HIPCHK(hipGetLastError());

    // ---- knot intervals and their calibration cells ----
    ALLOC(ctx->iv_off, ctx->K + 1, "iv_off");
    grid1d(ctx->K + 1, b2);
    k_offsets_time<<<b2, 256, 0, st>>>(n, ctx->t_t, ctx->knots, ctx->K, ctx->iv_off);
    HIPCHK(hipGetLastError());
    ALLOC(ctx->iv_cell, 2 * ctx->K, "iv_cell");
    HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), st));
    k_interval_cells<<<b2, 256, 0, st>>>(ctx->K, ctx->iv_off, ctx->t_cellfov, (int32_t)ctx->n_cells, ctx->iv_cell,
                                         flags);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> h_ivc(2 * ctx->K);
    HIPCHK(hipMemcpyAsync(h_ivc.data(), ctx->iv_cell, 2 * ctx->K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflags)
        return set_error(ctx, AGIS_E_SHAPE,
                         "observations of one field of view within one knot interval belong to different cells");
    // each cell must cover one contiguous run of intervals
    std::vector<int32_t> h_civ(2 * ctx->n_cells, -1);
    std::vector<int32_t> last_seen(ctx->n_cells, -2);
    for (int64_t j = 0; j < ctx->K; ++j) {
        for (int f = 0; f < 2; ++f) {
            const int32_t c = h_ivc[2 * j + f];
            if (c < 0) continue;
            if (h_civ[2 * c] < 0) {
                h_civ[2 * c] = (int32_t)j;
            } else if (last_seen[c] != (int32_t)j - 1 && last_seen[c] != (int32_t)j) {
                // gap: only allowed if every interval in between has no
                // observation of that cell's field of view
                for (int64_t jj = last_seen[c] + 1; jj < j; ++jj) {
                    if (h_ivc[2 * jj + f] >= 0 && h_ivc[2 * jj + f] != c)
                        return set_error(ctx, AGIS_E_SHAPE, "a calibration cell covers non-contiguous knot intervals");
                }
            }
            last_seen[c] = (int32_t)j;
            h_civ[2 * c + 1] = (int32_t)j + 1;
        }
    }
    for (int64_t c = 0; c < ctx->n_cells; ++c) {
        if (h_civ[2 * c] < 0) {
            h_civ[2 * c] = 0;
            h_civ[2 * c + 1] = 0;
        }
    }
    ALLOC(ctx->cell_iv, 2 * ctx->n_cells, "cell_iv");
    HIPCHK(hipMemcpyAsync(ctx->cell_iv, h_civ.data(), 2 * ctx->n_cells * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return AGIS_OK;
}

}  // namespace agis
