// Learned extrapolation of the simple iteration.  This is not part of the
// paper's method; it builds on the observation behind the accelerated simple
// iteration (Sect. 4.7): the updates decay geometrically along the slowest
// eigenvectors of the iteration.  Per source and per attitude coefficient a
// small MLP maps the last four recorded updates (normalised by their RMS)
// and two descriptors to four mixing coefficients c; the candidate is
// x + sum_k c_k u_k over the recorded updates u_k (newest first), a step
// inside the span of the recent updates, which late in the iteration is the
// slow subspace.  The gate that keeps or drops a candidate is host logic.
//
//   k_hist_record_*   push (current - anchor) into a ring of four updates
//   k_features_*      per unit: 20 (sources) or 16 (coefficients) normalised
//                     update values, two descriptors, the normalisation scale
//   k_mlp_forward     F -> 64 -> 64 -> 4, tanh hidden layers, weights rounded
//                     to BF16, FP32 accumulation; one thread per sample
//   k_mlp_grad        one block per 128 samples: layer vectors staged in LDS,
//                     backward pass, the block's weight-gradient sums in a
//                     fixed order
//   k_grad_reduce     sum of the block gradients in block order
//   k_adam            Adam on FP32 master weights and their BF16 copies
//   k_apply_*         candidate x + sum_k c_k u_k
//   k_chi2_partial    sum of W R^2 per knot interval block (time order)
#include "agis_internal.h"
#include "source_block.h"

namespace agis {

namespace {

constexpr int HID = 64;
constexpr int NH = 4;                   // recorded updates = mixing coefficients (network outputs)
constexpr int GB = 128;                 // samples per gradient block

template <int F, int O>
struct MlpShape {
    static constexpr int W1 = 0;
    static constexpr int B1 = HID * F;
    static constexpr int W2 = B1 + HID;
    static constexpr int B2 = W2 + HID * HID;
    static constexpr int W3 = B2 + HID;
    static constexpr int B3 = W3 + O * HID;
    static constexpr int NW = B3 + O;
};

// FP32 -> nearest BF16 (ties to even), returned as FP32
__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    return __builtin_bit_cast(float, u);
}

// ------------------------------------------------------------ histories
__global__ void k_hist_record_src(int64_t n, const double* __restrict__ s, double* __restrict__ anchor,
                                  double* __restrict__ ring, int slot) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double* x = s + 5 * i;
        double* a = anchor + 5 * i;
        double* r = ring + (int64_t)slot * 5 * n + 5 * i;
        r[0] = (x[0] - a[0]) * cos(x[1]);      // d alpha* = d alpha cos delta
        for (int c = 1; c < 5; ++c) r[c] = x[c] - a[c];
        for (int c = 0; c < 5; ++c) a[c] = x[c];
    }
}

__global__ void k_hist_record_att(int64_t n4, const double* __restrict__ a, double* __restrict__ anchor,
                                  double* __restrict__ ring, int slot) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        ring[(int64_t)slot * n4 + i] = a[i] - anchor[i];
        anchor[i] = a[i];
    }
}

// newest update first: ring slot (count - 1 - h) mod 4
__device__ __forceinline__ int ring_slot(int count, int h) { return ((count - 1 - h) % 4 + 4) % 4; }

__global__ void k_copy(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_features_src(int64_t n, const double* __restrict__ ring, int count, const double* __restrict__ s,
                               const int64_t* __restrict__ off, double sin_obl, double cos_obl,
                               float* __restrict__ X, float* __restrict__ scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double h[20];
        double ss = 0.0;
        for (int k = 0; k < 4; ++k) {
            const int slot = ring_slot(count, k);
            for (int c = 0; c < 5; ++c) {
                h[5 * k + c] = ring[(int64_t)slot * 5 * n + 5 * i + c];
                ss += h[5 * k + c] * h[5 * k + c];
            }
        }
        const double sc = sqrt(ss / 20.0);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        float* x = X + 22 * i;
        for (int e = 0; e < 20; ++e) x[e] = (float)(h[e] * inv);
        x[20] = (float)(log((double)(off[i + 1] - off[i]) + 1.0) / 5.0);
        // sine of the ecliptic latitude: r . (ecliptic pole in ICRS)
        const double al = s[5 * i], de = s[5 * i + 1];
        x[21] = (float)(-sin_obl * cos(de) * sin(al) + cos_obl * sin(de));
        scale[i] = (float)sc;
    }
}

__global__ void k_features_att(int64_t n, const double* __restrict__ ring, int count, const double* __restrict__ a,
                               float* __restrict__ X, float* __restrict__ scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double h[16];
        double ss = 0.0;
        for (int k = 0; k < 4; ++k) {
            const int slot = ring_slot(count, k);
            for (int c = 0; c < 4; ++c) {
                h[4 * k + c] = ring[(int64_t)slot * 4 * n + 4 * i + c];
                ss += h[4 * k + c] * h[4 * k + c];
            }
        }
        const double sc = sqrt(ss / 16.0);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        float* x = X + 18 * i;
        for (int e = 0; e < 16; ++e) x[e] = (float)(h[e] * inv);
        // spin phase: twice the angle of the coefficient about its z axis
        const double ph = 2.0 * atan2(a[4 * i + 2], a[4 * i + 3]);
        x[16] = (float)sin(ph);
        x[17] = (float)cos(ph);
        scale[i] = (float)sc;
    }
}

// ------------------------------------------------------------------- MLP
template <int F, int O>
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t n, const float* __restrict__ wb,
                                                     const float* __restrict__ X, float* __restrict__ Y) {
    using S = MlpShape<F, O>;
    __shared__ float w[S::NW];
    for (int e = threadIdx.x; e < S::NW; e += blockDim.x) w[e] = wb[e];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[F], h1[HID], y[O];
#pragma unroll
    for (int k = 0; k < F; ++k) x[k] = X[F * i + k];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        float acc = w[S::B1 + j];
#pragma unroll
        for (int k = 0; k < F; ++k) acc += w[S::W1 + j * F + k] * x[k];
        h1[j] = tanhf(acc);
    }
#pragma unroll
    for (int o = 0; o < O; ++o) y[o] = w[S::B3 + o];
    for (int j = 0; j < HID; ++j) {
        float acc = w[S::B2 + j];
#pragma unroll
        for (int k = 0; k < HID; ++k) acc += w[S::W2 + j * HID + k] * h1[k];
        const float h2 = tanhf(acc);
#pragma unroll
        for (int o = 0; o < O; ++o) y[o] += w[S::W3 + o * HID + j] * h2;
    }
#pragma unroll
    for (int o = 0; o < O; ++o) Y[O * i + o] = y[o];
}

// Gradient of L = sum over the batch of |yhat - t|^2 / (2 n_batch), with
// yhat_c = sum_k c_k x[k NC + c] the mixture of the sample's normalised
// updates by the network outputs c (t has NC columns): block b takes batch
// entries [b GB, (b + 1) GB); entry e is sample idx[e] (or e when idx is
// null).  part[b] receives the block's weight-gradient sums followed by its
// share of L.
template <int F, int O, int NC>
__global__ __launch_bounds__(GB) void k_mlp_grad(int64_t n_batch, const int64_t* __restrict__ idx,
                                                 const float* __restrict__ wb, const float* __restrict__ X,
                                                 const float* __restrict__ T, float* __restrict__ part) {
    using S = MlpShape<F, O>;
    __shared__ float w[S::NW];
    __shared__ float sx[GB][F + 1];
    __shared__ float s1[GB][HID + 1];     // h1, then delta1
    __shared__ float s2[GB][HID + 1];     // h2, then delta2
    __shared__ float sd[GB][O + 1];       // dL/dc
    __shared__ float sl[GB];
    for (int e = threadIdx.x; e < S::NW; e += blockDim.x) w[e] = wb[e];
    const int b = threadIdx.x;
    const int64_t e0 = blockIdx.x * (int64_t)GB + b;
    const bool valid = e0 < n_batch;
    const float inv_n = 1.0f / (float)n_batch;
    const int64_t i = valid ? (idx ? idx[e0] : e0) : 0;
    for (int k = 0; k < F; ++k) sx[b][k] = valid ? X[F * i + k] : 0.0f;
    __syncthreads();
    // forward, one sample per thread
    for (int j = 0; j < HID; ++j) {
        float acc = w[S::B1 + j];
        for (int k = 0; k < F; ++k) acc += w[S::W1 + j * F + k] * sx[b][k];
        s1[b][j] = tanhf(acc);
    }
    for (int j = 0; j < HID; ++j) {
        float acc = w[S::B2 + j];
        for (int k = 0; k < HID; ++k) acc += w[S::W2 + j * HID + k] * s1[b][k];
        s2[b][j] = tanhf(acc);
    }
    static_assert(O * NC <= F, "the first O NC features are the normalised updates");
    float cf[O];
    for (int o = 0; o < O; ++o) {
        float acc = w[S::B3 + o];
        for (int k = 0; k < HID; ++k) acc += w[S::W3 + o * HID + k] * s2[b][k];
        cf[o] = acc;
    }
    float l = 0.0f, r[NC];
    for (int c = 0; c < NC; ++c) {
        float yh = 0.0f;
        for (int o = 0; o < O; ++o) yh += cf[o] * sx[b][o * NC + c];
        r[c] = valid ? yh - T[NC * i + c] : 0.0f;
        l += r[c] * r[c];
    }
    for (int o = 0; o < O; ++o) {
        float acc = 0.0f;
        for (int c = 0; c < NC; ++c) acc += r[c] * sx[b][o * NC + c];
        sd[b][o] = acc * inv_n;
    }
    sl[b] = 0.5f * l * inv_n;
    __syncthreads();
    float* out = part + (int64_t)blockIdx.x * (S::NW + 1);
    // dW3 = sum_b dy h2', db3 = sum_b dy
    for (int e = threadIdx.x; e < O * HID + O; e += blockDim.x) {
        float acc = 0.0f;
        if (e < O * HID) {
            const int o = e / HID, k = e % HID;
            for (int q = 0; q < GB; ++q) acc += sd[q][o] * s2[q][k];
            out[S::W3 + e] = acc;
        } else {
            const int o = e - O * HID;
            for (int q = 0; q < GB; ++q) acc += sd[q][o];
            out[S::B3 + o] = acc;
        }
    }
    __syncthreads();
    // delta2 = (W3' dy) * (1 - h2^2), in place of h2
    for (int k = 0; k < HID; ++k) {
        float acc = 0.0f;
#pragma unroll
        for (int o = 0; o < O; ++o) acc += w[S::W3 + o * HID + k] * sd[b][o];
        s2[b][k] = acc * (1.0f - s2[b][k] * s2[b][k]);   // each entry reads only itself
    }
    __syncthreads();
    // dW2 = sum_b delta2 h1', db2 = sum_b delta2
    for (int e = threadIdx.x; e < HID * HID + HID; e += blockDim.x) {
        float acc = 0.0f;
        if (e < HID * HID) {
            const int j = e / HID, k = e % HID;
            for (int q = 0; q < GB; ++q) acc += s2[q][j] * s1[q][k];
            out[S::W2 + e] = acc;
        } else {
            const int j = e - HID * HID;
            for (int q = 0; q < GB; ++q) acc += s2[q][j];
            out[S::B2 + j] = acc;
        }
    }
    __syncthreads();
    // delta1 = (W2' delta2) * (1 - h1^2), in place of h1
    for (int k = 0; k < HID; ++k) {
        float acc = 0.0f;
        for (int j = 0; j < HID; ++j) acc += w[S::W2 + j * HID + k] * s2[b][j];
        s1[b][k] = acc * (1.0f - s1[b][k] * s1[b][k]);   // s2 (delta2) is not written here
    }
    __syncthreads();
    // dW1 = sum_b delta1 x', db1 = sum_b delta1
    for (int e = threadIdx.x; e < HID * F + HID; e += blockDim.x) {
        float acc = 0.0f;
        if (e < HID * F) {
            const int j = e / F, k = e % F;
            for (int q = 0; q < GB; ++q) acc += s1[q][j] * sx[q][k];
            out[S::W1 + e] = acc;
        } else {
            const int j = e - HID * F;
            for (int q = 0; q < GB; ++q) acc += s1[q][j];
            out[S::B1 + j] = acc;
        }
    }
    if (threadIdx.x == 0) {
        float acc = 0.0f;
        for (int q = 0; q < GB; ++q) acc += sl[q];
        out[S::NW] = acc;
    }
}

// g[e] = sum over blocks (in block order) of part[block][e], e <= nw
__global__ void k_grad_reduce(int64_t n_blocks, int nw, const float* __restrict__ part, float* __restrict__ g) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e <= nw; e += gridDim.x * blockDim.x) {
        float acc = 0.0f;
        for (int64_t q = 0; q < n_blocks; ++q) acc += part[q * (nw + 1) + e];
        g[e] = acc;
    }
}

// Adam (Kingma & Ba) with bias correction; t >= 1
__global__ void k_adam(int nw, const float* __restrict__ g, float* __restrict__ wm, float* __restrict__ m1,
                       float* __restrict__ m2, float* __restrict__ wb, float lr, float beta1, float beta2, float eps,
                       int t) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nw) return;
    const float ge = g[e];
    const float a = beta1 * m1[e] + (1.0f - beta1) * ge;
    const float v = beta2 * m2[e] + (1.0f - beta2) * ge * ge;
    m1[e] = a;
    m2[e] = v;
    const float ah = a / (1.0f - powf(beta1, (float)t));
    const float vh = v / (1.0f - powf(beta2, (float)t));
    const float nv = wm[e] - lr * ah / (sqrtf(vh) + eps);
    wm[e] = nv;
    wb[e] = bf16_round(nv);
}

__global__ void k_round_weights(int nw, const float* __restrict__ wm, float* __restrict__ wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nw) wb[e] = bf16_round(wm[e]);
}

// Minibatch indices: a counter-based hash (SplitMix64) of (seed, step, entry)
__global__ void k_batch_idx(int64_t nb, int64_t n, uint64_t seed, uint64_t step, int64_t* __restrict__ idx) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nb) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (step * 0x100000001ull + (uint64_t)e + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    idx[e] = (int64_t)(z % (uint64_t)n);
}

// ------------------------------------------------------------ candidate
__global__ void k_apply_src(int64_t n, const float* __restrict__ C, const double* __restrict__ ring, int count,
                            double* __restrict__ s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int h = 0; h < NH; ++h) {
            const double ch = (double)C[NH * i + h];
            const double* u = ring + (int64_t)ring_slot(count, h) * 5 * n + 5 * i;
            for (int c = 0; c < 5; ++c) d[c] += ch * u[c];
        }
        double* x = s + 5 * i;
        x[0] += d[0] / cos(x[1]);            // d alpha* -> d alpha
        for (int c = 1; c < 5; ++c) x[c] += d[c];
    }
}

__global__ void k_apply_att(int64_t n, const float* __restrict__ C, const double* __restrict__ ring, int count,
                            double* __restrict__ a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 4 * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / 4;
        double d = 0.0;
        for (int h = 0; h < NH; ++h) d += (double)C[NH * j + h] * ring[(int64_t)ring_slot(count, h) * 4 * n + i];
        a[i] += d;
    }
}

// ------------------------------------------------- accelerated iteration
// Sums over the sources i = 0, stride, 2 stride, ... of u1 u2 and u2 u2,
// u1 and u2 the parallax updates of the newest and the previous record;
// block b takes subset entries [256 b, 256 (b + 1)) and writes part[2 b],
// part[2 b + 1] (fixed order: wave sums, then the four waves in order).
__global__ __launch_bounds__(256) void k_asi_partial(int64_t n, int stride, const double* __restrict__ ring, int count,
                                                     double* __restrict__ part) {
    __shared__ double red[2][4];
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
    const int64_t i = e * stride;
    double xy = 0.0, yy = 0.0;
    if (i < n) {
        const double u1 = ring[(int64_t)ring_slot(count, 0) * 5 * n + 5 * i + 2];
        const double u2 = ring[(int64_t)ring_slot(count, 1) * 5 * n + 5 * i + 2];
        xy = u1 * u2;
        yy = u2 * u2;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        xy += __shfl_xor(xy, m, 64);
        yy += __shfl_xor(yy, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = xy;
        red[1][threadIdx.x >> 6] = yy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        part[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

__global__ void k_sum_partial2(int64_t nb, const double* __restrict__ part, double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int64_t q = 0; q < nb; ++q) {
        a += part[2 * q];
        b += part[2 * q + 1];
    }
    out[0] = a;
    out[1] = b;
}

// x <- x + f u1 (u1 the newest recorded update)
__global__ void k_asi_apply_src(int64_t n, const double* __restrict__ ring, int count, double f,
                                double* __restrict__ s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double* u = ring + (int64_t)ring_slot(count, 0) * 5 * n + 5 * i;
        double* x = s + 5 * i;
        x[0] += f * u[0] / cos(x[1]);        // d alpha* -> d alpha
        for (int c = 1; c < 5; ++c) x[c] += f * u[c];
    }
}

__global__ void k_asi_apply_vec(int64_t n, const double* __restrict__ ring, int count, double f,
                                double* __restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] += f * ring[(int64_t)ring_slot(count, 0) * n + i];
}

// sum of W R^2 over the observations of knot intervals [b * 64, (b + 1) * 64)
__global__ __launch_bounds__(64) void k_chi2_partial(DevConsts k, int64_t K, const int64_t* __restrict__ iv_off,
                                                     const double* __restrict__ ot, const double* __restrict__ oeta,
                                                     const float* __restrict__ osig,
                                                     const int32_t* __restrict__ ocellfov,
                                                     const int32_t* __restrict__ osrc,
                                                     const SrcPrep* __restrict__ prep,
                                                     const double* __restrict__ knots,
                                                     const KnotTab* __restrict__ ktab, const double* __restrict__ a,
                                                     const double* __restrict__ c, double* __restrict__ part) {
    const int lane = threadIdx.x;
    double acc = 0.0;
    const int64_t j0 = (int64_t)blockIdx.x * 64, j1 = j0 + 64 < K ? j0 + 64 : K;
    for (int64_t j = j0; j < j1; ++j) {
        const KnotTab kt = ktab[j];
        for (int64_t l = iv_off[j] + lane; l < iv_off[j + 1]; l += 64) {
            const SrcPrep sp = prep[osrc[l]];
            const int32_t cf = ocellfov[l];
            ObsEval o;
            observe(k, ot[l], oeta[l], c[cf >> 1], sp.r, sp.mu, sp.plx, a + 4 * j, knots + (j + 1), kt, o,
                    cf >= k.ac_cf0);
            const double sg = (double)osig[l];
            acc += o.R * o.R / (sg * sg);
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) part[blockIdx.x] = acc;
}

__global__ void k_sum_partial(int64_t n, const double* __restrict__ part, double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double acc = 0.0;
    for (int64_t q = 0; q < n; ++q) acc += part[q];
    out[0] = acc;
}

inline unsigned blocks_for(int64_t n, int t = 256) {
    int64_t b = (n + t - 1) / t;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

}  // namespace

// --------------------------------------------------------------- launchers
int mlp_num_weights(int which) { return which == 0 ? MlpShape<22, NH>::NW : MlpShape<18, NH>::NW; }
int mlp_num_inputs(int which) { return which == 0 ? 22 : 18; }
int mlp_num_outputs(int) { return NH; }
int mlp_num_targets(int which) { return which == 0 ? 5 : 4; }

void launch_hist_record(agis_ctx* ctx, int slot) {
    k_hist_record_src<<<blocks_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->n_src, ctx->s, ctx->lh_anchor_s,
                                                                        ctx->lh_ring_s, slot);
    k_hist_record_att<<<blocks_for(4 * ctx->N), 256, 0, ctx->stream>>>(4 * ctx->N, ctx->a, ctx->lh_anchor_a,
                                                                        ctx->lh_ring_a, slot);
    if (ctx->n_cells > 0)
        k_hist_record_att<<<blocks_for(ctx->n_cells), 256, 0, ctx->stream>>>(ctx->n_cells, ctx->c, ctx->lh_anchor_c,
                                                                              ctx->lh_ring_c, slot);
}

void launch_hist_anchor(agis_ctx* ctx) {
    k_copy<<<blocks_for(5 * ctx->n_src), 256, 0, ctx->stream>>>(5 * ctx->n_src, ctx->s, ctx->lh_anchor_s);
    k_copy<<<blocks_for(4 * ctx->N), 256, 0, ctx->stream>>>(4 * ctx->N, ctx->a, ctx->lh_anchor_a);
    k_copy<<<blocks_for(ctx->n_cells), 256, 0, ctx->stream>>>(ctx->n_cells, ctx->c, ctx->lh_anchor_c);
}

void launch_asi_sums(agis_ctx* ctx, int stride, double* part, double* out) {
    const int64_t n_sub = (ctx->n_src + stride - 1) / stride;
    const int64_t nb = std::max<int64_t>((n_sub + 255) / 256, 1);
    k_asi_partial<<<(unsigned)nb, 256, 0, ctx->stream>>>(ctx->n_src, stride, ctx->lh_ring_s, ctx->lh_count, part);
    k_sum_partial2<<<1, 64, 0, ctx->stream>>>(nb, part, out);
}

void launch_asi_apply(agis_ctx* ctx, double f) {
    k_asi_apply_src<<<blocks_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->n_src, ctx->lh_ring_s, ctx->lh_count, f,
                                                                      ctx->s);
    k_asi_apply_vec<<<blocks_for(4 * ctx->N), 256, 0, ctx->stream>>>(4 * ctx->N, ctx->lh_ring_a, ctx->lh_count, f,
                                                                      ctx->a);
    if (ctx->n_cells > 0)
        k_asi_apply_vec<<<blocks_for(ctx->n_cells), 256, 0, ctx->stream>>>(ctx->n_cells, ctx->lh_ring_c,
                                                                            ctx->lh_count, f, ctx->c);
}

void launch_features(agis_ctx* ctx, int which, float* X, float* scale) {
    if (which == 0)
        k_features_src<<<blocks_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->n_src, ctx->lh_ring_s, ctx->lh_count,
                                                                         ctx->s, ctx->src_off, ctx->k.sin_obl,
                                                                         ctx->k.cos_obl, X, scale);
    else
        k_features_att<<<blocks_for(ctx->N), 256, 0, ctx->stream>>>(ctx->N, ctx->lh_ring_a, ctx->lh_count, ctx->a, X,
                                                                     scale);
}

void launch_mlp_forward(agis_ctx* ctx, int which, int64_t n, const float* X, float* Y) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (n == 0) return;
    if (which == 0) k_mlp_forward<22, NH><<<g, 256, 0, ctx->stream>>>(n, ctx->mlp_wb[0], X, Y);
    else k_mlp_forward<18, NH><<<g, 256, 0, ctx->stream>>>(n, ctx->mlp_wb[1], X, Y);
}

// batch gradient into ctx->mlp_g[which] (last entry: loss); part must hold
// ceil(nb / 128) * (NW + 1) floats
void launch_mlp_grad(agis_ctx* ctx, int which, int64_t nb, const int64_t* idx, const float* X, const float* T,
                     float* part) {
    const int64_t blocks = (nb + GB - 1) / GB;
    const int nw = mlp_num_weights(which);
    if (which == 0)
        k_mlp_grad<22, NH, 5><<<(unsigned)blocks, GB, 0, ctx->stream>>>(nb, idx, ctx->mlp_wb[0], X, T, part);
    else
        k_mlp_grad<18, NH, 4><<<(unsigned)blocks, GB, 0, ctx->stream>>>(nb, idx, ctx->mlp_wb[1], X, T, part);
    k_grad_reduce<<<(unsigned)((nw + 256) / 256), 256, 0, ctx->stream>>>(blocks, nw, part, ctx->mlp_g[which]);
}

void launch_batch_idx(agis_ctx* ctx, int64_t nb, int64_t n, uint64_t seed, uint64_t step, int64_t* idx) {
    k_batch_idx<<<(unsigned)((nb + 255) / 256), 256, 0, ctx->stream>>>(nb, n, seed, step, idx);
}

void launch_adam(agis_ctx* ctx, int which, float lr, int t) {
    const int nw = mlp_num_weights(which);
    k_adam<<<(unsigned)((nw + 255) / 256), 256, 0, ctx->stream>>>(nw, ctx->mlp_g[which], ctx->mlp_w[which],
                                                                  ctx->mlp_m1[which], ctx->mlp_m2[which],
                                                                  ctx->mlp_wb[which], lr, 0.9f, 0.999f, 1e-8f, t);
}

void launch_round_weights(agis_ctx* ctx, int which) {
    const int nw = mlp_num_weights(which);
    k_round_weights<<<(unsigned)((nw + 255) / 256), 256, 0, ctx->stream>>>(nw, ctx->mlp_w[which],
                                                                           ctx->mlp_wb[which]);
}

void launch_apply_candidate(agis_ctx* ctx, const float* Cs, const float* Ca) {
    k_apply_src<<<blocks_for(ctx->n_src), 256, 0, ctx->stream>>>(ctx->n_src, Cs, ctx->lh_ring_s, ctx->lh_count,
                                                                  ctx->s);
    k_apply_att<<<blocks_for(4 * ctx->N), 256, 0, ctx->stream>>>(ctx->N, Ca, ctx->lh_ring_a, ctx->lh_count, ctx->a);
}

void launch_copy(agis_ctx* ctx, int64_t n, const double* src, double* dst) {
    k_copy<<<blocks_for(n), 256, 0, ctx->stream>>>(n, src, dst);
}

// sum W R^2 at the current parameters into *out (device)
void launch_chi2(agis_ctx* ctx, double* part, double* out) {
    const int64_t nb = (ctx->K + 63) / 64;
    if (nb == 0) return;
    k_chi2_partial<<<(unsigned)nb, 64, 0, ctx->stream>>>(ctx->k, ctx->K, ctx->iv_off, ctx->t_t, ctx->t_eta,
                                                         ctx->t_sig, ctx->t_cellfov, ctx->t_src, ctx->prep,
                                                         ctx->knots, ctx->ktab, ctx->a, ctx->c, part);
    k_sum_partial<<<1, 64, 0, ctx->stream>>>(nb, part, out);
}

}  // namespace agis
