// The learned pivot: a small network predicting, from statistics of a strided
// row sample, where the k-th smallest entry of a row lies, so that the first
// partition pass of the quick multi-select keeps just over k keys.  Kernels for
// features, inference, and training (forward/backward per sample, fixed-order
// weight-gradient sums, Adam on FP32 master weights with a BF16 copy), and the
// C ABI around them (weights in/out, file save/load).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "handle.hpp"
#include "internal.hpp"
#include "pivot_net.hpp"

namespace knn {

knn_status_t ensure_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg);

constexpr int kFeatThreads = 256;
// knn_pivot_train: batch size, initial learning rate and pinball quantile
constexpr int64_t kTrainBatch = 4096;
constexpr float kTrainLr = 2e-3f;
constexpr float kTrainQuantile = 0.99f;

// Features of each row: 4 sorted sample blocks merged in LDS, then one wave.
__global__ __launch_bounds__(kFeatThreads) void net_features_kernel(const float *__restrict__ D, int64_t rows,
                                                                    uint32_t N, int64_t ld, uint32_t k,
                                                                    float *__restrict__ feats,
                                                                    float *__restrict__ loc_scale) {
    __shared__ uint64_t keys[kNetSample];
    __shared__ float v[kNetSample];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const float *row = D + r * ld;
        const uint32_t j = net_sample_start(wave, N) + lane;
        keys[tid] = make_key(row[j], j);
        __syncthreads();
        block_sort<kFeatThreads>(keys, kNetSample);
        v[tid] = ord_to_float(key_ord(keys[tid]));
        __syncthreads();
        if (wave == 0) {
            float x[kNetIn], m, s;
            net_features(v, N, k, x, m, s);
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < kNetIn; ++i) feats[r * kNetIn + i] = x[i];
            }
            if (loc_scale && lane == 0) {
                loc_scale[2 * r] = m;
                loc_scale[2 * r + 1] = s;
            }
        }
        __syncthreads();
    }
}

// Standardised prediction for each feature row (one wave per row).
__global__ __launch_bounds__(256) void net_predict_kernel(const float *__restrict__ feats, int64_t rows,
                                                          const uint16_t *__restrict__ w, float *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (r >= rows) return;
    float x[kNetIn];
#pragma unroll
    for (int i = 0; i < kNetIn; ++i) x[i] = feats[r * kNetIn + i];
    const float y = net_forward_wave(w, x);
    if (lane_id() == 0) out[r] = y;
}

// Training, pass 1: one thread per sample, forward and backward through the
// network with the BF16-rounded weights `wr` (stored as FP32), FP32 arithmetic
// in a fixed order.  Writes the activations H1, H2 (B x 64), the back-propagated
// signals D1, D2 (B x 64), dL/dy_hat and the per-sample pinball loss.
__global__ __launch_bounds__(256) void net_fwd_bwd_kernel(const float *__restrict__ X, const float *__restrict__ y,
                                                          int64_t B, const float *__restrict__ wr, float q,
                                                          float *__restrict__ H1, float *__restrict__ H2,
                                                          float *__restrict__ D1, float *__restrict__ D2,
                                                          float *__restrict__ dy, float *__restrict__ lossv) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[kNetIn];
#pragma unroll
    for (int i = 0; i < kNetIn; ++i) x[i] = X[b * kNetIn + i];
    float *h1 = H1 + b * kNetHidden, *h2 = H2 + b * kNetHidden;
    float *d1 = D1 + b * kNetHidden, *d2 = D2 + b * kNetHidden;
    for (int j = 0; j < kNetHidden; ++j) {
        float z = wr[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kNetIn; ++i) z = fmaf(wr[kOffW1 + j * kNetIn + i], x[i], z);
        h1[j] = z > 0.f ? z : 0.f;
    }
    float yh = 0.f;
    for (int j = 0; j < kNetHidden; ++j) {
        float z = wr[kOffB2 + j];
        for (int i = 0; i < kNetHidden; ++i) z = fmaf(wr[kOffW2 + j * kNetHidden + i], h1[i], z);
        const float hj = z > 0.f ? z : 0.f;
        h2[j] = hj;
        yh = fmaf(wr[kOffW3 + j], hj, yh);
    }
    yh += wr[kOffB3];
    const float u = y[b] - yh;
    lossv[b] = u >= 0.f ? q * u : (q - 1.0f) * u;
    const float g = (u > 0.f ? -q : (u < 0.f ? 1.0f - q : 0.f)) / (float)B;
    dy[b] = g;
    for (int j = 0; j < kNetHidden; ++j) d2[j] = h2[j] > 0.f ? g * wr[kOffW3 + j] : 0.f;
    for (int i = 0; i < kNetHidden; ++i) {
        float s = 0.f;
        for (int j = 0; j < kNetHidden; ++j) s = fmaf(d2[j], wr[kOffW2 + j * kNetHidden + i], s);
        d1[i] = h1[i] > 0.f ? s : 0.f;
    }
}

// Training, pass 2: one thread per parameter, sum over the batch in sample
// order (deterministic).  Thread kNetParams writes the mean loss.
__global__ __launch_bounds__(256) void net_wgrad_kernel(const float *__restrict__ X, const float *__restrict__ H1,
                                                        const float *__restrict__ H2, const float *__restrict__ D1,
                                                        const float *__restrict__ D2, const float *__restrict__ dy,
                                                        const float *__restrict__ lossv, int64_t B,
                                                        float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNetParams) return;
    float s = 0.f;
    if (p == kNetParams) {
        for (int64_t b = 0; b < B; ++b) s += lossv[b];
        if (loss) *loss = s / (float)B;
        return;
    }
    if (p < kOffB1) {
        const int j = p / kNetIn, i = p % kNetIn;
        for (int64_t b = 0; b < B; ++b) s = fmaf(D1[b * kNetHidden + j], X[b * kNetIn + i], s);
    } else if (p < kOffW2) {
        const int j = p - kOffB1;
        for (int64_t b = 0; b < B; ++b) s += D1[b * kNetHidden + j];
    } else if (p < kOffB2) {
        const int j = (p - kOffW2) / kNetHidden, i = (p - kOffW2) % kNetHidden;
        for (int64_t b = 0; b < B; ++b) s = fmaf(D2[b * kNetHidden + j], H1[b * kNetHidden + i], s);
    } else if (p < kOffW3) {
        const int j = p - kOffB2;
        for (int64_t b = 0; b < B; ++b) s += D2[b * kNetHidden + j];
    } else if (p < kOffB3) {
        const int j = p - kOffW3;
        for (int64_t b = 0; b < B; ++b) s = fmaf(dy[b], H2[b * kNetHidden + j], s);
    } else {
        for (int64_t b = 0; b < B; ++b) s += dy[b];
    }
    grad[p] = s;
}

// Adam on the FP32 master weights, then the BF16 copy (and its FP32 image).
__global__ __launch_bounds__(256) void net_adam_kernel(float *__restrict__ theta, float *__restrict__ m,
                                                       float *__restrict__ v, const float *__restrict__ grad, float lr,
                                                       float b1, float b2, float eps, float c1, float c2,
                                                       float *__restrict__ theta_r, uint16_t *__restrict__ wbf) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNetParams) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float t = theta[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    theta[p] = t;
    const uint16_t bf = f32_to_bf16(t);
    wbf[p] = bf;
    theta_r[p] = bf16_to_f32(bf);
}

__global__ __launch_bounds__(256) void net_round_kernel(const float *__restrict__ theta, float *__restrict__ theta_r,
                                                        uint16_t *__restrict__ wbf) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNetParams) return;
    const uint16_t bf = f32_to_bf16(theta[p]);
    wbf[p] = bf;
    theta_r[p] = bf16_to_f32(bf);
}

// ---- training examples and the training loop -----------------------------------
// Counter-based 64-bit mixer (SplitMix64, Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Examples from `rows` rows: the standardised target y = (v_k - m) / s from the
// row's exact k-th smallest value v_k and its sample location and scale (m, s);
// rows whose features or target are not finite are dropped.  The kept rows are
// appended in row order at ex_x / ex_y + base (one workgroup: per chunk of 256
// rows, wave ballots and an LDS prefix give each kept row its slot), and their
// number is written to *kept.
__global__ __launch_bounds__(256) void net_examples_kernel(const float *__restrict__ feats,
                                                           const float *__restrict__ loc_scale,
                                                           const float *__restrict__ vals, int64_t rows, int k,
                                                           float *__restrict__ ex_x, float *__restrict__ ex_y,
                                                           int64_t base, uint32_t *__restrict__ kept) {
    __shared__ uint32_t wcount[4];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    uint32_t total = 0;
    for (int64_t r0 = 0; r0 < rows; r0 += 256) {
        const int64_t r = r0 + tid;
        bool ok = r < rows;
        float x[kNetIn], y = 0.f;
        if (ok) {
#pragma unroll
            for (int i = 0; i < kNetIn; ++i) {
                x[i] = feats[r * kNetIn + i];
                ok = ok && fabsf(x[i]) <= 3.4028235e38f;
            }
            y = (vals[r * k + k - 1] - loc_scale[2 * r]) / loc_scale[2 * r + 1];
            ok = ok && fabsf(y) <= 3.4028235e38f;
        }
        const uint64_t m = __ballot(ok);
        if (lane == 0) wcount[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = total;
        for (uint32_t w = 0; w < wave; ++w) before += wcount[w];
        if (ok) {
            const int64_t o = base + before + lanes_below(m);
#pragma unroll
            for (int i = 0; i < kNetIn; ++i) ex_x[o * kNetIn + i] = x[i];
            ex_y[o] = y;
        }
        total += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
    if (tid == 0) *kept = total;
}

// He initialisation from the seed: W1 ~ N(0, 2/8), W2 ~ N(0, 2/64), w3 ~ N(0,
// 1/64), biases 0; each weight a Box-Muller normal from two counter-based
// uniforms of (seed, parameter index).  Clears the Adam moments.
__global__ __launch_bounds__(256) void net_init_kernel(uint64_t seed, float *__restrict__ theta, float *__restrict__ m,
                                                       float *__restrict__ v) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNetParams) return;
    m[p] = 0.f;
    v[p] = 0.f;
    double sd = 0.0;
    if (p < kOffB1) sd = sqrt(2.0 / kNetIn);
    else if (p >= kOffW2 && p < kOffB2) sd = sqrt(2.0 / kNetHidden);
    else if (p >= kOffW3 && p < kOffB3) sd = sqrt(1.0 / kNetHidden);
    float w = 0.f;
    if (sd > 0.0) {
        const uint64_t a = splitmix64(splitmix64(seed) + 2ull * (uint64_t)p);
        const uint64_t b = splitmix64(splitmix64(seed) + 2ull * (uint64_t)p + 1ull);
        const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
        const double u2 = (double)(b >> 11) * 0x1.0p-53;          // [0, 1)
        w = (float)(sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    }
    theta[p] = w;
}

// The output bias starts at the lower median of a strided sample of at most 2048
// targets (one workgroup).
__global__ __launch_bounds__(256) void net_median_bias_kernel(const float *__restrict__ ex_y, int64_t n,
                                                              float *__restrict__ theta) {
    __shared__ uint64_t keys[2048];
    const uint32_t S = n < 2048 ? (uint32_t)n : 2048u;
    for (uint32_t t = threadIdx.x; t < S; t += 256) keys[t] = make_key(ex_y[((int64_t)t * n) / S], t);
    __syncthreads();
    block_sort<256, 8>(keys, S);
    if (threadIdx.x == 0) theta[kOffB3] = ord_to_float(key_ord(keys[(S - 1) / 2]));
}

// A training batch of B examples drawn uniformly with replacement: example
// splitmix64(stream + b) mod n for slot b, stream = (seed, step).
__global__ __launch_bounds__(256) void net_draw_kernel(const float *__restrict__ ex_x, const float *__restrict__ ex_y,
                                                       int64_t n, uint64_t stream, int64_t B, float *__restrict__ bx,
                                                       float *__restrict__ by) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t e = (int64_t)(splitmix64(stream + (uint64_t)b) % (uint64_t)n);
#pragma unroll
    for (int i = 0; i < kNetIn; ++i) bx[b * kNetIn + i] = ex_x[e * kNetIn + i];
    by[b] = ex_y[e];
}

}  // namespace knn

using namespace knn;

namespace {

knn_status_t hfail(knn_handle_t h, knn_status_t s, const std::string &m) { return fail_msg(h, s, m); }

knn_status_t ensure_net(knn_handle_t h) {
    if (h->net_theta) return KNN_SUCCESS;
    const size_t f = kNetParams * sizeof(float);
    hipError_t e = hipMalloc(&h->net_theta, f);
    if (e == hipSuccess) e = hipMalloc(&h->net_theta_r, f);
    if (e == hipSuccess) e = hipMalloc(&h->net_m, f);
    if (e == hipSuccess) e = hipMalloc(&h->net_v, f);
    if (e == hipSuccess) e = hipMalloc(&h->net_grad, f);
    // one spare element so that the network can be copied as 32-bit words
    if (e == hipSuccess) e = hipMalloc(&h->net_bf16, (kNetParams + 1) * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemset(h->net_bf16, 0, (kNetParams + 1) * sizeof(uint16_t));
    if (e != hipSuccess) return hfail(h, KNN_ERROR_OUT_OF_MEMORY, "pivot network allocation failed");
    return KNN_SUCCESS;
}

knn_status_t upload_params(knn_handle_t h, const float *host, int64_t step) {
    knn_status_t st = ensure_net(h);
    if (st != KNN_SUCCESS) return st;
    const size_t f = kNetParams * sizeof(float);
    hipError_t e = hipMemcpy(h->net_theta, host, f, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->net_m, 0, f);
    if (e == hipSuccess) e = hipMemset(h->net_v, 0, f);
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("pivot weights upload: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(net_round_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, nullptr, h->net_theta,
                       h->net_theta_r, h->net_bf16);
    if ((e = hipDeviceSynchronize()) != hipSuccess)
        return hfail(h, KNN_ERROR_DEVICE, std::string("pivot weights rounding: ") + hipGetErrorString(e));
    h->net_step = step;
    h->has_net = true;
    return KNN_SUCCESS;
}

const char kMagic[8] = {'K', 'N', 'N', 'P', 'I', 'V', '0', '1'};

}  // namespace

extern "C" {

knn_status_t knn_pivot_set_weights(knn_handle_t h, const float *host_params, int32_t n) {
    if (!h || !host_params) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_set_weights: null argument");
    if (n != kNetParams) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_set_weights: expected 4801 parameters");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(host_params[i])) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_set_weights: non-finite");
    hipSetDevice(h->device);
    return upload_params(h, host_params, 0);
}

knn_status_t knn_pivot_get_weights(knn_handle_t h, float *host_params, int32_t n) {
    if (!h || !host_params) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_get_weights: null argument");
    if (n != kNetParams) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_get_weights: expected 4801 parameters");
    if (!h->has_net) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_get_weights: no pivot network loaded");
    hipSetDevice(h->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host_params, h->net_theta, kNetParams * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_get_weights: ") + hipGetErrorString(e));
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_save(knn_handle_t h, const char *path) {
    if (!h || !path) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_save: null argument");
    std::vector<float> w(kNetParams);
    knn_status_t st = knn_pivot_get_weights(h, w.data(), kNetParams);
    if (st != KNN_SUCCESS) return st;
    FILE *f = std::fopen(path, "wb");
    if (!f) return hfail(h, KNN_ERROR_IO, std::string("knn_pivot_save: cannot open ") + path);
    uint32_t hdr[4] = {1u, (uint32_t)kNetParams, (uint32_t)kNetIn, (uint32_t)kNetHidden};
    int64_t step = h->net_step;
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(&step, sizeof(step), 1, f) == 1 && std::fwrite(&h->net_quantile, sizeof(float), 1, f) == 1 &&
              std::fwrite(w.data(), sizeof(float), kNetParams, f) == (size_t)kNetParams;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return hfail(h, KNN_ERROR_IO, std::string("knn_pivot_save: write failed: ") + path);
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_load(knn_handle_t h, const char *path) {
    if (!h || !path) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_load: null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return hfail(h, KNN_ERROR_IO, std::string("knn_pivot_load: cannot open ") + path);
    char magic[8];
    uint32_t hdr[4];
    int64_t step = 0;
    float q = 0;
    std::vector<float> w(kNetParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 1u && hdr[1] == (uint32_t)kNetParams &&
              hdr[2] == (uint32_t)kNetIn && hdr[3] == (uint32_t)kNetHidden && std::fread(&step, sizeof(step), 1, f) == 1 &&
              std::fread(&q, sizeof(q), 1, f) == 1 &&
              std::fread(w.data(), sizeof(float), kNetParams, f) == (size_t)kNetParams;
    std::fclose(f);
    if (!ok) return hfail(h, KNN_ERROR_IO, std::string("knn_pivot_load: not a pivot weights file: ") + path);
    for (float x : w)
        if (!std::isfinite(x)) return hfail(h, KNN_ERROR_IO, "knn_pivot_load: non-finite weight");
    hipSetDevice(h->device);
    knn_status_t st = upload_params(h, w.data(), step);
    if (st == KNN_SUCCESS) h->net_quantile = q;
    return st;
}

knn_status_t knn_pivot_features(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld, int32_t k,
                                float *feats, float *loc_scale, void *stream) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_pivot_features: handle is null");
    if (rows < 0 || ld < cols || k < 1 || k > cols)
        return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_features: bad sizes");
    if (cols < kNetSample) return hfail(h, KNN_ERROR_UNSUPPORTED, "knn_pivot_features: rows shorter than 256");
    if (cols > INT32_MAX) return hfail(h, KNN_ERROR_UNSUPPORTED, "knn_pivot_features: cols > INT32_MAX");
    if (rows == 0) return KNN_SUCCESS;
    if (!dist || !feats) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_features: null pointer");
    hipSetDevice(h->device);
    int64_t grid = rows < 65536 ? rows : 65536;
    hipLaunchKernelGGL(net_features_kernel, dim3((unsigned)grid), dim3(kFeatThreads), 0, (hipStream_t)stream, dist,
                       rows, (uint32_t)cols, ld, (uint32_t)k, feats, loc_scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("features kernel: ") + hipGetErrorString(e));
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_predict(knn_handle_t h, const float *feats, int64_t rows, float *out, void *stream) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_pivot_predict: handle is null");
    if (rows < 0) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_predict: rows < 0");
    if (!h->has_net) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_predict: no pivot network loaded");
    if (rows == 0) return KNN_SUCCESS;
    if (!feats || !out) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_predict: null pointer");
    hipSetDevice(h->device);
    hipLaunchKernelGGL(net_predict_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, (hipStream_t)stream, feats,
                       rows, h->net_bf16, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("predict kernel: ") + hipGetErrorString(e));
    return KNN_SUCCESS;
}

static knn_status_t grad_common(knn_handle_t h, const char *fn, const float *feats, const float *targets, int64_t B,
                                float q, float *grad, float *loss, hipStream_t stream) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": handle is null");
    if (B < 1) return hfail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": batch < 1");
    if (!(q > 0.f && q < 1.f)) return hfail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": quantile outside (0, 1)");
    if (!feats || !targets || !grad) return hfail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": null pointer");
    if (!h->has_net) return hfail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": no pivot network loaded");
    hipSetDevice(h->device);
    void *ws = nullptr;
    const size_t per = (size_t)B * kNetHidden;
    knn_status_t st = ensure_ws(h, (4 * per + 2 * (size_t)B) * sizeof(float) + 1024, stream, &ws);
    if (st != KNN_SUCCESS) return st;
    float *H1 = static_cast<float *>(ws), *H2 = H1 + per, *D1 = H2 + per, *D2 = D1 + per, *dy = D2 + per, *lv = dy + B;
    hipLaunchKernelGGL(net_fwd_bwd_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, feats, targets, B,
                       h->net_theta_r, q, H1, H2, D1, D2, dy, lv);
    hipLaunchKernelGGL(net_wgrad_kernel, dim3((kNetParams + 1 + 255) / 256), dim3(256), 0, stream, feats, H1, H2, D1,
                       D2, dy, lv, B, grad, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string(fn) + ": " + hipGetErrorString(e));
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_grad(knn_handle_t h, const float *feats, const float *targets, int64_t B, float quantile,
                            float *grad, float *loss, void *stream) {
    return grad_common(h, "knn_pivot_grad", feats, targets, B, quantile, grad, loss, (hipStream_t)stream);
}

static knn_status_t adam_step(knn_handle_t h, float quantile, float lr, hipStream_t s);

knn_status_t knn_pivot_train_step(knn_handle_t h, const float *feats, const float *targets, int64_t B, float quantile,
                                  float lr, float *loss, void *stream) {
    if (h && !(lr > 0.f)) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train_step: lr <= 0");
    if (h && !h->has_net) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train_step: no pivot network loaded");
    hipStream_t s = (hipStream_t)stream;
    knn_status_t st = grad_common(h, "knn_pivot_train_step", feats, targets, B, quantile, h ? h->net_grad : nullptr,
                                  loss, s);
    if (st != KNN_SUCCESS) return st;
    return adam_step(h, quantile, lr, s);
}

static knn_status_t adam_step(knn_handle_t h, float quantile, float lr, hipStream_t s) {
    h->net_step += 1;
    h->net_quantile = quantile;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)h->net_step), c2 = 1.f - std::pow(b2, (float)h->net_step);
    hipLaunchKernelGGL(net_adam_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, s, h->net_theta, h->net_m,
                       h->net_v, h->net_grad, lr, b1, b2, eps, c1, c2, h->net_theta_r, h->net_bf16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("adam kernel: ") + hipGetErrorString(e));
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_clear_examples(knn_handle_t h) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_pivot_clear_examples: handle is null");
    h->ex_n = 0;
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_example_count(knn_handle_t h, int64_t *count) {
    if (!h || !count) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_example_count: null argument");
    *count = h->ex_n;
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_get_examples(knn_handle_t h, float *feats, float *targets, int64_t max_rows) {
    if (!h || !feats || !targets) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_get_examples: null argument");
    if (max_rows < h->ex_n) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_get_examples: buffer too small");
    if (h->ex_n == 0) return KNN_SUCCESS;
    hipSetDevice(h->device);
    hipError_t e = hipMemcpy(feats, h->ex_x, (size_t)h->ex_n * kNetIn * sizeof(float), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(targets, h->ex_y, (size_t)h->ex_n * sizeof(float), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_get_examples: ") + hipGetErrorString(e));
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_add_examples(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld,
                                    int32_t k, void *stream_) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_pivot_add_examples: handle is null");
    if (rows < 0 || cols < 1 || ld < cols || k < 1 || k > cols)
        return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_add_examples: bad sizes");
    if (cols < kNetSample) return hfail(h, KNN_ERROR_UNSUPPORTED, "knn_pivot_add_examples: rows shorter than 256");
    if (cols > INT32_MAX) return hfail(h, KNN_ERROR_UNSUPPORTED, "knn_pivot_add_examples: cols > INT32_MAX");
    if (k > kSelectMaxK) return hfail(h, KNN_ERROR_UNSUPPORTED, "knn_pivot_add_examples: k > 1024");
    if (rows == 0) return KNN_SUCCESS;
    if (!dist) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_add_examples: null pointer");
    hipSetDevice(h->device);
    hipStream_t s = (hipStream_t)stream_;
    hipError_t e = hipSuccess;
    if (h->ex_n + rows > h->ex_cap) {
        int64_t cap = h->ex_cap ? h->ex_cap : 65536;
        while (cap < h->ex_n + rows) cap *= 2;
        float *nx = nullptr, *ny = nullptr;
        e = hipMalloc(&nx, (size_t)cap * kNetIn * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&ny, (size_t)cap * sizeof(float));
        if (e != hipSuccess) {
            if (nx) hipFree(nx);
            (void)hipGetLastError();
            return hfail(h, KNN_ERROR_OUT_OF_MEMORY, "knn_pivot_add_examples: example buffer");
        }
        if (h->ex_n) {
            e = hipMemcpyAsync(nx, h->ex_x, (size_t)h->ex_n * kNetIn * sizeof(float), hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ny, h->ex_y, (size_t)h->ex_n * sizeof(float), hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (h->ex_x) hipFree(h->ex_x);
        if (h->ex_y) hipFree(h->ex_y);
        h->ex_x = nx;
        h->ex_y = ny;
        h->ex_cap = cap;
        if (e != hipSuccess) {
            h->ex_n = 0;
            return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_add_examples: ") + hipGetErrorString(e));
        }
    }
    // workspace: features, (m, s), the selected values, the selection's own
    // workspace, the kept count
    const int cap = select_cap_for_k((uint32_t)k);
    const int grid = select_grid(cap, rows, h->num_cu);
    const size_t selws = select_ws_bytes(cap, (uint32_t)cols, grid);
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t fb = up((size_t)rows * kNetIn * 4), lb = up((size_t)rows * 8), vb = up((size_t)rows * k * 4),
                 ib = up((size_t)rows * k * 4);
    void *ws = nullptr;
    knn_status_t st = ensure_ws(h, fb + lb + vb + ib + up(selws) + 256, s, &ws);
    if (st != KNN_SUCCESS) return st;
    char *w = static_cast<char *>(ws);
    float *feats = reinterpret_cast<float *>(w), *ls = reinterpret_cast<float *>(w + fb);
    float *vals = reinterpret_cast<float *>(w + fb + lb);
    int32_t *idx = reinterpret_cast<int32_t *>(w + fb + lb + vb);
    void *sws = w + fb + lb + vb + ib;
    uint32_t *kept = reinterpret_cast<uint32_t *>(w + fb + lb + vb + ib + up(selws));
    const int64_t g = rows < 65536 ? rows : 65536;
    hipLaunchKernelGGL(net_features_kernel, dim3((unsigned)g), dim3(kFeatThreads), 0, s, dist, rows, (uint32_t)cols, ld,
                       (uint32_t)k, feats, ls);
    SelectArgs a{};
    a.dist = dist;
    a.rows = rows;
    a.cols = (uint32_t)cols;
    a.ld = ld;
    a.k = (uint32_t)k;
    a.out_val = vals;
    a.out_idx = idx;
    a.mode = kPivotSample;
    if ((e = launch_select(a, cap, grid, sws, s)) != hipSuccess)
        return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_add_examples: select: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(net_examples_kernel, dim3(1), dim3(256), 0, s, feats, ls, vals, rows, k, h->ex_x, h->ex_y,
                       h->ex_n, kept);
    uint32_t *hk = h->pinned;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hk, kept, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_add_examples: ") + hipGetErrorString(e));
    h->ex_n += *hk;
    return KNN_SUCCESS;
}

knn_status_t knn_pivot_train(knn_handle_t h, const char *out_path, uint64_t seed, int32_t steps) {
    if (!h) return hfail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_pivot_train: handle is null");
    if (steps < 0) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train: steps < 0");
    if (h->ex_n < 1) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train: no training examples");
    hipSetDevice(h->device);
    knn_status_t st = ensure_net(h);
    if (st != KNN_SUCCESS) return st;
    hipStream_t s = nullptr;
    const int64_t n = h->ex_n, B = n < kTrainBatch ? n : kTrainBatch;
    // workspace: the gradient pass's region first (grad_common uses it from the
    // start), then the batch
    const size_t per = (size_t)B * kNetHidden;
    const size_t gbytes = ((4 * per + 2 * (size_t)B) * sizeof(float) + 1024 + 255) & ~size_t(255);
    void *ws = nullptr;
    st = ensure_ws(h, gbytes + (size_t)B * (kNetIn + 1) * sizeof(float) + 512, s, &ws);
    if (st != KNN_SUCCESS) return st;
    float *bx = reinterpret_cast<float *>(static_cast<char *>(ws) + gbytes), *by = bx + (size_t)B * kNetIn;
    float *loss = by + B;
    hipLaunchKernelGGL(net_init_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, s, seed, h->net_theta, h->net_m,
                       h->net_v);
    hipLaunchKernelGGL(net_median_bias_kernel, dim3(1), dim3(256), 0, s, h->ex_y, n, h->net_theta);
    hipLaunchKernelGGL(net_round_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, s, h->net_theta, h->net_theta_r,
                       h->net_bf16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_train: init: ") + hipGetErrorString(e));
    h->has_net = true;
    h->net_step = 0;
    for (int32_t it = 0; it < steps; ++it) {
        // learning rate decays exponentially from kTrainLr to kTrainLr / 10
        const float lr = kTrainLr * std::pow(0.1f, (float)it / (float)steps);
        const uint64_t stream = (seed * 0x100000001B3ull) ^ ((uint64_t)it << 32);
        hipLaunchKernelGGL(net_draw_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, h->ex_x, h->ex_y, n,
                           stream, B, bx, by);
        st = grad_common(h, "knn_pivot_train", bx, by, B, kTrainQuantile, h->net_grad, loss, s);
        if (st != KNN_SUCCESS) return st;
        if ((st = adam_step(h, kTrainQuantile, lr, s)) != KNN_SUCCESS) return st;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return hfail(h, KNN_ERROR_DEVICE, std::string("knn_pivot_train: ") + hipGetErrorString(e));
    h->net_quantile = kTrainQuantile;
    if (out_path) return knn_pivot_save(h, out_path);
    return KNN_SUCCESS;
}

}  // extern "C"
