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

knn_status_t knn_pivot_train_step(knn_handle_t h, const float *feats, const float *targets, int64_t B, float quantile,
                                  float lr, float *loss, void *stream) {
    if (h && !(lr > 0.f)) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train_step: lr <= 0");
    if (h && !h->has_net) return hfail(h, KNN_ERROR_INVALID_VALUE, "knn_pivot_train_step: no pivot network loaded");
    hipStream_t s = (hipStream_t)stream;
    knn_status_t st = grad_common(h, "knn_pivot_train_step", feats, targets, B, quantile, h ? h->net_grad : nullptr,
                                  loss, s);
    if (st != KNN_SUCCESS) return st;
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

}  // extern "C"
