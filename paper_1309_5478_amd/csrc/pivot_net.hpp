// The pivot network, device side: the 8 row features computed from a sorted
// 256-entry strided sample, and the 8 -> 64 -> 64 -> 1 ReLU network with BF16
// weights and FP32 accumulation, evaluated by one wave (lane j = hidden unit j).
//
// Sample: 4 blocks of 64 contiguous entries, block b at floor(b (N - 64) / 3).
// Features: x0 = log2 N / 16, x1 = log2 k / 10, then with m = v_127 (lower
// median), s = max((v_191 - v_63) / 1.349, 1e-30 (|m| + 1)) and
// r = clamp(ceil(256 k / N) - 1, 0, 255):
//   x2 = (v_0 - m)/s, x3 = (v_r - m)/s, x4 = (v_{r+1} - m)/s, x5 = (v_25 - m)/s,
//   x6 = (mean - m)/s, x7 = log(s / (|m| + s)).
// The network predicts y = (v_k - m) / s, the standardised k-th smallest value;
// the pivot is m + s * y.
#pragma once
#include "keys.hpp"

namespace knn {

constexpr int kNetIn = 8;
constexpr int kNetHidden = 64;
constexpr int kNetParams = kNetHidden * kNetIn + kNetHidden + kNetHidden * kNetHidden + kNetHidden + kNetHidden + 1;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNetHidden * kNetIn;
constexpr int kOffW2 = kOffB1 + kNetHidden;
constexpr int kOffB2 = kOffW2 + kNetHidden * kNetHidden;
constexpr int kOffW3 = kOffB2 + kNetHidden;
constexpr int kOffB3 = kOffW3 + kNetHidden;
constexpr int kNetSample = 256;
constexpr int kNetBlocks = 4;

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even, FP32 -> BF16 (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t net_sample_start(uint32_t b, uint32_t N) {
    return (uint32_t)(((uint64_t)b * (N - kWave)) / (kNetBlocks - 1));
}

// Features from the ascending sample v[0..255] (all lanes of the calling wave
// compute the same values; called by one wave).  Returns m and s too.
__device__ __forceinline__ void net_features(const float *v, uint32_t N, uint32_t k, float x[kNetIn], float &m,
                                             float &s) {
    const uint32_t lane = lane_id();
    float part = v[lane] + v[lane + 64] + v[lane + 128] + v[lane + 192];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    const float mean = part * (1.0f / kNetSample);
    m = v[127];
    s = (v[191] - v[63]) * (1.0f / 1.349f);
    const float floor_s = 1e-30f * (fabsf(m) + 1.0f);
    s = s > floor_s ? s : floor_s;
    const uint64_t num = (uint64_t)kNetSample * k;
    int64_t r = (int64_t)((num + N - 1) / N) - 1;
    r = r < 0 ? 0 : (r > kNetSample - 1 ? kNetSample - 1 : r);
    const int64_t r1 = r + 1 < kNetSample ? r + 1 : kNetSample - 1;
    const float inv = 1.0f / s;
    x[0] = log2f((float)N) * (1.0f / 16.0f);
    x[1] = log2f((float)k) * (1.0f / 10.0f);
    x[2] = (v[0] - m) * inv;
    x[3] = (v[r] - m) * inv;
    x[4] = (v[r1] - m) * inv;
    x[5] = (v[25] - m) * inv;
    x[6] = (mean - m) * inv;
    x[7] = logf(s / (fabsf(m) + s));
}

// Forward pass by one wave; x is uniform across the wave.  Weights are BF16
// (w 4-byte aligned, global memory or LDS), accumulation FP32 in a fixed order.
// Each lane loads its unit's weight rows up front, so that all the loads are in
// flight together.  Returns y_hat in every lane.
__device__ __forceinline__ float net_forward_wave(const uint16_t *__restrict__ w, const float x[kNetIn]) {
    const uint32_t j = lane_id();
    const uint32_t *w1 = reinterpret_cast<const uint32_t *>(w + kOffW1 + j * kNetIn);
    const uint32_t *w2 = reinterpret_cast<const uint32_t *>(w + kOffW2 + j * kNetHidden);
    uint32_t r1[kNetIn / 2], r2[kNetHidden / 2];
#pragma unroll
    for (int i = 0; i < kNetIn / 2; ++i) r1[i] = w1[i];
#pragma unroll
    for (int i = 0; i < kNetHidden / 2; ++i) r2[i] = w2[i];
    const float b1 = bf16_to_f32(w[kOffB1 + j]), b2 = bf16_to_f32(w[kOffB2 + j]);
    const float w3 = bf16_to_f32(w[kOffW3 + j]), b3 = bf16_to_f32(w[kOffB3]);
    // element i of a packed row: the low half of word i / 2 for even i
    auto elem = [](const uint32_t *r, int i) {
        return __uint_as_float((i & 1) ? (r[i >> 1] & 0xFFFF0000u) : (r[i >> 1] << 16));
    };
    float z1 = b1;
#pragma unroll
    for (int i = 0; i < kNetIn; ++i) z1 = fmaf(elem(r1, i), x[i], z1);
    const float h1 = z1 > 0.f ? z1 : 0.f;
    float z2 = b2;
#pragma unroll
    for (int i = 0; i < kNetHidden; ++i) {
        const float hi = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(h1), i));  // h1 of unit i
        z2 = fmaf(elem(r2, i), hi, z2);
    }
    const float h2 = z2 > 0.f ? z2 : 0.f;
    float y = w3 * h2;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) y += __shfl_xor(y, off);
    return y + b3;
}

}  // namespace knn
