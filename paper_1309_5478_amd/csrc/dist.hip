// Distance kernels around the matrix-core product (Methods, "Distance
// calculation"): squared norms, unit vectors for the cosine and Pearson
// distances, reduced-precision operands, candidate bookkeeping, the
// certificate, and the exact direct-form re-rank of the surviving candidates
// (and of uncertified rows).  The product itself is in gemm.hip.
#include <cstdlib>
#include <cstring>
#include "dist.hpp"
#include "keys.hpp"

namespace knn {

// ---- unit vectors (cosine and Pearson distances) ------------------------------
// Methods, "Distance calculation": the cosine similarity of x and y is
// x.y / (|x| |y|), and Pearson's correlation is the cosine similarity of the
// vectors minus their means.  With u = x / |x| and v = y / |y|,
// 1 - cos = |u - v|^2 / 2, so both distances are half the squared Euclidean
// distance of unit vectors, and the Euclidean path ranks them unchanged.  One
// wave per row: lane-strided sums in a fixed order reduced by a lane tree; the
// norm is taken of the row scaled by its largest magnitude (no overflow or
// underflow in the squares), and every element is divided once.
__device__ __forceinline__ float wave_sum(float s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}
__device__ __forceinline__ float wave_max(float s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmaxf(s, __shfl_xor(s, off));
    return s;
}
__device__ __forceinline__ float wave_min(float s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fminf(s, __shfl_xor(s, off));
    return s;
}

__global__ __launch_bounds__(256) void unit_rows_kernel(const float *__restrict__ X, int64_t n, int d, int centre,
                                                        float *__restrict__ out) {
    const uint32_t lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const float *x = X + i * d;
    float *o = out + i * d;
    float mu = 0.f;
    bool flat = false;
    if (centre) {
        float s = 0.f, lo = __uint_as_float(0x7f800000u), hi = -lo;
        for (int t = (int)lane; t < d; t += kWave) {
            const float v = x[t];
            s += v;
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        mu = wave_sum(s) / (float)d;
        // a constant row is exactly zero once centred, whatever the rounding of its mean
        flat = wave_min(lo) == wave_max(hi);
    }
    float amax = 0.f;
    bool nan = false;
    for (int t = (int)lane; t < d; t += kWave) {
        const float v = x[t] - mu;
        nan |= v != v;
        amax = fmaxf(amax, fabsf(v));
    }
    amax = wave_max(amax);
    nan = __ballot(nan) != 0;
    const bool ok = !flat && !nan && amax > 0.f && amax <= 3.4028235e38f;
    float ss = 0.f;
    if (ok)
        for (int t = (int)lane; t < d; t += kWave) {
            const float v = (x[t] - mu) / amax;
            ss = fmaf(v, v, ss);
        }
    const float nrm = sqrtf(wave_sum(ss));
    const float qnan = __uint_as_float(0x7fc00000u);
    for (int t = (int)lane; t < d; t += kWave) o[t] = ok ? ((x[t] - mu) / amax) / nrm : qnan;
}

hipError_t launch_unit_rows(const float *X, int64_t n, int d, bool centre, float *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 3) / 4;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(unit_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, n, d, centre ? 1 : 0, out);
    return hipGetLastError();
}

// ---- squared norms ----------------------------------------------------------
// G lanes per point (the power of two covering the point's 16-byte chunks, or
// its elements without 16-byte loads; at most 64), 64 / G points per wave,
// grid-stride over points.  Each lane accumulates its strided elements in
// order, then a fixed xor-shuffle tree over the G lanes.  With max_bits, the
// largest norm (as FP32 bits; norms are non-negative) is folded into *max_bits
// with one atomic per workgroup.
template <int G, bool VEC>
__global__ __launch_bounds__(256) void sqnorm_kernel(const float *__restrict__ X, int64_t n, int d,
                                                     float *__restrict__ out, unsigned int *__restrict__ max_bits) {
    constexpr int PPW = kWave / G;
    __shared__ float wmax[256 / kWave];
    const uint32_t lane = lane_id(), sub = lane % G, grp = lane / G, wave = threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * (256 / kWave) * PPW;
    float mx = 0.f;
    // two points per group per step (independent loads in flight)
    for (int64_t base = ((int64_t)blockIdx.x * (256 / kWave) + wave) * PPW; base < n; base += 2 * stride) {
        float acc[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = base + u * stride + grp;
            float s = 0.f;
            if (i < n) {
                const float *x = X + i * d;
                if (VEC) {
                    for (int t = (int)sub * 4; t < d; t += G * 4) {
                        const f32x4 v = *reinterpret_cast<const f32x4 *>(x + t);
                        s = fmaf(v[0], v[0], s);
                        s = fmaf(v[1], v[1], s);
                        s = fmaf(v[2], v[2], s);
                        s = fmaf(v[3], v[3], s);
                    }
                } else {
                    for (int t = (int)sub; t < d; t += G) s = fmaf(x[t], x[t], s);
                }
            }
            acc[u] = s;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off);
            const int64_t i = base + u * stride + grp;
            if (i < n && sub == 0) out[i] = acc[u];
            mx = fmaxf(mx, acc[u]);
        }
    }
    if (max_bits) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if (lane == 0) wmax[wave] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = wmax[0];
            for (int w = 1; w < 256 / kWave; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(max_bits, __float_as_uint(m));
        }
    }
}

// Lanes per point or candidate for a row length d: the power of two covering
// its 16-byte chunks (or its elements), at most a wave.
static int lanes_for(int d, bool vec) {
    const int units = vec ? (d + 3) / 4 : d;
    int g = 1;
    while (g < units && g < kWave) g <<= 1;
    return g;
}

// ---- gather rows (and their norms) -----------------------------------------
// dst row t = src row idx[t] (idx null: row floor(t * n / rows)).
__global__ __launch_bounds__(256) void gather_rows_kernel(const float *__restrict__ src, int64_t n, int d,
                                                          const int32_t *__restrict__ idx, int64_t rows,
                                                          float *__restrict__ dst, const float *__restrict__ norms,
                                                          float *__restrict__ dst_norms) {
    const int64_t t = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (t >= rows) return;
    const int64_t s = idx ? (int64_t)idx[t] : (t * n) / rows;
    const uint32_t lane = lane_id();
    for (int c = lane; c < d; c += kWave) dst[t * d + c] = src[s * d + c];
    if (norms && lane == 0) dst_norms[t] = norms[s];
}

// ---- candidate bookkeeping ----------------------------------------------------
// Rows whose candidate count is below `need` or above `cap` are listed for the
// exact fallback.
__global__ __launch_bounds__(256) void flag_rows_kernel(const uint32_t *__restrict__ cnt, int64_t m, uint32_t need,
                                                        uint32_t cap, int force, uint32_t *__restrict__ nflag,
                                                        int32_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t c = cnt[i];
    if (force || c < need || c > cap) {
        uint32_t p = atomicAdd(nflag, 1u);
        flags[p] = (int32_t)i;
    }
}

// Replaces the candidate lists of the flagged rows by the exact selection made
// on their materialised distance rows.
__global__ __launch_bounds__(256) void scatter_fallback_kernel(const int32_t *__restrict__ rows, int64_t nrows,
                                                               const float *__restrict__ val,
                                                               const int32_t *__restrict__ idx, int kk,
                                                               uint64_t *__restrict__ cand, uint32_t *__restrict__ cnt,
                                                               int cap) {
    const int64_t f = blockIdx.x;
    if (f >= nrows) return;
    const int64_t i = rows[f];
    for (int t = threadIdx.x; t < kk; t += blockDim.x)
        cand[i * cap + t] = make_key(val[f * kk + t], (uint32_t)idx[f * kk + t]);
    if (threadIdx.x == 0) cnt[i] = (uint32_t)kk;
}

// ---- exact re-rank ----------------------------------------------------------
// One workgroup per query: the exact FP32 squared distance sum_t (q_t - c_t)^2
// to each of the row's kk candidates, then a bitonic sort of the (distance,
// index) keys; the first k are written (missing entries: +inf, index -1).
// G lanes per candidate (the power of two covering d's 16-byte chunks, at
// most a wave), so a wave works on 64 / G candidates at once, two per lane
// group per step to keep more loads in flight; each lane accumulates its
// strided elements in order, then a fixed xor-shuffle tree over the G lanes.
constexpr int kRerankThreads = 256;
constexpr int kRerankMax = 1024;

template <int G, bool VEC>
__device__ __forceinline__ float rerank_dist(const float *__restrict__ q, const float *__restrict__ y, int d,
                                             uint32_t sub) {
    float s = 0.f;
    if (VEC) {
        for (int t = (int)sub * 4; t < d; t += G * 4) {
            const f32x4 qv = *reinterpret_cast<const f32x4 *>(q + t);
            const f32x4 yv = *reinterpret_cast<const f32x4 *>(y + t);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float df = qv[e] - yv[e];
                s = fmaf(df, df, s);
            }
        }
    } else {
        for (int t = (int)sub; t < d; t += G) {
            const float df = q[t] - y[t];
            s = fmaf(df, df, s);
        }
    }
    return s;
}

template <int G, bool VEC>
__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(RerankArgs a) {
    constexpr uint32_t PPW = kWave / G;                       // candidates per wave per pass
    constexpr uint32_t STEP = (kRerankThreads / kWave) * PPW;  // per workgroup per pass
    __shared__ uint64_t keys[kRerankMax];
    const int64_t i = blockIdx.x;
    if (i >= a.m) return;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave, sub = lane % G, grp = lane / G;
    const float *q = a.Q + i * a.d;
    const uint32_t kk = a.kk;
    const int32_t *ci = a.cidx + i * kk;
    const int64_t own = a.self_offset >= 0 ? a.self_offset + i : (int64_t)-1;
    for (uint32_t c0 = wave * PPW + grp; c0 < kk; c0 += 2 * STEP) {
        const uint32_t c1 = c0 + STEP;
        const uint32_t j0 = (uint32_t)ci[c0];
        const uint32_t j1 = c1 < kk ? (uint32_t)ci[c1] : 0xFFFFFFFFu;
        // missing candidates (never for valid lists) and the query's own index
        // (a candidate only when its row has no other finite key) are dropped
        const bool ok0 = (int64_t)j0 < a.n && (int64_t)j0 != own, ok1 = (int64_t)j1 < a.n && (int64_t)j1 != own;
        float s0 = ok0 ? rerank_dist<G, VEC>(q, a.C + (int64_t)j0 * a.d, a.d, sub) : 0.f;
        float s1 = ok1 ? rerank_dist<G, VEC>(q, a.C + (int64_t)j1 * a.d, a.d, sub) : 0.f;
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
        }
        if (sub == 0) {
            keys[c0] = ok0 ? make_key(s0, j0) : kKeyMax;
            if (c1 < kk) keys[c1] = ok1 ? make_key(s1, j1) : kKeyMax;
        }
    }
    __syncthreads();
    block_sort<kRerankThreads>(keys, kk);
    for (uint32_t t = tid; t < (uint32_t)a.k; t += kRerankThreads) {
        const uint64_t key = t < kk ? keys[t] : kKeyMax;
        if (key == kKeyMax) {
            a.out_dist[i * a.k + t] = __uint_as_float(0x7f800000u);
            a.out_idx[i * a.k + t] = -1;
        } else {
            a.out_dist[i * a.k + t] = a.out_scale * ord_to_float(key_ord(key));
            a.out_idx[i * a.k + t] = (int32_t)key_idx(key);
        }
    }
}

// ---- reduced-precision operands ---------------------------------------------
// OCP e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits, no infinity),
// round to nearest even, saturating at +-448 (also for infinities); a NaN
// becomes the NaN code S.1111.111.
__device__ __forceinline__ uint8_t f32_to_e4m3(float x) {
    const uint8_t sign = (uint8_t)((__float_as_uint(x) >> 24) & 0x80u);
    const float a = fabsf(x);
    if (a != a) return sign | 0x7Fu;
    if (!(a < 448.0f)) return sign | 0x7Eu;
    if (a < 0.015625f) {                               // below 2^-6: subnormals, step 2^-9
        return sign | (uint8_t)rintf(a * 512.0f);      // 8 (= 2^-6) encodes the smallest normal
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;  // floor(log2 a), in [-6, 8]
    float r = rintf(ldexpf(a, 3 - e));                 // mantissa with the hidden bit, in [8, 16]
    if (r >= 16.0f) {
        r = 8.0f;
        e += 1;
    }
    if (e > 8 || (e == 8 && r > 14.0f)) return sign | 0x7Eu;
    return sign | (uint8_t)(((e + 7) << 3) | ((int)r - 8));
}

// BF16 by round to nearest even on the low 16 bits; a NaN stays a quiet NaN
// (the rounding carry could otherwise turn a NaN with only low payload bits
// into an infinity).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if (f != f) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One wave per point.  FP8: e = the largest integer with amax * 2^e <= 448,
// amax the largest finite magnitude of the point (e = 0 without a finite
// non-zero element; e limited to [-100, 100]), elements x * 2^e rounded to
// e4m3, scale 2^-e.
__global__ __launch_bounds__(256) void quantize_kernel(const float *__restrict__ X, int64_t n, int d, int prec, int dq,
                                                       void *__restrict__ out, float *__restrict__ scale_out) {
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (i >= n) return;
    const uint32_t lane = lane_id();
    const float *x = X + i * d;
    if (prec == kPrecBF16) {
        uint16_t *o = static_cast<uint16_t *>(out) + i * dq;
        for (int t = lane; t < dq; t += kWave) o[t] = t < d ? f32_to_bf16_rne(x[t]) : (uint16_t)0;
        return;
    }
    float amax = 0.f;
    for (int t = lane; t < d; t += kWave) {
        const float v = fabsf(x[t]);
        if (v <= 3.4028235e38f) amax = fmaxf(amax, v);  // finite magnitudes only
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    int e = 0;
    if (amax > 0.f) {
        // amax = f 2^E with f in [0.5, 1): amax 2^e <= 448 = 0.875 * 2^9 exactly
        // when e <= 9 - E, less one when f > 0.875
        int E;
        const float f = frexpf(amax, &E);
        e = 9 - E - (f > 0.875f ? 1 : 0);
        e = e < -100 ? -100 : (e > 100 ? 100 : e);
    }
    uint8_t *o = static_cast<uint8_t *>(out) + i * dq;
    for (int t = lane; t < dq; t += kWave) o[t] = t < d ? f32_to_e4m3(ldexpf(x[t], e)) : (uint8_t)0;
    if (lane == 0) scale_out[i] = ldexpf(1.0f, -e);
}

// Per-row candidate certificate (see launch_certify in dist.hpp for the bound).
__global__ __launch_bounds__(256) void certify_kernel(CertifyArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < a.m) {
        const float ak = a.sorted_keys[i * a.kk + a.k - 1];
        const float gap = a.sorted_keys[i * a.kk + a.kk - 1] - ak;
        const float c2 = __uint_as_float(*a.cmax2_bits), cm = sqrtf(c2), qm = sqrtf(a.qnorm2[i]);
        constexpr float u2 = 2.0f * 5.9604645e-8f;  // 2^-23
        // 1.001: slack for the FP32 evaluation of the bound itself
        const float E = 1.001f * ((a.gamma + u2) * c2 + 2.0f * (a.rel + u2) * qm * cm);
        bad = a.force || !(gap > 2.0f * E);
        if (bad && a.list) {
            const uint32_t p = atomicAdd(a.nlist, 1u);
            a.list[p] = (int32_t)i;
            a.tfix[i] = ak + 2.0f * E;
        }
    }
    const uint64_t b = __ballot(bad);
    if (lane_id() == 0 && b) atomicAdd(a.count, (unsigned long long)__popcll(b));
}

// ---- exact re-run of uncertified rows ------------------------------------------
// One workgroup per listed row.  The row's reduced keys are scanned in tiles of
// 1024; columns at or below the threshold are compacted into LDS (ballot +
// population count, one LDS reservation per wave) and, once 1024 or more are
// pending, re-ranked by exact distance, sorted and merged into the running
// 1024 smallest (distance, index) keys: the elementwise minimum of the
// ascending running list and the reversed lower half of the sorted batch holds
// exactly the 1024 smallest of both, as a bitonic sequence, which ten
// half-cleaning steps sort.
constexpr int kFixThreads = 256;
constexpr int kFixTop = 1024;
constexpr int kFixBatch = 2048;

template <int G, bool VEC>
__global__ __launch_bounds__(kFixThreads) void exact_rows_kernel(FixupArgs a) {
    constexpr uint32_t PPW = kWave / G;
    constexpr uint32_t STEP = (kFixThreads / kWave) * PPW;
    __shared__ uint64_t top[kFixTop];
    __shared__ uint64_t batch[kFixBatch];
    __shared__ uint32_t cidx[kFixBatch];
    __shared__ uint32_t cnt;
    const int64_t f = blockIdx.x;
    if (f >= a.nrows) return;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave, sub = lane % G, grp = lane / G;
    const int64_t i = a.rows[f];
    const float *drow = a.D + (a.by_row ? i : f) * a.ldd;
    const float T = a.tfix[i];
    const bool bounded = fabsf(T) <= 3.4028235e38f;  // finite (false for NaN)
    const float *q = a.Q + i * a.d;
    const int64_t own = a.self_offset >= 0 ? a.self_offset + i : (int64_t)-1;
    for (uint32_t t = tid; t < (uint32_t)kFixTop; t += kFixThreads) top[t] = kKeyMax;
    if (tid == 0) cnt = 0;
    __syncthreads();

    auto flush = [&](uint32_t c) {
        for (uint32_t c0 = wave * PPW + grp; c0 < c; c0 += STEP) {
            const uint32_t j = cidx[c0];
            float s = rerank_dist<G, VEC>(q, a.C + (int64_t)j * a.d, a.d, sub);
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (sub == 0) batch[c0] = (int64_t)j == own ? kKeyMax : make_key(s, j);
        }
        for (uint32_t t = c + tid; t < (uint32_t)kFixTop; t += kFixThreads) batch[t] = kKeyMax;
        __syncthreads();
        block_sort<kFixThreads, 8>(batch, c < (uint32_t)kFixTop ? (uint32_t)kFixTop : c);
        for (uint32_t t = tid; t < (uint32_t)kFixTop; t += kFixThreads) {
            const uint64_t x = top[t], y = batch[kFixTop - 1 - t];
            top[t] = x < y ? x : y;
        }
        __syncthreads();
        for (uint32_t st = kFixTop / 2; st > 0; st >>= 1) {
            for (uint32_t t = tid; t < (uint32_t)kFixTop / 2; t += kFixThreads) {
                const uint32_t lo = (t / st) * 2 * st + t % st, hi = lo + st;
                const uint64_t x = top[lo], y = top[hi];
                if (y < x) {
                    top[lo] = y;
                    top[hi] = x;
                }
            }
            __syncthreads();
        }
    };

    constexpr uint32_t kTileCols = 4 * kFixThreads;
    for (int64_t j0 = 0; j0 < a.n; j0 += kTileCols) {
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const int64_t j = j0 + u * kFixThreads + tid;
            const bool valid = j < a.n;
            const float v = valid ? drow[j] : 0.f;
            const bool pass = valid && (!bounded || v <= T);
            const uint64_t m = __ballot(pass);
            if (m) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&cnt, (uint32_t)__popcll(m));
                base = wave_bcast0(base);
                if (pass) cidx[base + lanes_below(m)] = (uint32_t)j;
            }
        }
        __syncthreads();
        const uint32_t c = cnt;
        __syncthreads();
        if (c > 0 && (c >= (uint32_t)kFixTop || j0 + kTileCols >= a.n)) {
            flush(c);
            if (tid == 0) cnt = 0;
            __syncthreads();
        }
    }
    for (uint32_t t = tid; t < (uint32_t)a.k; t += kFixThreads) {
        const uint64_t key = top[t];
        const int64_t o = i * a.k + t;
        if (key == kKeyMax) {
            a.out_dist[o] = __uint_as_float(0x7f800000u);
            a.out_idx[o] = -1;
        } else {
            a.out_dist[o] = a.out_scale * ord_to_float(key_ord(key));
            a.out_idx[o] = (int32_t)key_idx(key);
        }
    }
}

template <int G>
static void launch_sqnorm_g(const float *X, int64_t n, int d, float *out, unsigned int *max_bits, bool vec,
                            hipStream_t stream) {
    constexpr int PPW = kWave / G;
    int64_t blocks = (n + 8 * PPW - 1) / (8 * PPW);
    if (blocks > 4096) blocks = 4096;
    if (vec)
        hipLaunchKernelGGL((sqnorm_kernel<G, true>), dim3((unsigned)blocks), dim3(256), 0, stream, X, n, d, out,
                           max_bits);
    else
        hipLaunchKernelGGL((sqnorm_kernel<G, false>), dim3((unsigned)blocks), dim3(256), 0, stream, X, n, d, out,
                           max_bits);
}

hipError_t launch_sqnorm(const float *X, int64_t n, int d, float *out, unsigned int *max_bits, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const bool vec = d % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
    switch (lanes_for(d, vec)) {
        case 1: launch_sqnorm_g<1>(X, n, d, out, max_bits, vec, stream); break;
        case 2: launch_sqnorm_g<2>(X, n, d, out, max_bits, vec, stream); break;
        case 4: launch_sqnorm_g<4>(X, n, d, out, max_bits, vec, stream); break;
        case 8: launch_sqnorm_g<8>(X, n, d, out, max_bits, vec, stream); break;
        case 16: launch_sqnorm_g<16>(X, n, d, out, max_bits, vec, stream); break;
        case 32: launch_sqnorm_g<32>(X, n, d, out, max_bits, vec, stream); break;
        default: launch_sqnorm_g<64>(X, n, d, out, max_bits, vec, stream); break;
    }
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float *src, int64_t n, int d, const int32_t *idx, int64_t rows, float *dst,
                              const float *norms, float *dst_norms, hipStream_t stream) {
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, src, n, d, idx,
                       rows, dst, norms, dst_norms);
    return hipGetLastError();
}

hipError_t launch_flag_rows(const uint32_t *cnt, int64_t m, uint32_t need, uint32_t cap, int force, uint32_t *nflag,
                            int32_t *flags, hipStream_t stream) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(flag_rows_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, cnt, m, need, cap,
                       force, nflag, flags);
    return hipGetLastError();
}

hipError_t launch_scatter_fallback(const int32_t *rows, int64_t nrows, const float *val, const int32_t *idx, int kk,
                                   uint64_t *cand, uint32_t *cnt, int cap, hipStream_t stream) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_fallback_kernel, dim3((unsigned)nrows), dim3(256), 0, stream, rows, nrows, val, idx, kk,
                       cand, cnt, cap);
    return hipGetLastError();
}

hipError_t launch_quantize(const float *X, int64_t n, int d, int prec, void *out, float *scale_out,
                           hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int dq = (d + kQuantPad - 1) / kQuantPad * kQuantPad;
    hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n, d, prec, dq, out,
                       scale_out);
    return hipGetLastError();
}

hipError_t launch_certify(const CertifyArgs &a, hipStream_t stream) {
    if (a.m == 0) return hipSuccess;
    hipLaunchKernelGGL(certify_kernel, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <int G>
static void launch_fixup_g(const FixupArgs &a, bool vec, hipStream_t stream) {
    if (vec)
        hipLaunchKernelGGL((exact_rows_kernel<G, true>), dim3((unsigned)a.nrows), dim3(kFixThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((exact_rows_kernel<G, false>), dim3((unsigned)a.nrows), dim3(kFixThreads), 0, stream, a);
}

hipError_t launch_fixup(const FixupArgs &a, hipStream_t stream) {
    if (a.nrows == 0) return hipSuccess;
    if (a.k < 1 || a.k > kFixTop || a.nrows > 0x7fffffff) return hipErrorInvalidValue;
    // the same lane grouping as the re-rank, so a pair's distance has the same bits
    const bool vec = a.d % 4 == 0 && (reinterpret_cast<uintptr_t>(a.Q) & 15u) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.C) & 15u) == 0;
    switch (lanes_for(a.d, vec)) {
        case 1: launch_fixup_g<1>(a, vec, stream); break;
        case 2: launch_fixup_g<2>(a, vec, stream); break;
        case 4: launch_fixup_g<4>(a, vec, stream); break;
        case 8: launch_fixup_g<8>(a, vec, stream); break;
        case 16: launch_fixup_g<16>(a, vec, stream); break;
        case 32: launch_fixup_g<32>(a, vec, stream); break;
        default: launch_fixup_g<64>(a, vec, stream); break;
    }
    return hipGetLastError();
}

template <int G>
static void launch_rerank_g(const RerankArgs &a, bool vec, hipStream_t stream) {
    if (vec)
        hipLaunchKernelGGL((rerank_kernel<G, true>), dim3((unsigned)a.m), dim3(kRerankThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((rerank_kernel<G, false>), dim3((unsigned)a.m), dim3(kRerankThreads), 0, stream, a);
}

hipError_t launch_rerank(const RerankArgs &a, hipStream_t stream) {
    if (a.m == 0) return hipSuccess;
    if (a.kk > kRerankMax) return hipErrorInvalidValue;
    const bool vec = a.d % 4 == 0 && (reinterpret_cast<uintptr_t>(a.Q) & 15u) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.C) & 15u) == 0;
    switch (lanes_for(a.d, vec)) {
        case 1: launch_rerank_g<1>(a, vec, stream); break;
        case 2: launch_rerank_g<2>(a, vec, stream); break;
        case 4: launch_rerank_g<4>(a, vec, stream); break;
        case 8: launch_rerank_g<8>(a, vec, stream); break;
        case 16: launch_rerank_g<16>(a, vec, stream); break;
        case 32: launch_rerank_g<32>(a, vec, stream); break;
        default: launch_rerank_g<64>(a, vec, stream); break;
    }
    return hipGetLastError();
}

}  // namespace knn
