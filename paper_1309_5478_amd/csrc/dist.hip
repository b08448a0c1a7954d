// Distance kernels (Methods, "Distance calculation"): squared norms, the
// matrix-core product of queries and corpus, the reduced key
// d'_ij = ||c_j||^2 - 2 q_i . c_j (the per-row constant ||q_i||^2 dropped), and the
// exact direct-form re-rank of the surviving candidates.
//
// GEMM: FP32 inputs on v_mfma_f32_32x32x2f32, FP32 accumulation.  A workgroup of
// WM x WN waves computes a (64 WM) x (64 WN) tile; each wave a 64 x 64 block as
// 2 x 2 MFMA blocks of 32 x 32.  Operands are staged through LDS in 32-wide
// k-chunks (row-major, stride 36 floats so that 16-byte fragment reads are
// bank-conflict free), double-buffered: the next chunk's global loads are in
// flight while the current chunk feeds the matrix cores.  Each 16-byte LDS read
// supplies one operand for four consecutive MFMAs (lane half h of MFMA q holds
// k = 8s + 4h + q).
//
// Epilogues: DENSE writes d' (a materialised distance block); FILTER keeps only
// d' <= tau_i and appends (d', j) keys to a per-row candidate list, one global
// reservation per 32-lane half-row per MFMA register.
#include <cstdlib>
#include <cstring>

#include <type_traits>

#include "dist.hpp"
#include "keys.hpp"

namespace knn {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBK = 32;       // k-chunk
constexpr int kLdsStride = 36;  // floats per staged row

// A workgroup tile of BM x BN outputs: WM x WN waves, each wave BI x BJ MFMA
// blocks of 32 x 32.
template <int WM, int WN, int BI, int BJ>
struct Tile {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int BM = 32 * BI * WM;
    static constexpr int BN = 32 * BJ * WN;
};

template <int BM, int BN, int ST>
struct GemmSmem {
    float A[ST][BM][kLdsStride];  // ST operand stages (2: double-buffered)
    float B[ST][BN][kLdsStride];
    float tau[BM];
    int64_t qid[BM];  // global id of each query row (self exclusion), -1 if none
    float qn[BM];
    float qs[BM];     // FP8 row scales 2^-e (1 otherwise)
    float cn[BN];
    float cs[BN];     // -2 * column scale
};

// XCD-aware tile order: workgroups are dispatched round-robin over the eight
// XCDs, so block b runs on XCD b % 8.  Each XCD gets a contiguous range of tile
// ids, walked in groups of G query tiles across the corpus tiles, so that the
// workgroups resident on one XCD share A and B tiles in that XCD's L2.
__device__ __forceinline__ void tile_of_block(uint32_t b, uint32_t tiles_m, uint32_t tiles_n, uint32_t &tm,
                                              uint32_t &tn, bool &valid) {
    const uint32_t T = tiles_m * tiles_n;
    const uint32_t per = (T + 7) / 8;
    uint32_t t = (b % 8) * per + b / 8;
    valid = t < T;
    if (!valid) return;
    constexpr uint32_t G = 4;
    uint32_t group = t / (G * tiles_n);
    uint32_t first = group * G;
    uint32_t gsize = tiles_m - first < G ? tiles_m - first : G;
    uint32_t in = t - group * G * tiles_n;
    tm = first + in % gsize;
    tn = in / gsize;
}

// One 128-byte k-chunk per staged row: 32 FP32, 64 BF16 or 128 FP8 elements.
// Each thread moves 16-byte pieces (row r = f / 8, piece c = f % 8).
template <int NT, int BM, int BN, int PREC, bool VEC>
__device__ __forceinline__ void load_chunk(const DistArgs &a, uint32_t row0, uint32_t col0, uint32_t kc, f32x4 *ra,
                                           f32x4 *rb) {
    constexpr int A4 = BM * 8 / NT;  // 16-byte loads per thread for A
    constexpr int B4 = BN * 8 / NT;
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int x = 0; x < A4 + B4; ++x) {
        const bool isA = x < A4;
        const uint32_t f = tid + NT * (isA ? x : x - A4), r = f / 8, c = f % 8;
        const uint32_t gi = (isA ? row0 : col0) + r;
        const int64_t lim = isA ? a.m : a.n;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if ((int64_t)gi < lim) {
            if (PREC == kPrecF32) {
                const uint32_t k0 = kc * 32 + c * 4;
                const float *p = (isA ? a.Q : a.C) + (int64_t)gi * a.d + k0;
                if (VEC) {
                    if (k0 < (uint32_t)a.d) v = *reinterpret_cast<const f32x4 *>(p);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (k0 + e < (uint32_t)a.d) v[e] = p[e];
                }
            } else {
                const char *p = static_cast<const char *>(isA ? a.Qq : a.Cq) + (int64_t)gi * a.ldq + kc * 128 + c * 16;
                v = *reinterpret_cast<const f32x4 *>(p);
            }
        }
        if (isA) ra[x] = v;
        else rb[x - A4] = v;
    }
}

template <int NT, int BM, int BN, int ST>
__device__ __forceinline__ void store_chunk(GemmSmem<BM, BN, ST> &sm, int buf, const f32x4 *ra, const f32x4 *rb) {
    constexpr int A4 = BM * 8 / NT;
    constexpr int B4 = BN * 8 / NT;
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int x = 0; x < A4; ++x) {
        uint32_t f = tid + NT * x, r = f / 8, c = f % 8;
        *reinterpret_cast<f32x4 *>(&sm.A[buf][r][c * 4]) = ra[x];
    }
#pragma unroll
    for (int x = 0; x < B4; ++x) {
        uint32_t f = tid + NT * x, r = f / 8, c = f % 8;
        *reinterpret_cast<f32x4 *>(&sm.B[buf][r][c * 4]) = rb[x];
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// The MFMAs of one staged 128-byte chunk for a wave's 2 x 2 blocks of 32 x 32.
//  FP32: 4 steps of 8 k; one 16-byte read per operand feeds 4 v_mfma_f32_32x32x2f32
//        (lane half h holds k = 8s + 4h + q of MFMA q).
//  BF16: 4 steps of 16 k; one 16-byte read per operand per v_mfma_f32_32x32x16_bf16
//        (lane half h holds k = 16s + 8h .. +7).
//  FP8:  2 steps of 64 k; two 16-byte reads per operand per
//        v_mfma_scale_f32_32x32x64_f8f6f4 with OCP e4m3 operands and unit scales
//        (lane half h holds k = 64s + 32h .. +31).
template <int BM, int BN, int BI, int BJ, int PREC, int ST>
__device__ __forceinline__ void mma_chunk(GemmSmem<BM, BN, ST> &sm, int cur, uint32_t r0, uint32_t c0, uint32_t h,
                                          uint32_t l32, f32x16 (&acc)[BI][BJ]) {
    if (PREC == kPrecF32) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            f32x4 fa[BI], fb[BJ];
#pragma unroll
            for (int i = 0; i < BI; ++i)
                fa[i] = *reinterpret_cast<const f32x4 *>(&sm.A[cur][r0 + i * 32 + l32][8 * s + 4 * h]);
#pragma unroll
            for (int j = 0; j < BJ; ++j)
                fb[j] = *reinterpret_cast<const f32x4 *>(&sm.B[cur][c0 + j * 32 + l32][8 * s + 4 * h]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int j = 0; j < BJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][q], fb[j][q], acc[i][j], 0, 0, 0);
        }
    } else if (PREC == kPrecBF16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            bf16x8 fb[BJ];
#pragma unroll
            for (int j = 0; j < BJ; ++j)
                fb[j] = *reinterpret_cast<const bf16x8 *>(
                    reinterpret_cast<const char *>(&sm.B[cur][c0 + j * 32 + l32][0]) + 32 * s + 16 * h);
#pragma unroll
            for (int i = 0; i < BI; ++i) {
                const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(
                    reinterpret_cast<const char *>(&sm.A[cur][r0 + i * 32 + l32][0]) + 32 * s + 16 * h);
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            i32x8 fb[BJ];
#pragma unroll
            for (int j = 0; j < BJ; ++j)
                fb[j] = *reinterpret_cast<const i32x8 *>(
                    reinterpret_cast<const char *>(&sm.B[cur][c0 + j * 32 + l32][0]) + 64 * s + 32 * h);
#pragma unroll
            for (int i = 0; i < BI; ++i) {
                const i32x8 fa = *reinterpret_cast<const i32x8 *>(
                    reinterpret_cast<const char *>(&sm.A[cur][r0 + i * 32 + l32][0]) + 64 * s + 32 * h);
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa, fb[j], acc[i][j], 0, 0, 0, 127, 0,
                                                                                127);
            }
        }
    }
}

// One output tile (tm, tn) of one product: staged K loop on the matrix cores,
// then the dense or filter epilogue.  Called by every thread of the workgroup.
template <int WM, int WN, int BI, int BJ, int EPI, int PREC, bool VEC, int ST>
__device__ __forceinline__ void gemm_tile(const DistArgs &a, uint32_t tm, uint32_t tn,
                                          GemmSmem<Tile<WM, WN, BI, BJ>::BM, Tile<WM, WN, BI, BJ>::BN, ST> &sm) {
    using T = Tile<WM, WN, BI, BJ>;
    constexpr int NT = T::NT, BM = T::BM, BN = T::BN;
    constexpr int A4 = BM * 8 / NT;
    constexpr int B4 = BN * 8 / NT;
    static_assert(A4 >= 1 && B4 >= 1 && A4 * NT == BM * 8 && B4 * NT == BN * 8, "tile / thread mismatch");
    const uint32_t row0 = tm * BM, col0 = tn * BN;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t wm = wave % WM, wn = wave / WM;
    const uint32_t r0 = wm * 32 * BI, c0 = wn * 32 * BJ;  // wave origin in the tile
    const uint32_t h = lane / 32, l32 = lane % 32;

    // per-row thresholds / ids / scales and per-column norms / scales for the epilogue
    bool self_hit = false;  // some row's own index falls in this tile's columns
    for (uint32_t t = tid; t < (uint32_t)BM; t += NT) {
        uint32_t gi = row0 + t;
        sm.tau[t] = (EPI == kEpiFilter && gi < a.m) ? a.tau[(int64_t)gi * a.tau_stride] : 0.f;
        sm.qn[t] = (a.qnorm && gi < a.m) ? a.qnorm[gi] : 0.f;
        sm.qs[t] = (PREC == kPrecFP8 && gi < a.m) ? a.qscale[gi] : 1.f;
        const int64_t q = (a.self_offset >= 0 && gi < a.m)
                              ? a.self_offset + (a.row_ids ? (int64_t)a.row_ids[gi] : (int64_t)gi)
                              : (int64_t)-1;
        sm.qid[t] = q;
        self_hit |= q >= (int64_t)col0 && q < (int64_t)col0 + BN;
    }
    for (uint32_t t = tid; t < (uint32_t)BN; t += NT) {
        uint32_t gj = col0 + t;
        sm.cn[t] = gj < a.n ? a.cnorm[gj] : 0.f;
        sm.cs[t] = (PREC == kPrecFP8 && gj < a.n) ? -2.0f * a.cscale[gj] : -2.0f;
    }

    f32x16 acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    constexpr uint32_t per_chunk = PREC == kPrecF32 ? 32 : (PREC == kPrecBF16 ? 64 : 128);
    const uint32_t nk = ((uint32_t)a.d + per_chunk - 1) / per_chunk;
    // (also the barrier that publishes the per-row and per-column values)
    const bool may_self = __syncthreads_or(self_hit) != 0;
    f32x4 ra[A4], rb[B4];
    load_chunk<NT, BM, BN, PREC, VEC>(a, row0, col0, 0, ra, rb);
    store_chunk<NT, BM, BN, ST>(sm, 0, ra, rb);
    __syncthreads();

    // two stages: the next chunk goes to the other buffer while this one is
    // consumed; one stage (half the LDS, so more workgroups per CU): it waits
    // in registers until every wave is done with the buffer
    for (uint32_t kc = 0; kc < nk; ++kc) {
        const int cur = ST == 2 ? (int)(kc & 1) : 0;
        if (kc + 1 < nk) load_chunk<NT, BM, BN, PREC, VEC>(a, row0, col0, kc + 1, ra, rb);
        mma_chunk<BM, BN, BI, BJ, PREC, ST>(sm, cur, r0, c0, h, l32, acc);
        if (ST == 1 && kc + 1 < nk) __syncthreads();
        if (kc + 1 < nk) store_chunk<NT, BM, BN, ST>(sm, ST == 2 ? cur ^ 1 : 0, ra, rb);
        __syncthreads();
    }

    // epilogue: element (i, j) of block (bi, bj), register r, lane l:
    //   row = r0 + bi*32 + 8*(r/4) + 4*h + r%4, col = c0 + bj*32 + l%32
    // d' = ||c_j||^2 - 2 q_i.c_j, with q_i.c_j = acc * qscale_i * cscale_j (FP8).
    // Instantiated four ways so that interior tiles skip the bounds tests and
    // tiles holding no row's own index skip the self test.
    auto epilogue = [&](auto bounds_t, auto self_t) {
        constexpr bool BOUNDS = decltype(bounds_t)::value, SELF = decltype(self_t)::value;
#pragma unroll
        for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t rl = r0 + bi * 32 + 8 * (r / 4) + 4 * h + (r % 4);
                const uint32_t gi = row0 + rl;
                const float tau = EPI == kEpiFilter ? sm.tau[rl] : 0.f;
                const int64_t qid = SELF ? sm.qid[rl] : (int64_t)-1;
                const float qs = PREC == kPrecFP8 ? sm.qs[rl] : 1.f;
#pragma unroll
                for (int bj = 0; bj < BJ; ++bj) {
                    const uint32_t cl = c0 + bj * 32 + l32;
                    const uint32_t gj = col0 + cl;
                    const float cn = sm.cn[cl];
                    const float cs = sm.cs[cl];
                    const float dot = PREC == kPrecFP8 ? acc[bi][bj][r] * qs : acc[bi][bj][r];
                    const float dp = fmaf(cs, dot, cn);
                    const bool in = !BOUNDS || ((gi < a.m) & (gj < a.n));
                    const bool self = SELF && (int64_t)gj == qid;
                    if (EPI == kEpiDense) {
                        // with query norms: ||q||^2 + ||c||^2 - 2 q.c; without: the reduced key d'
                        const float v = a.qnorm ? fmaf(cs, dot, sm.qn[rl] + cn) : dp;
                        if (in) a.out[(int64_t)gi * a.ldo + gj] = self ? __uint_as_float(0x7f800000u) : v;
                    } else {
                        const bool pass = in & !self & (dp <= tau);
                        const uint64_t m = __ballot(pass);
                        if (m) {
                            const uint32_t half = h ? (uint32_t)(m >> 32) : (uint32_t)m;
                            uint32_t v = 0;
                            if (l32 == 0 && half) v = atomicAdd(&a.cnt[gi], (uint32_t)__popc(half));
                            const uint32_t b0 = __shfl(v, 0), b1 = __shfl(v, 32);
                            if (pass) {
                                const uint32_t below = lanes_below(m) - (h ? (uint32_t)__popc((uint32_t)m) : 0u);
                                const uint32_t slot = (h ? b1 : b0) + below;
                                if (slot < (uint32_t)a.cap) a.cand[(int64_t)gi * a.cap + slot] = make_key(dp, gj);
                            }
                        }
                    }
                }
            }
        }
    };
    const bool interior = row0 + BM <= a.m && col0 + BN <= a.n;
    if (interior) {
        if (may_self) epilogue(std::false_type{}, std::true_type{});
        else epilogue(std::false_type{}, std::false_type{});
    } else {
        if (may_self) epilogue(std::true_type{}, std::true_type{});
        else epilogue(std::true_type{}, std::false_type{});
    }
}

template <int WM, int WN, int BI, int BJ, int EPI, int PREC, bool VEC, int ST>
__global__ __launch_bounds__(64 * WM * WN) void dist_gemm_kernel(DistArgs a) {
    using T = Tile<WM, WN, BI, BJ>;
    __shared__ GemmSmem<T::BM, T::BN, ST> sm;
    uint32_t tm, tn;
    bool valid;
    tile_of_block(blockIdx.x, a.tiles_m, a.tiles_n, tm, tn, valid);
    if (!valid) return;  // whole workgroup leaves together
    gemm_tile<WM, WN, BI, BJ, EPI, PREC, VEC, ST>(a, tm, tn, sm);
}

// Grouped product: workgroup b computes item b of a list of (job, row tile,
// column tile) items that the host has put in dispatch order (workgroup b runs
// on XCD b % 8).  One item per workgroup, as in the single product: a
// persistent loop over items would keep the tile set-up live across items and
// spill.
template <int WM, int WN, int BI, int BJ, int EPI, int PREC, bool VEC>
__global__ __launch_bounds__(64 * WM * WN) void dist_gemm_grouped_kernel(const DistArgs *__restrict__ jobs,
                                                                         const GemmItem *__restrict__ items) {
    using T = Tile<WM, WN, BI, BJ>;
    __shared__ GemmSmem<T::BM, T::BN, 2> sm;
    const GemmItem w = uniform_load(items + blockIdx.x);
    const DistArgs a = uniform_load(jobs + w.job);
    gemm_tile<WM, WN, BI, BJ, EPI, PREC, VEC, 2>(a, w.tm, w.tn, sm);
}

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

// ---- host launchers ----------------------------------------------------------
template <int WM, int WN, int BI, int BJ, int EPI, int ST = 2>
static hipError_t launch_gemm_t(const DistArgs &a0, hipStream_t stream) {
    using T = Tile<WM, WN, BI, BJ>;
    DistArgs a = a0;
    a.tiles_m = (uint32_t)((a.m + T::BM - 1) / T::BM);
    a.tiles_n = (uint32_t)((a.n + T::BN - 1) / T::BN);
    uint64_t tiles = (uint64_t)a.tiles_m * a.tiles_n;
    uint64_t grid = ((tiles + 7) / 8) * 8;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid), b(T::NT);
    if (a.prec == kPrecBF16) {
        hipLaunchKernelGGL((dist_gemm_kernel<WM, WN, BI, BJ, EPI, kPrecBF16, true, ST>), g, b, 0, stream, a);
    } else if (a.prec == kPrecFP8) {
        if constexpr (BI * BJ <= 4)
            hipLaunchKernelGGL((dist_gemm_kernel<WM, WN, BI, BJ, EPI, kPrecFP8, true, ST>), g, b, 0, stream, a);
        else
            return hipErrorInvalidValue;
    }
    else if (a.d % 4 == 0)
        hipLaunchKernelGGL((dist_gemm_kernel<WM, WN, BI, BJ, EPI, kPrecF32, true, ST>), g, b, 0, stream, a);
    else
        hipLaunchKernelGGL((dist_gemm_kernel<WM, WN, BI, BJ, EPI, kPrecF32, false, ST>), g, b, 0, stream, a);
    return hipGetLastError();
}

// Tile shapes: small 128 x 128 (4 waves of 64 x 64), wide 128 x 256 (8 waves of
// 64 x 64), big 256 x 256 (8 waves of 128 x 64; FP32 and BF16 only, its FP8
// variant exceeds the register file), and small with one operand stage (half
// the LDS: more workgroups per CU to hide load latency when the K loop is
// short).  Default for products that fill the device: BF16 / FP8 with
// d <= 512 small with one stage, otherwise big (wide for FP8); small for the
// rest.  KNN_GEMM_TILE (small / wide / big / small1) overrides the default
// where the shape is legal.
int gemm_tile_choice(const DistArgs &a) {
    if (a.tile >= kTileSmall && a.tile <= kTileSmall1)
        return (a.tile == kTileBig && a.prec == kPrecFP8) ? kTileWide : a.tile;
    const bool large = a.m >= 2048 && a.n >= 2048;
    int t = kTileSmall;
    if (large && a.prec != kPrecF32 && a.d <= 512) t = kTileSmall1;  // short K loop: latency-bound
    else if (large) t = a.prec == kPrecFP8 ? kTileWide : kTileBig;
    if (const char *e = std::getenv("KNN_GEMM_TILE")) {
        if (!std::strcmp(e, "small")) t = kTileSmall;
        else if (!std::strcmp(e, "wide")) t = kTileWide;
        else if (!std::strcmp(e, "big") && a.prec != kPrecFP8) t = kTileBig;
        else if (!std::strcmp(e, "small1")) t = kTileSmall1;
    }
    return t;
}

hipError_t launch_dist_gemm(const DistArgs &a, int epi, hipStream_t stream) {
    if (a.m == 0 || a.n == 0) return hipSuccess;
    switch (gemm_tile_choice(a)) {
        case kTileBig:
            return epi == kEpiDense ? launch_gemm_t<2, 4, 4, 2, kEpiDense>(a, stream)
                                    : launch_gemm_t<2, 4, 4, 2, kEpiFilter>(a, stream);
        case kTileWide:
            return epi == kEpiDense ? launch_gemm_t<2, 4, 2, 2, kEpiDense>(a, stream)
                                    : launch_gemm_t<2, 4, 2, 2, kEpiFilter>(a, stream);
        case kTileSmall1:
            return epi == kEpiDense ? launch_gemm_t<2, 2, 2, 2, kEpiDense, 1>(a, stream)
                                    : launch_gemm_t<2, 2, 2, 2, kEpiFilter, 1>(a, stream);
        default:
            return epi == kEpiDense ? launch_gemm_t<2, 2, 2, 2, kEpiDense>(a, stream)
                                    : launch_gemm_t<2, 2, 2, 2, kEpiFilter>(a, stream);
    }
}

void gemm_tile_dims(int tile, int *bm, int *bn) {
    switch (tile) {
        case kTileBig: *bm = Tile<2, 4, 4, 2>::BM; *bn = Tile<2, 4, 4, 2>::BN; break;
        case kTileWide: *bm = Tile<2, 4, 2, 2>::BM; *bn = Tile<2, 4, 2, 2>::BN; break;
        default: *bm = Tile<2, 2, 2, 2>::BM; *bn = Tile<2, 2, 2, 2>::BN; break;
    }
}

template <int WM, int WN, int BI, int BJ, int EPI>
static hipError_t launch_grouped_t(const DistArgs *jobs, const GemmItem *items, int64_t grid, int prec,
                                   hipStream_t stream) {
    const dim3 g((unsigned)grid), b(Tile<WM, WN, BI, BJ>::NT);
    if (prec == kPrecBF16)
        hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecBF16, true>), g, b, 0, stream, jobs,
                           items);
    else if (prec == kPrecFP8) {
        if constexpr (BI * BJ <= 4)
            hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecFP8, true>), g, b, 0, stream, jobs,
                               items);
        else
            return hipErrorInvalidValue;
    } else
        hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecF32, true>), g, b, 0, stream, jobs,
                           items);
    return hipGetLastError();
}

hipError_t launch_dist_gemm_grouped(const DistArgs *jobs, const GemmItem *items, int64_t nitems, int prec, int tile,
                                    hipStream_t stream, int epi) {
    if (nitems == 0) return hipSuccess;
    if (nitems > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t grid = nitems;
    if (epi == kEpiDense) {
        if (tile != kTileSmall) return hipErrorInvalidValue;
        return launch_grouped_t<2, 2, 2, 2, kEpiDense>(jobs, items, grid, prec, stream);
    }
    switch (tile) {
        case kTileBig:
            if (prec == kPrecFP8) return hipErrorInvalidValue;  // FP8 has no 256 x 256 instance
            if (prec == kPrecBF16)
                return launch_grouped_t<2, 4, 4, 2, kEpiFilter>(jobs, items, grid, kPrecBF16, stream);
            return launch_grouped_t<2, 4, 4, 2, kEpiFilter>(jobs, items, grid, kPrecF32, stream);
        case kTileWide: return launch_grouped_t<2, 4, 2, 2, kEpiFilter>(jobs, items, grid, prec, stream);
        default: return launch_grouped_t<2, 2, 2, 2, kEpiFilter>(jobs, items, grid, prec, stream);
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
