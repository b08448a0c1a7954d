// The distance product (Methods, "Distance calculation": the dot products of
// all query / corpus pairs as one matrix product), fused with the reduced key
// d'_ij = ||c_j||^2 - 2 q_i . c_j (the per-row constant ||q_i||^2 dropped).
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

// 16-byte aligned: the staging writes and fragment reads are then single
// ds_write_b128 / ds_read_b128 (8-byte alignment split each into two 8-byte
// accesses; 16384-row BF16 product at d = 1024: 27.4 -> 24.4 ms)
template <int BM, int BN, int ST>
struct __align__(16) GemmSmem {
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
template <int WM, int WN, int BI, int BJ, int EPI, int PREC, bool VEC, int ST>
__global__ __launch_bounds__(64 * WM * WN) void dist_gemm_grouped_kernel(const DistArgs *__restrict__ jobs,
                                                                         const GemmItem *__restrict__ items) {
    using T = Tile<WM, WN, BI, BJ>;
    __shared__ GemmSmem<T::BM, T::BN, ST> sm;
    const GemmItem w = uniform_load(items + blockIdx.x);
    const DistArgs a = uniform_load(jobs + w.job);
    gemm_tile<WM, WN, BI, BJ, EPI, PREC, VEC, ST>(a, w.tm, w.tn, sm);
}

// Persistent grouped product: a resident grid whose workgroups take items from
// eight atomic queues, one per XCD (workgroup b is dispatched to XCD b % 8 and
// takes the items b % 8, b % 8 + 8, ... of the same dispatch-ordered list, so
// the per-XCD tile order, and with it the L2 reuse, is that of the one-item-per-
// workgroup launch).  Each queue's counter starts at zero.
template <int WM, int WN, int BI, int BJ, int EPI, int PREC, bool VEC>
__global__ __launch_bounds__(64 * WM * WN) void dist_gemm_queue_kernel(const DistArgs *__restrict__ jobs,
                                                                       const GemmItem *__restrict__ items,
                                                                       uint32_t nitems, uint32_t *__restrict__ queues) {
    using T = Tile<WM, WN, BI, BJ>;
    __shared__ GemmSmem<T::BM, T::BN, 2> sm;
    __shared__ uint32_t claimed;
    const uint32_t xcd = blockIdx.x % 8;
    for (;;) {
        if (threadIdx.x == 0) claimed = xcd + 8u * atomicAdd(&queues[xcd], 1u);
        // (also: every wave is done with the previous item's LDS)
        __syncthreads();
        const uint32_t it = claimed;
        if (it >= nitems) break;  // uniform: the whole workgroup leaves together
        const GemmItem w = uniform_load(items + it);
        const DistArgs a = uniform_load(jobs + w.job);
        gemm_tile<WM, WN, BI, BJ, EPI, PREC, VEC, 2>(a, w.tm, w.tn, sm);
        __syncthreads();  // `claimed` is read by every thread before it is rewritten
    }
}

__global__ void zero_queues_kernel(uint32_t *q) {
    if (threadIdx.x < 8) q[threadIdx.x] = 0;
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
// the LDS: more workgroups per CU to hide load latency).  Default: small with
// one stage.  One chunk of prefetch inside a workgroup does not hide the loads
// behind a chunk's MFMAs; more resident workgroups per CU do, in every
// precision (32768 x 262144, d = 1024: BF16 22.6 ms against 24.4 for big and
// 29.8 for wide; FP32 136.0 against 138.0 for big; 32768 x 2^20, d = 256,
// FP32: 147.7 against 156.1).  KNN_GEMM_TILE (small / wide / big / small1)
// overrides the default where the shape is legal.
int gemm_tile_choice(const DistArgs &a) {
    if (a.tile >= kTileSmall && a.tile <= kTileSmall1)
        return (a.tile == kTileBig && a.prec == kPrecFP8) ? kTileWide : a.tile;
    int t = kTileSmall1;
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
    // short reduced-precision rows: the resident-corpus product (gemm_sk.hip)
    if (gemm_sk_applies(a, epi)) return launch_dist_gemm_sk(a, stream);
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

template <int WM, int WN, int BI, int BJ, int EPI, int PREC>
static int queue_grid(int64_t nitems, int num_cu) {
    static int per = 0;  // resident workgroups per CU of this instance
    if (per == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dist_gemm_queue_kernel<WM, WN, BI, BJ, EPI, PREC, true>,
                                                         Tile<WM, WN, BI, BJ>::NT, 0) != hipSuccess || n < 1)
            n = 1;
        per = n;
    }
    int64_t g = (int64_t)per * num_cu;
    const int64_t need = (nitems + 7) / 8 * 8;
    if (g > need) g = need;
    g = (g + 7) / 8 * 8;  // every XCD queue has workgroups
    return (int)g;
}

template <int WM, int WN, int BI, int BJ, int EPI>
static hipError_t launch_queue_t(const DistArgs *jobs, const GemmItem *items, int64_t nitems, int prec,
                                 uint32_t *queues, int num_cu, hipStream_t stream) {
    const dim3 b(Tile<WM, WN, BI, BJ>::NT);
    hipLaunchKernelGGL(zero_queues_kernel, dim3(1), dim3(64), 0, stream, queues);
    if (prec == kPrecBF16) {
        const dim3 g(queue_grid<WM, WN, BI, BJ, EPI, kPrecBF16>(nitems, num_cu));
        hipLaunchKernelGGL((dist_gemm_queue_kernel<WM, WN, BI, BJ, EPI, kPrecBF16, true>), g, b, 0, stream, jobs, items,
                           (uint32_t)nitems, queues);
    } else if (prec == kPrecFP8) {
        if constexpr (BI * BJ <= 4) {
            const dim3 g(queue_grid<WM, WN, BI, BJ, EPI, kPrecFP8>(nitems, num_cu));
            hipLaunchKernelGGL((dist_gemm_queue_kernel<WM, WN, BI, BJ, EPI, kPrecFP8, true>), g, b, 0, stream, jobs,
                               items, (uint32_t)nitems, queues);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        const dim3 g(queue_grid<WM, WN, BI, BJ, EPI, kPrecF32>(nitems, num_cu));
        hipLaunchKernelGGL((dist_gemm_queue_kernel<WM, WN, BI, BJ, EPI, kPrecF32, true>), g, b, 0, stream, jobs, items,
                           (uint32_t)nitems, queues);
    }
    return hipGetLastError();
}

template <int WM, int WN, int BI, int BJ, int EPI, int ST = 2>
static hipError_t launch_grouped_t(const DistArgs *jobs, const GemmItem *items, int64_t grid, int prec,
                                   hipStream_t stream) {
    const dim3 g((unsigned)grid), b(Tile<WM, WN, BI, BJ>::NT);
    if (prec == kPrecBF16)
        hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecBF16, true, ST>), g, b, 0, stream, jobs,
                           items);
    else if (prec == kPrecFP8) {
        if constexpr (BI * BJ <= 4)
            hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecFP8, true, ST>), g, b, 0, stream,
                               jobs, items);
        else
            return hipErrorInvalidValue;
    } else
        hipLaunchKernelGGL((dist_gemm_grouped_kernel<WM, WN, BI, BJ, EPI, kPrecF32, true, ST>), g, b, 0, stream, jobs,
                           items);
    return hipGetLastError();
}

hipError_t launch_dist_gemm_queue(const DistArgs *jobs, const GemmItem *items, int64_t nitems, int prec, int tile,
                                  uint32_t *queues, int num_cu, hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    if (nitems > 0x7ffffff0 || !queues) return hipErrorInvalidValue;
    switch (tile) {
        case kTileBig:
            if (prec == kPrecFP8) return hipErrorInvalidValue;
            return launch_queue_t<2, 4, 4, 2, kEpiFilter>(jobs, items, nitems, prec, queues, num_cu, stream);
        case kTileWide: return launch_queue_t<2, 4, 2, 2, kEpiFilter>(jobs, items, nitems, prec, queues, num_cu, stream);
        default: return launch_queue_t<2, 2, 2, 2, kEpiFilter>(jobs, items, nitems, prec, queues, num_cu, stream);
    }
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
        case kTileSmall1: return launch_grouped_t<2, 2, 2, 2, kEpiFilter, 1>(jobs, items, grid, prec, stream);
        default: return launch_grouped_t<2, 2, 2, 2, kEpiFilter>(jobs, items, grid, prec, stream);
    }
}

}  // namespace knn
