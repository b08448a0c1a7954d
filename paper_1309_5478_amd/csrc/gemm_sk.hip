// Short-K distance product for BF16 / FP8 operands with the threshold filter
// (the fused first pass of the quick multi-select), for short operand rows
// (BF16 d <= 256, FP8 d <= 256).
//
// With so short a K loop, the one-tile-per-workgroup product of gemm.hip spends
// most of its time waiting: each tile's operands arrive one 128-byte chunk ahead
// of the matrix cores, the first chunk and the epilogue are not overlapped, and
// LDS carries both operands.  Here a workgroup of eight waves keeps one corpus
// tile of 256 columns (the whole K) resident in LDS and walks its range of query
// rows; each wave computes 32 rows x all 256 columns per step (each query
// fragment feeds eight MFMAs, the corpus fragments come from LDS) and reads its
// query fragments straight from global memory into registers, a few k-steps
// ahead, in a ring that runs on from one row block into the next, so loads are
// in flight during the MFMAs and during the epilogue.  The waves never wait for each
// other after the corpus tile is loaded, so one wave's epilogue overlaps the
// other waves' MFMAs on the same SIMD.
//
// Each dot product uses the same MFMA instruction over the same k-steps in the
// same order as gemm.hip, so the reduced keys are the same bits.
//
// Measured on the k-NN graph of 2^20 x 256 BF16 points with about 1500 keys kept
// per row: 700 TFLOP/s per launch against 464 for the tiled product.  With waves of 64 rows x 128 columns (a query fragment feeding four
// MFMAs, both column halves loading the same fragments) it was 636; without the
// epilogue that loop reached 920, and with the query fragments read from LDS
// instead of global memory 1300: what bounds it is the query fragment loads,
// each touching 32 rows for 32 bytes apiece (the MFMA operand layout), and then
// the epilogue.  Then come the kept keys: the same launch keeping none runs at
// 1108 TFLOP/s.  Appended to its row in the product, each kept key needs a slot
// reservation, an atomic whose result the wave waits for; so each wave appends
// its keys and their rows to a staging part of its own instead, at positions
// that follow from the ballots, and a second pass moves them to the rows
// (graph of 2^20 x 256 points, about a thousand keys kept per row: BF16 21.6 ->
// 19.4 ms per launch with that pass, FP8 21.2 -> 17.0).  A wave whose part is
// full appends the rest directly.
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "dist.hpp"
#include "keys.hpp"

namespace knn {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kSkCols = 256;   // corpus columns resident per workgroup
constexpr int kSkWaves = 8;    // 8 row groups of 32 rows, each wave all 256 columns
constexpr int kSkThreads = 64 * kSkWaves;
constexpr int kSkPad = 16;     // bytes of padding per LDS row (conflict-free 16-byte reads)

template <int PREC, int KB>
struct Sk {
    static constexpr int STEP = PREC == kPrecBF16 ? 32 : 64;  // bytes of a row per MFMA k-step
    static constexpr int STEPS = KB / STEP;
    static constexpr int LS = KB + kSkPad;                    // LDS row stride
    static constexpr int P = PREC == kPrecBF16 ? (STEPS < 4 ? STEPS : 4) : 1;  // prefetch depth in k-steps
    using frag = typename std::conditional<PREC == kPrecBF16, i32x4, i32x8>::type;
};

template <int PREC>
__device__ __forceinline__ f32x16 mfma(i32x8 a, i32x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}
template <int PREC>
__device__ __forceinline__ f32x16 mfma(i32x4 a, i32x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

template <class F>
__device__ __forceinline__ F load_frag(const unsigned char *p) {
    if constexpr (sizeof(F) == 16) {
        return *reinterpret_cast<const i32x4 *>(p);
    } else {
        const i32x4 x = *reinterpret_cast<const i32x4 *>(p), y = *reinterpret_cast<const i32x4 *>(p + 16);
        return F{x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
    }
}

// Staging of the kept keys: wave w of the grid appends up to wcap keys and
// their rows to key[w * wcap ...] / row[w * wcap ...] and leaves its count in
// cnt[w]; wcap = 0 turns staging off.
struct SkStage {
    uint32_t *cnt;
    uint32_t *row;
    uint64_t *key;
    uint32_t wcap;
};

}  // namespace

// grid: col_tiles x row_splits workgroups; workgroup b takes corpus tile
// b % col_tiles and row split b / col_tiles (row blocks of 32, one per wave in
// turn).
template <int PREC, int KB>
__global__ __launch_bounds__(kSkThreads) void dist_gemm_sk_kernel(DistArgs a, uint32_t col_tiles, uint32_t row_splits,
                                                                   SkStage st) {
    using T = Sk<PREC, KB>;
    using F = typename T::frag;
    constexpr int S = T::STEPS, P = T::P, LS = T::LS, STEP = T::STEP;
    constexpr int NB = 8;  // column blocks of 32 per wave
    __shared__ __align__(16) unsigned char sB[kSkCols * LS];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t h = lane / 32, l32 = lane % 32;
    const uint32_t ct = blockIdx.x % col_tiles, rs = blockIdx.x / col_tiles;
    const int64_t col0 = (int64_t)ct * kSkCols;
    const int64_t nrb = (a.m + 31) / 32;
    const int64_t rb0 = nrb * rs / row_splits, rb1 = nrb * (rs + 1) / row_splits;

    const unsigned char *Cq = static_cast<const unsigned char *>(a.Cq);
    constexpr int PER_ROW = KB / 16;
    for (int p = (int)tid; p < kSkCols * PER_ROW; p += kSkThreads) {
        const int r = p / PER_ROW, c = p % PER_ROW;
        i32x4 v = {0, 0, 0, 0};
        if (col0 + r < a.n) v = *reinterpret_cast<const i32x4 *>(Cq + (col0 + r) * a.ldq + c * 16);
        *reinterpret_cast<i32x4 *>(sB + r * LS + c * 16) = v;
    }
    float cn[NB], cs[NB];
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
        const int64_t j = col0 + bj * 32 + l32;
        const bool in = j < a.n;
        cn[bj] = in ? a.cnorm[j] : 0.f;
        cs[bj] = (PREC == kPrecFP8 && in) ? -2.0f * a.cscale[j] : -2.0f;
    }
    const uint32_t gj0 = (uint32_t)(col0 + l32);
    __syncthreads();

    const unsigned char *Qq = static_cast<const unsigned char *>(a.Qq);
    const int64_t mlast = a.m - 1;
    // query fragment (row block rb, k-step s); rows beyond m read row m - 1
    // (their results are never kept)
    auto qfrag = [&](int64_t rb, int s) -> F {
        int64_t row = rb * 32 + l32;
        row = row < mlast ? row : mlast;
        return load_frag<F>(Qq + row * a.ldq + s * STEP + h * (STEP / 2));
    };
    auto bfrag = [&](int s, int bj) -> F {
        return load_frag<F>(sB + (bj * 32 + l32) * LS + s * STEP + h * (STEP / 2));
    };

    // this wave's staging part and its fill (the same in every lane)
    const size_t gw = (size_t)blockIdx.x * kSkWaves + wave;
    uint32_t *const srow = st.row + gw * st.wcap;
    uint64_t *const skey = st.key + gw * st.wcap;
    uint32_t wn = 0;

    F ring[P];
    int64_t rb = rb0 + wave;
    if (rb < rb1) {
#pragma unroll
        for (int p = 0; p < P; ++p) ring[p] = qfrag(rb, p);
    }
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (; rb < rb1; rb += kSkWaves) {
        const int64_t nxt = rb + kSkWaves;
        const bool more = nxt < rb1;
        // the accumulators start from zero (set here, not chosen per k-step:
        // in a rolled loop that choice is a select per accumulator element)
        f32x16 acc[NB];
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) acc[bj] = zero;
        // each corpus fragment is read from LDS where it is used; BF16 takes
        // the k-steps unrolled, FP8 (fragments twice the size) one at a time,
        // so that the eight accumulator blocks and the rest fit 256 registers
#pragma unroll(PREC == kPrecFP8 ? 1 : S)
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int bj = 0; bj < NB; ++bj) {
                const F b = bfrag(s, bj);
                acc[bj] = mfma<PREC>(ring[s % P], b, acc[bj]);
            }
            // refill the slot just read: this block's step s + P, or the next block's
            if (s + P < S) ring[s % P] = qfrag(rb, s + P);
            else if (more) ring[s % P] = qfrag(nxt, s + P - S);
            // keep the loads where the ring puts them (the scheduler would
            // otherwise hoist every step's loads and run out of registers)
            __builtin_amdgcn_sched_barrier(0);
        }

        // epilogue: lanes 0..31 hold rows rb * 32 + l32's threshold, scale and id;
        // element (bj, r) is row 8*(r/4) + 4h + r%4, column gj0 + 32 bj
        const int64_t myrow = rb * 32 + l32;
        const bool rin = myrow < a.m;
        const float tau_l = rin ? a.tau[myrow * a.tau_stride] : 0.f;
        const float qs_l = (PREC == kPrecFP8 && rin) ? a.qscale[myrow] : 1.f;
        int64_t qid_l = -1;
        if (a.self_offset >= 0 && rin) qid_l = a.self_offset + (a.row_ids ? (int64_t)a.row_ids[myrow] : myrow);
        const bool may_self = __ballot(qid_l >= col0 && qid_l < col0 + kSkCols) != 0;
        // the lane half, opaque to the compiler here: the row offsets of the
        // epilogue are then computed in place, not hoisted out of the row-block
        // loop (where they would hold registers through the MFMAs)
        uint32_t hv = h;
        asm volatile("" : "+v"(hv));
        // Instantiated for blocks wholly inside the matrix (no row or column
        // tests) and without own columns (no self test): there each key costs
        // one fused multiply-add and one compare, whose results stay in
        // scalar masks.
        auto epilogue = [&](auto edge_t, auto self_t) {
            constexpr bool EDGE = decltype(edge_t)::value, SELF = decltype(self_t)::value;
            float taus[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) taus[r] = __shfl(tau_l, 8 * (r / 4) + 4 * (int)hv + (r % 4));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rl = 8 * (r / 4) + 4 * (int)hv + (r % 4);
                const int64_t gi = rb * 32 + rl;
                const float tau = taus[r];
                const float qs = PREC == kPrecFP8 ? __shfl(qs_l, rl) : 1.f;
                int64_t qid = -1;
                if (SELF) qid = (int64_t)__shfl((long long)qid_l, rl);
                const bool row_ok = !EDGE || gi < a.m;
                float dp[NB];
                uint64_t m[NB];
                uint64_t any = 0;
#pragma unroll
                for (int bj = 0; bj < NB; ++bj) {
                    const float dot = PREC == kPrecFP8 ? acc[bj][r] * qs : acc[bj][r];
                    dp[bj] = fmaf(cs[bj], dot, cn[bj]);
                    bool pass = dp[bj] <= tau;
                    const uint32_t gj = gj0 + 32 * bj;
                    if (EDGE) pass = pass & row_ok & ((int64_t)gj < a.n);
                    if (SELF) pass = pass & ((int64_t)gj != qid);
                    m[bj] = __ballot(pass);
                    any |= m[bj];
                }
                // most accumulator rows keep nothing: one test for all eight
                if (any == 0) {
                    __builtin_amdgcn_sched_barrier(0);
                    continue;
                }
#pragma unroll
                for (int bj = 0; bj < NB; ++bj) {
                    if (m[bj]) {
                        const bool mine = (m[bj] >> lane) & 1ull;
                        // staged: the position follows from the ballot, and
                        // nothing is waited for
                        const uint32_t nk = (uint32_t)__popcll(m[bj]);
                        if (wn + nk <= st.wcap) {
                            if (mine) {
                                const uint32_t pos = wn + lanes_below(m[bj]);
                                skey[pos] = make_key(dp[bj], gj0 + 32 * bj);
                                srow[pos] = (uint32_t)gi;
                            }
                            wn += nk;
                            continue;
                        }
                        const uint32_t hm = h ? (uint32_t)(m[bj] >> 32) : (uint32_t)m[bj];
                        uint32_t v = 0;
                        if (l32 == 0 && hm) v = atomicAdd(&a.cnt[gi], (uint32_t)__popc(hm));
                        const uint32_t b0 = __shfl(v, 0), b1 = __shfl(v, 32);
                        if (mine) {
                            const uint32_t below = lanes_below(m[bj]) - (h ? (uint32_t)__popc((uint32_t)m[bj]) : 0u);
                            const uint32_t slot = (h ? b1 : b0) + below;
                            if (slot < (uint32_t)a.cap) a.cand[gi * a.cap + slot] = make_key(dp[bj], gj0 + 32 * bj);
                        }
                    }
                }
                // one accumulator row at a time (hoisting the others' work
                // would hold them all in registers)
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        const bool edge = rb * 32 + 32 > a.m || col0 + kSkCols > a.n;
        if (edge) {
            if (may_self) epilogue(std::true_type{}, std::true_type{});
            else epilogue(std::true_type{}, std::false_type{});
        } else {
            if (may_self) epilogue(std::false_type{}, std::true_type{});
            else epilogue(std::false_type{}, std::false_type{});
        }
    }
    if (st.wcap && lane == 0) st.cnt[gw] = wn;
}

// Second pass of the staged keys: each wave of this grid moves one staging
// part's keys to their rows (a slot per key by atomic, as the product does
// without staging; keys beyond a row's capacity are counted, not stored).
__global__ __launch_bounds__(256) void sk_append_kernel(SkStage st, uint64_t nwaves, uint32_t *cnt, uint64_t *cand,
                                                        int cap) {
    const uint64_t w = (uint64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (w >= nwaves) return;
    const uint32_t n = st.cnt[w], lane = threadIdx.x % kWave;
    const uint32_t *__restrict__ srow = st.row + w * st.wcap;
    const uint64_t *__restrict__ skey = st.key + w * st.wcap;
    // two keys per lane at a time, each key loaded with its row, so that both
    // slot reservations are in flight together
    for (uint32_t i = lane; i < n; i += 2 * kWave) {
        const uint32_t j = i + kWave;
        const bool two = j < n;
        const uint32_t r0 = srow[i];
        const uint64_t k0 = skey[i];
        uint32_t r1 = 0;
        uint64_t k1 = 0;
        if (two) {
            r1 = srow[j];
            k1 = skey[j];
        }
        const uint32_t s0 = atomicAdd(&cnt[r0], 1u);
        uint32_t s1 = 0xffffffffu;
        if (two) s1 = atomicAdd(&cnt[r1], 1u);
        if (s0 < (uint32_t)cap) cand[(size_t)r0 * cap + s0] = k0;
        if (s1 < (uint32_t)cap) cand[(size_t)r1 * cap + s1] = k1;
    }
}

// ---- host side --------------------------------------------------------------
static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                    hipSuccess || n < 1)
            n = 256;
        cus = n;
    }
    return cus;
}

bool gemm_sk_applies(const DistArgs &a, int epi) {
    if (epi != kEpiFilter || (a.prec != kPrecBF16 && a.prec != kPrecFP8)) return false;
    if (const char *e = std::getenv("KNN_GEMM_SK"))
        if (e[0] == '0') return false;
    // (FP8 rows of more than 256 bytes are left to the tiled product: not
    // measured here)
    const bool kb_ok = a.prec == kPrecBF16 ? (a.ldq == 256 || a.ldq == 512) : (a.ldq == 128 || a.ldq == 256);
    // enough corpus tiles x row blocks to fill the device
    return kb_ok && a.m >= 256 && a.n >= 8 * kSkCols;
}

template <int PREC, int KB>
static hipError_t launch_sk_t(const DistArgs &a, hipStream_t stream) {
    const uint32_t col_tiles = (uint32_t)((a.n + kSkCols - 1) / kSkCols);
    const int64_t nrb = (a.m + 63) / 64;
    // Row splits: the workgroups resident at a time are those of one split
    // (consecutive ids), all streaming the same rows, so a split's query rows
    // (about 2 MiB of operands) stay in the L2 of every XCD while its workgroups
    // pass over them; and at least two workgroups per CU in all.
    const int64_t rows_l2 = ((int64_t)(2u << 20) / a.ldq) / 64 * 64;
    int64_t splits = (a.m + rows_l2 - 1) / (rows_l2 > 64 ? rows_l2 : 64);
    const int64_t fill = (2 * (int64_t)device_cus() + col_tiles - 1) / col_tiles;
    if (splits < fill) splits = fill;
    const int64_t max_splits = nrb / 8 > 1 ? nrb / 8 : 1;  // >= 8 row blocks (two per row group of waves)
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    const uint64_t grid = (uint64_t)col_tiles * (uint64_t)splits;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    // staging: the waves' counts, then wcap keys and wcap rows per wave
    // (KNN_SK_STAGE=0 turns it off, KNN_SK_STAGE_KEYS caps wcap)
    SkStage st{nullptr, nullptr, nullptr, 0};
    const uint64_t nwaves = grid * kSkWaves;
    const char *off = std::getenv("KNN_SK_STAGE");
    if (a.stage && a.stage_bytes > 0 && a.m <= 0xffffffffll && !(off && off[0] == '0')) {
        const uint64_t head = (nwaves * sizeof(uint32_t) + 255) / 256 * 256;
        uint64_t wcap = (uint64_t)a.stage_bytes > head ? ((uint64_t)a.stage_bytes - head) / (nwaves * 12) : 0;
        if (const char *e = std::getenv("KNN_SK_STAGE_KEYS")) {
            const long v = std::atol(e);
            if (v > 0 && (uint64_t)v < wcap) wcap = (uint64_t)v;
        }
        if (wcap > (1u << 20)) wcap = 1u << 20;
        if (wcap >= 64) {
            char *base = static_cast<char *>(a.stage);
            st.cnt = reinterpret_cast<uint32_t *>(base);
            st.key = reinterpret_cast<uint64_t *>(base + head);
            st.row = reinterpret_cast<uint32_t *>(base + head + nwaves * wcap * sizeof(uint64_t));
            st.wcap = (uint32_t)wcap;
        }
    }
    hipLaunchKernelGGL((dist_gemm_sk_kernel<PREC, KB>), dim3((unsigned)grid), dim3(kSkThreads), 0, stream, a, col_tiles,
                       (uint32_t)splits, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || st.wcap == 0) return e;
    const uint64_t agrid = (nwaves + 3) / 4;
    if (agrid > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sk_append_kernel, dim3((unsigned)agrid), dim3(256), 0, stream, st, nwaves, a.cnt, a.cand, a.cap);
    return hipGetLastError();
}

hipError_t launch_dist_gemm_sk(const DistArgs &a, hipStream_t stream) {
    if (a.m == 0 || a.n == 0) return hipSuccess;
    if (a.prec == kPrecBF16) {
        if (a.ldq == 256) return launch_sk_t<kPrecBF16, 256>(a, stream);
        if (a.ldq == 512) return launch_sk_t<kPrecBF16, 512>(a, stream);
    } else if (a.prec == kPrecFP8) {
        if (a.ldq == 128) return launch_sk_t<kPrecFP8, 128>(a, stream);
        if (a.ldq == 256) return launch_sk_t<kPrecFP8, 256>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace knn
