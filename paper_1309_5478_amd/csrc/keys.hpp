// Device helpers shared by the HIP kernels of libknn: ordered keys, wavefront
// vote helpers, in-register and LDS bitonic sorts.  gfx950, wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr uint64_t kKeyMax = ~0ull;       // above every real key (indices are < 2^31)
constexpr uint32_t kOrdNaN = 0xFFFFFFFFu;  // every NaN maps here
constexpr uint32_t kOrdZero = 0x80000000u; // -0 and +0 map here

// Order-preserving map of an FP32 value to uint32 under the total order used by
// selection: -0 == +0, NaN == NaN above +inf, otherwise IEEE order.
__device__ __forceinline__ uint32_t ord32(float v) {
    uint32_t u = __float_as_uint(v);
    u = (v == 0.0f) ? 0u : u;
    uint32_t o = u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
    return (v != v) ? kOrdNaN : o;
}

// ord32 of a value known not to be NaN.
__device__ __forceinline__ uint32_t ord32_not_nan(float v) {
    uint32_t u = __float_as_uint(v);
    u = (v == 0.0f) ? 0u : u;
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}

// Inverse of ord32 for every class that has one representative (not for the
// zero class, which returns +0, nor the NaN class).
__device__ __forceinline__ float ord_to_float(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
    return __uint_as_float(u);
}

// A selection key: value class in the high word, column index in the low word,
// so keys are distinct and ties resolve to the lower index.
__device__ __forceinline__ uint64_t make_key(float v, uint32_t idx) {
    return ((uint64_t)ord32(v) << 32) | idx;
}
// The same from an ordered value class, as a register pair (no 64-bit shift or add).
__device__ __forceinline__ uint64_t key_of(uint32_t ord, uint32_t idx) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 w = {idx, ord};
    return __builtin_bit_cast(uint64_t, w);
}
__device__ __forceinline__ uint32_t key_idx(uint64_t k) { return (uint32_t)k; }
__device__ __forceinline__ uint32_t key_ord(uint64_t k) { return (uint32_t)(k >> 32); }

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// Number of set bits of `m` in lanes below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_bcast0(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// A pivot key prepared for fast comparison against (value, index) pairs.
struct Pivot {
    float pv;       // representative value of the pivot's class (+0 for zeros)
    uint32_t pidx;  // pivot index
    uint32_t nan;   // pivot is in the NaN class
    uint32_t inf;   // pivot is the +infinity sentinel (every key is below)
};

__device__ __forceinline__ Pivot make_pivot(uint64_t key) {
    Pivot p;
    uint32_t o = key_ord(key);
    p.inf = (key == kKeyMax) ? 1u : 0u;
    p.nan = (o == kOrdNaN) ? 1u : 0u;
    p.pv = (o == kOrdZero) ? 0.0f : ord_to_float(o);
    p.pidx = key_idx(key);
    return p;
}

// (v, j) < pivot in the key order.
__device__ __forceinline__ bool key_below(float v, uint32_t j, const Pivot &p) {
    if (p.inf) return true;
    bool lt = p.nan ? (v == v) : (v < p.pv);
    bool eq = p.nan ? (v != v) : (v == p.pv);
    return lt || (eq && j < p.pidx);
}

// The value of lane (lane ^ mask), every lane of the wave active.  Masks 1, 2
// and 8 are single DPP moves (quad permutations, a rotation by 8 within rows
// of 16), mask 4 two DPP moves (half-row mirror, quad reversal), mask 16 a
// swizzle within halves of 32; only mask 32 and others go through the LDS
// crossbar.
__device__ __forceinline__ uint32_t xor_lanes32(uint32_t v, int mask) {
    const int x = (int)v;
    switch (mask) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
        case 4: {
            // lane ^ 7 within groups of 8 (row_half_mirror), then lane ^ 3
            // within quads: (i ^ 7) ^ 3 = i ^ 4
            const int m = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);  // row_half_mirror
            return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);  // quad_perm 3,2,1,0
        }
        case 8: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);  // row_ror:8
        case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);                    // xor 16 in 32
        default: return (uint32_t)__shfl_xor(x, mask);
    }
}

// For masks known at compile time (unrolled loops): the DPP forms above.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    const uint32_t lo = xor_lanes32((uint32_t)v, mask);
    const uint32_t hi = xor_lanes32((uint32_t)(v >> 32), mask);
    return ((uint64_t)hi << 32) | lo;
}

// For masks only known at run time: one LDS-crossbar permute per half.
__device__ __forceinline__ uint64_t shfl_xor_u64_rt(uint64_t v, int mask) {
    const uint32_t lo = __shfl_xor((unsigned int)(uint32_t)v, mask);
    const uint32_t hi = __shfl_xor((unsigned int)(uint32_t)(v >> 32), mask);
    return ((uint64_t)hi << 32) | lo;
}

// A structure at an address that is the same in every lane, held in scalar
// registers (vector loads of the same words, then the first lane's copy).
template <class T>
__device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    T v;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return v;
}

// Ascending bitonic sort of one key per lane across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t other = shfl_xor_u64(key, stride);
            const bool take_min = ((lane & stride) == 0) == ((lane & size) == 0);
            key = ((key < other) == take_min) ? key : other;
        }
    }
    return key;
}

__device__ __forceinline__ uint64_t wave_readlane_u64(uint64_t v, int lane) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of NT * J keys of buf (J = 1, 2, 4 or 8), with the keys
// in registers: thread t holds keys t*J .. t*J + J - 1, so compare-exchange
// partners less than J apart are in the same thread, partners less than 64*J
// apart are in the same wave (one shuffle), and only the strides of J*64 and
// above go through LDS, with a barrier each.
//
// The keys come from load(i) for i in [0, NT * J); buf is the exchange area and
// receives the sorted keys.  With SYNC the threads wait for each other after
// loading (needed when load reads LDS that other threads overwrite).
template <int NT, int J, bool SYNC, class Load>
__device__ __forceinline__ void block_sort_regs_from(uint64_t *buf, Load load) {
    constexpr uint32_t N = (uint32_t)NT * J;
    const uint32_t t = threadIdx.x;
    uint64_t k[J];
#pragma unroll
    for (int j = 0; j < J; ++j) k[j] = load(t * J + j);
    if (SYNC) __syncthreads();
    auto cas = [](uint64_t &lo, uint64_t &hi, bool up) {
        const uint64_t a = lo, b = hi;
        const bool swap = (a > b) == up;
        lo = swap ? b : a;
        hi = swap ? a : b;
    };
#pragma unroll
    for (uint32_t size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < (uint32_t)J) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if ((j & stride) == 0) cas(k[j], k[j + stride], ((t * J + j) & size) == 0);
            } else {
                // partners in other threads: the direction is the same for all J
                // keys of a thread (stride and size are multiples of J), and a
                // key stays where it is exactly when it is already on the side
                // its direction asks for (one compare and one select per key)
                const uint32_t i0 = t * J;
                const bool take_min = ((i0 & stride) == 0) == ((i0 & size) == 0);
                uint64_t o[J];
                if (stride < (uint32_t)J * kWave) {
                    const int ls = (int)(stride / J);
#pragma unroll
                    for (int j = 0; j < J; ++j) o[j] = shfl_xor_u64(k[j], ls);
                } else {
#pragma unroll
                    for (int j = 0; j < J; ++j) buf[i0 + j] = k[j];
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < J; ++j) o[j] = buf[(i0 + j) ^ stride];
                    __syncthreads();
                }
#pragma unroll
                for (int j = 0; j < J; ++j) k[j] = ((k[j] < o[j]) == take_min) ? k[j] : o[j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) buf[t * J + j] = k[j];
    __syncthreads();
}

// In place: every thread loads exactly the positions it later writes.
template <int NT, int J>
__device__ __forceinline__ void block_sort_regs(uint64_t *buf) {
    block_sort_regs_from<NT, J, false>(buf, [buf](uint32_t i) { return buf[i]; });
}

// Ascending sort of the first n keys of buf (n <= MAXJ * NT, MAXJ = 4 or 8):
// pads to the next of NT, 2 NT, 4 NT (, 8 NT) keys with the largest key, then
// sorts in registers (the buffer must hold the padded length).  Callers have
// made the n keys visible (barrier).
template <int NT, int MAXJ = 4>
__device__ __forceinline__ void block_sort(uint64_t *buf, uint32_t n) {
    static_assert(MAXJ == 4 || MAXJ == 8, "4 or 8 keys per thread at most");
    const uint32_t m = n <= (uint32_t)NT ? NT : (n <= 2u * NT ? 2 * NT : (n <= 4u * NT ? 4 * NT : 8 * NT));
    for (uint32_t t = n + threadIdx.x; t < m; t += NT) buf[t] = kKeyMax;
    __syncthreads();
    if (m == (uint32_t)NT)
        block_sort_regs<NT, 1>(buf);
    else if (m == 2u * NT)
        block_sort_regs<NT, 2>(buf);
    else if (MAXJ == 4 || m == 4u * NT)
        block_sort_regs<NT, 4>(buf);
    else
        block_sort_regs<NT, MAXJ>(buf);
}

}  // namespace knn
