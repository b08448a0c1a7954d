// Quick multi-select over the rows of a given FP32 distance matrix (Methods,
// "GPU-based quick multi-select").
//
// Coarse level: rows are independent; a persistent grid of workgroups strides
// over them (one workgroup per row at a time, the paper's block-per-query
// variant, with 256-lane workgroups of four 64-lane waves).
//
// Fine level, per row:
//  1. A pivot is chosen from a strided sample of the row (16 blocks of 64
//     contiguous entries, sorted in LDS): its lower median (plain mode), the
//     sample order statistic just above the expected rank of the k-th key
//     (sample mode), or a per-row value supplied by the pivot network.
//  2. The row is streamed once from HBM with 16-byte loads.  Each wave votes
//     "key below pivot" with a 64-lane ballot; a lane's slot is the population
//     count of the set lanes below it (mbcnt), the wave reserves its slots with
//     one LDS atomic on the running counter (the paper's g< counter), and the
//     survivors are written to an on-chip buffer.  Keys at or above the pivot
//     are not needed while L >= K (the paper's K < L case: only the left side is
//     processed) and are not stored.  If L < K the left side is kept (pushed as
//     a segment reference) and the row is streamed again for the band between
//     the old pivot and a higher one.
//  3. Quickselect passes over the survivors, each a two-sided partition from one
//     buffer into the other at the same positions (keys below the pivot from the
//     left end, the others from the right end), K-versus-L recursion, and a stack
//     of segment references to kept left sides instead of copying them.
//  4. The kept keys are gathered, bitonic-sorted in LDS and written out.
//
// Keys are (ordered value, column index), so every key is distinct, every pass
// makes progress and equal values resolve to the lower index.  The on-chip
// buffers hold CAP keys; positions at or above CAP live in a per-workgroup
// global workspace, so overflowing rows stay exact.
#include "internal.hpp"
#include "keys.hpp"

namespace knn {

constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / kWave;
constexpr int kSortN = 1024;        // sample size; also the largest k
constexpr int kSampleBlocks = kSortN / kWave;
constexpr int kStackDepth = 64;
constexpr int kMaxPasses = 4096;    // hard bound; unreachable with distinct keys

template <int CAP>
struct SelSmem {
    uint64_t buf[2][CAP];
    uint64_t sortbuf[kSortN];
    uint64_t finals[kWave];
    uint32_t st_b[kStackDepth];
    uint32_t st_s[kStackDepth];
    uint32_t st_e[kStackDepth];
    uint64_t pivot;
    uint32_t cnt_lt;
    uint32_t cnt_ge;
};

template <int CAP>
struct VBuf {
    SelSmem<CAP> &sm;
    uint64_t *g[2];  // global parts (positions >= CAP), per buffer

    __device__ __forceinline__ uint64_t ld(uint32_t b, uint32_t p) const {
        return p < CAP ? sm.buf[b][p] : g[b][p - CAP];
    }
    __device__ __forceinline__ void st(uint32_t b, uint32_t p, uint64_t v) const {
        if (p < CAP) sm.buf[b][p] = v;
        else g[b][p - CAP] = v;
    }
};

// Wave-level append of the lanes set in `m` into buffer 0 at the running counter.
template <int CAP>
__device__ __forceinline__ void wave_append(const VBuf<CAP> &vb, uint64_t m, bool mine, float v,
                                            uint32_t j) {
    const uint32_t lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&vb.sm.cnt_lt, (uint32_t)__popcll(m));
    base = wave_bcast0(base);
    if (mine) vb.st(0, base + lanes_below(m), make_key(v, j));
}

// Ballot of one entry per lane against the pivot (and, in band passes, the lower
// bound) followed by the wave append of the survivors.
template <int CAP, bool BAND>
__device__ __forceinline__ void vote_append(const VBuf<CAP> &vb, float v, uint32_t j, bool valid,
                                            const Pivot &P, const Pivot &LO) {
    if (!BAND && !P.nan && !P.inf) {
        uint64_t m = __ballot(valid && v < P.pv);
        uint64_t meq = __ballot(valid && v == P.pv);
        if (meq) m |= __ballot(valid && v == P.pv && j < P.pidx);
        if (m) wave_append(vb, m, (m >> lane_id()) & 1ull, v, j);
    } else {
        bool s = valid && key_below(v, j, P) && !(BAND && key_below(v, j, LO));
        uint64_t m = __ballot(s);
        if (m) wave_append(vb, m, s, v, j);
    }
}

// One streaming pass over the row: appends the keys in [LO, P) to buffer 0.
template <int CAP, bool BAND>
__device__ void stream_pass(const VBuf<CAP> &vb, const float *__restrict__ row, uint32_t N,
                            bool vec, const Pivot &P, const Pivot &LO) {
    const uint32_t tid = threadIdx.x;
    constexpr int U = 4;
    if (vec) {
        const uint32_t n4 = N >> 2;
        const f32x4 *r4 = reinterpret_cast<const f32x4 *>(row);
        for (uint32_t it = 0; it < n4; it += kSelThreads * U) {
            f32x4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t i4 = it + u * kSelThreads + tid;
                v[u] = i4 < n4 ? __builtin_nontemporal_load(r4 + i4) : f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t i4 = it + u * kSelThreads + tid;
                bool valid = i4 < n4;
                uint32_t j = i4 * 4;
                vote_append<CAP, BAND>(vb, v[u].x, j + 0, valid, P, LO);
                vote_append<CAP, BAND>(vb, v[u].y, j + 1, valid, P, LO);
                vote_append<CAP, BAND>(vb, v[u].z, j + 2, valid, P, LO);
                vote_append<CAP, BAND>(vb, v[u].w, j + 3, valid, P, LO);
            }
        }
        for (uint32_t j0 = n4 * 4; j0 < N; j0 += kSelThreads) {
            uint32_t j = j0 + tid;
            bool valid = j < N;
            float v = valid ? row[j] : 0.f;
            vote_append<CAP, BAND>(vb, v, j, valid, P, LO);
        }
    } else {
        for (uint32_t j0 = 0; j0 < N; j0 += kSelThreads * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t j = j0 + u * kSelThreads + tid;
                v[u] = j < N ? row[j] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t j = j0 + u * kSelThreads + tid;
                vote_append<CAP, BAND>(vb, v[u], j, j < N, P, LO);
            }
        }
    }
}

// Two-sided partition of segment [s, e) of buffer xb into buffer xb^1 (same
// positions): keys below P from the left end, the others from the right end.
// Returns L, the number of keys below P.
template <int CAP>
__device__ uint32_t partition_pass(const VBuf<CAP> &vb, uint32_t xb, uint32_t s, uint32_t e,
                                   uint64_t P) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t yb = xb ^ 1u;
    if (tid == 0) {
        vb.sm.cnt_lt = 0;
        vb.sm.cnt_ge = 0;
    }
    __syncthreads();
    for (uint32_t p0 = s + wave * kWave; p0 < e; p0 += kSelWaves * kWave) {
        uint32_t p = p0 + lane;
        bool valid = p < e;
        uint64_t key = valid ? vb.ld(xb, p) : kKeyMax;
        bool lt = valid && key < P;
        bool ge = valid && !lt;
        uint64_t mlt = __ballot(lt), mge = __ballot(ge);
        uint32_t bl = 0, bg = 0;
        if (lane == 0) {
            bl = atomicAdd(&vb.sm.cnt_lt, (uint32_t)__popcll(mlt));
            bg = atomicAdd(&vb.sm.cnt_ge, (uint32_t)__popcll(mge));
        }
        bl = wave_bcast0(bl);
        bg = wave_bcast0(bg);
        if (lt) vb.st(yb, s + bl + lanes_below(mlt), key);
        if (ge) vb.st(yb, e - 1 - (bg + lanes_below(mge)), key);
    }
    __syncthreads();
    uint32_t L = vb.sm.cnt_lt;
    __syncthreads();
    return L;
}

// Copies the referenced kept segments into sortbuf[agg...), returns the new agg.
template <int CAP>
__device__ uint32_t flush_stack(const VBuf<CAP> &vb, uint32_t nstack, uint32_t agg) {
    for (uint32_t i = 0; i < nstack; ++i) {
        uint32_t b = vb.sm.st_b[i], s = vb.sm.st_s[i], e = vb.sm.st_e[i];
        for (uint32_t p = s + threadIdx.x; p < e; p += kSelThreads) vb.sm.sortbuf[agg + (p - s)] = vb.ld(b, p);
        agg += e - s;
    }
    __syncthreads();
    return agg;
}

// Pushes a kept segment reference.  Every thread calls it with the same values
// and tracks nstack / agg identically.
template <int CAP>
__device__ void push_seg(const VBuf<CAP> &vb, uint32_t b, uint32_t s, uint32_t e, uint32_t &nstack,
                         uint32_t &agg, bool sortbuf_free) {
    if (s == e) return;
    if (nstack == kStackDepth) {
        // Only reachable after the sample is no longer needed (the stream phase
        // pushes at most a handful of segments).
        (void)sortbuf_free;
        agg = flush_stack(vb, nstack, agg);
        nstack = 0;
    }
    if (threadIdx.x == 0) {
        vb.sm.st_b[nstack] = b;
        vb.sm.st_s[nstack] = s;
        vb.sm.st_e[nstack] = e;
    }
    ++nstack;
    __syncthreads();
}

__device__ __forceinline__ uint32_t target_rank(uint32_t S, uint32_t K, uint32_t len, float z,
                                                float add) {
    float mu = (float)S * (float)K / (float)len;
    float r = mu + z * sqrtf(mu) + add;
    return r >= (float)(S - 1) ? S - 1 : (uint32_t)r;
}

template <int CAP>
__global__ __launch_bounds__(kSelThreads) void select_rows_kernel(SelectArgs a, uint64_t *ws,
                                                                   uint64_t ws_slot) {
    __shared__ SelSmem<CAP> sm;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t N = a.cols, k = a.k;
    VBuf<CAP> vb{sm, {ws + (uint64_t)blockIdx.x * 2 * ws_slot, ws + (uint64_t)blockIdx.x * 2 * ws_slot + ws_slot}};
    const bool vec = ((reinterpret_cast<uintptr_t>(a.dist) & 15u) == 0) && ((a.ld & 3) == 0);

    for (int64_t r = blockIdx.x; r < a.rows; r += gridDim.x) {
        const float *row = a.dist + r * a.ld;
        uint32_t nstack = 0, agg = 0, passes = 0, stream_passes = 0, spill = 0, first = 0;
        uint32_t sb, ss, se, Kp;  // active segment (buffer, start, end) and keys still needed

        if (N <= (uint32_t)CAP) {
            for (uint32_t p = tid; p < N; p += kSelThreads) sm.buf[0][p] = make_key(row[p], p);
            __syncthreads();
            sb = 0; ss = 0; se = N; Kp = k;
        } else {
            // 1. strided sample: 16 blocks of 64 contiguous entries
            for (uint32_t b = wave; b < (uint32_t)kSampleBlocks; b += kSelWaves) {
                uint32_t start = (uint32_t)(((uint64_t)b * (N - kWave)) / (kSampleBlocks - 1));
                uint32_t j = start + lane;
                sm.sortbuf[b * kWave + lane] = make_key(row[j], j);
            }
            __syncthreads();
            block_bitonic_sort<kSelThreads>(sm.sortbuf, kSortN);

            uint32_t rr;
            uint64_t P;
            if (a.mode == kPivotPlain) {
                rr = (kSortN - 1) / 2;
                P = sm.sortbuf[rr];
            } else {
                rr = target_rank(kSortN, k, N, 3.0f, 3.0f);
                P = sm.sortbuf[rr];
                if (a.mode == kPivotLearned && a.pivot_hint) {
                    float h = a.pivot_hint[r];
                    // a usable hint is finite and above the smallest sampled key
                    if (h == h && fabsf(h) <= 3.0e38f) {
                        uint64_t hk = ((uint64_t)ord32(h) << 32);
                        if (hk > sm.sortbuf[0]) P = hk;
                    }
                }
            }
            // 2. streaming passes until at least Kp keys are below the pivot
            uint64_t LOk = 0;
            uint32_t base = 0;
            Kp = k;
            for (;;) {
                if (tid == 0) sm.cnt_lt = base;
                __syncthreads();
                Pivot Pv = make_pivot(P);
                if (LOk == 0) {
                    stream_pass<CAP, false>(vb, row, N, vec, Pv, Pv);
                } else {
                    Pivot Lv = make_pivot(LOk);
                    stream_pass<CAP, true>(vb, row, N, vec, Pv, Lv);
                }
                __syncthreads();
                uint32_t total = sm.cnt_lt;
                __syncthreads();
                uint32_t L = total - base;
                ++stream_passes;
                if (stream_passes == 1) first = L;
                if (total > (uint32_t)CAP) spill = 1;
                if (L >= Kp) {
                    sb = 0; ss = base; se = total;
                    break;
                }
                // too few below the pivot: keep them all, move the band up
                push_seg(vb, 0, base, total, nstack, agg, false);
                Kp -= L;
                base = total;
                LOk = P;
                if (P == kKeyMax) break;  // unreachable: all keys are below the sentinel
                // next pivot: a sample key well above the old one, else the sentinel
                rr = rr * 2 + 8 < (uint32_t)kSortN - 1 ? rr * 2 + 8 : (uint32_t)kSortN - 1;
                while (rr < (uint32_t)kSortN - 1 && sm.sortbuf[rr] <= LOk) ++rr;
                P = sm.sortbuf[rr] > LOk ? sm.sortbuf[rr] : kKeyMax;
            }
        }

        // 3. quickselect passes over the active segment
        uint32_t nfinal = 0;
        for (;;) {
            uint32_t len = se - ss;
            if (Kp == len) {
                push_seg(vb, sb, ss, se, nstack, agg, true);
                break;
            }
            if (passes >= (uint32_t)kMaxPasses) {
                // unreachable (each pass shrinks the segment); reported, never hangs
                if (tid == 0 && a.stats) atomicAdd(&a.stats[kStatErrors], 1ull);
                nfinal = 0;
                break;
            }
            if (len <= (uint32_t)kWave) {
                // finish: sort the (at most 64) remaining keys in one wave
                if (wave == 0) {
                    uint64_t key = lane < len ? vb.ld(sb, ss + lane) : kKeyMax;
                    key = wave_sort64(key);
                    if (lane < Kp) sm.finals[lane] = key;
                }
                nfinal = Kp;
                __syncthreads();
                break;
            }
            if (wave == 0) {
                uint32_t p = ss + (uint32_t)(((uint64_t)lane * len) >> 6);
                uint64_t key = wave_sort64(vb.ld(sb, p));
                uint32_t rk = (a.mode == kPivotPlain) ? 31u : target_rank(kWave, Kp, len, 2.0f, 1.0f);
                uint64_t piv = wave_readlane_u64(key, rk);
                if (lane == 0) sm.pivot = piv;
            }
            __syncthreads();
            uint64_t P = sm.pivot;
            uint32_t L = partition_pass(vb, sb, ss, se, P);
            ++passes;
            uint32_t yb = sb ^ 1u;
            if (Kp < L) {
                sb = yb; se = ss + L;
            } else if (Kp > L) {
                push_seg(vb, yb, ss, ss + L, nstack, agg, true);
                sb = yb; ss = ss + L; Kp -= L;
            } else {
                push_seg(vb, yb, ss, ss + L, nstack, agg, true);
                break;
            }
        }

        // 4. gather kept keys, sort, write out
        agg = flush_stack(vb, nstack, agg);
        for (uint32_t t = tid; t < nfinal; t += kSelThreads) sm.sortbuf[agg + t] = sm.finals[t];
        agg += nfinal;
        const uint32_t kp2 = next_pow2(k);
        // (agg == k on every normal exit)
        for (uint32_t t = agg + tid; t < kp2; t += kSelThreads) sm.sortbuf[t] = kKeyMax;
        __syncthreads();
        block_bitonic_sort<kSelThreads>(sm.sortbuf, kp2);
        for (uint32_t t = tid; t < k; t += kSelThreads) {
            uint64_t key = sm.sortbuf[t];
            uint32_t idx = key_idx(key), o = key_ord(key);
            float v;
            if (key == kKeyMax) {  // only on the reported internal-error path
                v = __uint_as_float(0x7fc00000u);
                idx = 0xFFFFFFFFu;
            } else {
                v = (o == kOrdZero || o == kOrdNaN) ? row[idx] : ord_to_float(o);
            }
            a.out_val[r * k + t] = v;
            a.out_idx[r * k + t] = (int32_t)idx;
        }
        if (tid == 0 && a.stats) {
            atomicAdd(&a.stats[kStatRows], 1ull);
            atomicAdd(&a.stats[kStatPasses], (unsigned long long)passes);
            atomicMax(&a.stats[kStatPassesMax], (unsigned long long)passes);
            atomicAdd(&a.stats[kStatStreamPasses], (unsigned long long)stream_passes);
            atomicAdd(&a.stats[kStatSpillRows], (unsigned long long)spill);
            atomicAdd(&a.stats[kStatFirstSurvivors], (unsigned long long)first);
        }
        __syncthreads();
    }
}

// ---- one partition pass per row, one wave per row (Figures 1-3) -------------
__global__ __launch_bounds__(256) void partition_rows_kernel(const float *__restrict__ in, int64_t rows,
                                                             uint32_t cols, int64_t ld,
                                                             const float *__restrict__ piv_val,
                                                             const int32_t *__restrict__ piv_idx,
                                                             float *__restrict__ out_val,
                                                             int32_t *__restrict__ out_idx,
                                                             int32_t *__restrict__ out_left) {
    const uint32_t lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= rows) return;  // whole wave leaves together
    const float *row = in + r * ld;
    Pivot P = make_pivot(make_key(piv_val[r], (uint32_t)piv_idx[r]));
    float *ov = out_val + r * (int64_t)cols;
    int32_t *oi = out_idx + r * (int64_t)cols;
    uint32_t g_lt = 0, g_ge = 0;  // running counts of each side (wave-uniform)
    for (uint32_t base = 0; base < cols; base += kWave) {
        uint32_t j = base + lane;
        bool valid = j < cols;
        float v = valid ? row[j] : 0.f;
        bool lt = valid && key_below(v, j, P);
        bool ge = valid && !lt;
        uint64_t mlt = __ballot(lt), mge = __ballot(ge);
        if (lt) {
            uint32_t pos = g_lt + lanes_below(mlt);
            ov[pos] = v;
            oi[pos] = (int32_t)j;
        }
        if (ge) {
            uint32_t pos = cols - 1 - (g_ge + lanes_below(mge));
            ov[pos] = v;
            oi[pos] = (int32_t)j;
        }
        g_lt += (uint32_t)__popcll(mlt);
        g_ge += (uint32_t)__popcll(mge);
    }
    if (lane == 0) out_left[r] = (int32_t)g_lt;
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---- host side --------------------------------------------------------------
int select_cap_for_k(uint32_t k) {
    if (k <= 64) return 1024;
    if (k <= 256) return 2048;
    return 4096;
}

template <int CAP>
static int blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, select_rows_kernel<CAP>, kSelThreads, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

int select_grid(int cap, int64_t rows, int num_cu) {
    int per = cap == 1024 ? blocks_per_cu<1024>() : cap == 2048 ? blocks_per_cu<2048>() : blocks_per_cu<4096>();
    int64_t g = (int64_t)per * num_cu;
    if (g > rows) g = rows;
    return g < 1 ? 1 : (int)g;
}

size_t select_ws_bytes(int cap, uint32_t cols, int grid) {
    uint64_t slot = cols > (uint32_t)cap ? (uint64_t)cols - cap : 0;
    return (size_t)grid * 2 * slot * sizeof(uint64_t);
}

hipError_t launch_select(const SelectArgs &a, int cap, int grid, void *ws, hipStream_t stream) {
    uint64_t slot = a.cols > (uint32_t)cap ? (uint64_t)a.cols - cap : 0;
    uint64_t *w = static_cast<uint64_t *>(ws);
    switch (cap) {
        case 1024: hipLaunchKernelGGL(select_rows_kernel<1024>, dim3(grid), dim3(kSelThreads), 0, stream, a, w, slot); break;
        case 2048: hipLaunchKernelGGL(select_rows_kernel<2048>, dim3(grid), dim3(kSelThreads), 0, stream, a, w, slot); break;
        case 4096: hipLaunchKernelGGL(select_rows_kernel<4096>, dim3(grid), dim3(kSelThreads), 0, stream, a, w, slot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_partition(const float *in, int64_t rows, uint32_t cols, int64_t ld, const float *piv_val,
                            const int32_t *piv_idx, float *out_val, int32_t *out_idx, int32_t *out_left,
                            hipStream_t stream) {
    const int waves_per_block = 4;
    int64_t blocks = (rows + waves_per_block - 1) / waves_per_block;
    hipLaunchKernelGGL(partition_rows_kernel, dim3((unsigned)blocks), dim3(waves_per_block * kWave), 0, stream, in,
                       rows, cols, ld, piv_val, piv_idx, out_val, out_idx, out_left);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace knn
