// Quick multi-select over the rows of a given FP32 distance matrix (Methods,
// "GPU-based quick multi-select").
//
// Coarse level: rows are independent; a persistent grid of workgroups takes
// them one at a time (strided, or claimed from a row counter where row costs
// vary; the paper's block-per-query variant, with 256-lane workgroups of four
// 64-lane waves).
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
//     survivors are written on chip (both buffers while streaming).  Keys at
//     or above the pivot are not needed while L >= K (the paper's K < L case:
//     only the left side is processed) and are not stored.  If L < K every key
//     of the left side belongs to the answer; the row is then streamed again
//     from the start with a higher pivot, which keeps those keys and the band
//     above them as one segment.
//  3. Quickselect passes over the survivors, each a two-sided partition from one
//     buffer into the other at the same positions (keys below the pivot from the
//     left end, the others from the right end), K-versus-L recursion, and a stack
//     of segment references to kept left sides instead of copying them -- until
//     a segment with nothing set aside is short enough to be sorted whole.
//  4. The kept keys are gathered, bitonic-sorted in registers and LDS and
//     written out (or the short segment is sorted and its first k written).
//
// Keys are (ordered value, column index), so every key is distinct, every pass
// makes progress and equal values resolve to the lower index.  The on-chip
// buffers hold CAP keys each; positions beyond them live in a per-workgroup
// global workspace, so overflowing rows stay exact.
#include "internal.hpp"
#include "keys.hpp"
#include "pivot_net.hpp"

namespace knn {

constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / kWave;
constexpr int kSortN = 1024;        // sample size; also the largest k
constexpr int kSampleBlocks = kSortN / kWave;
constexpr int kStackDepth = 64;
constexpr int kMaxPasses = 4096;    // hard bound; unreachable with distinct keys
constexpr int kAccSlots = 10;       // per-workgroup statistics totals

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
    unsigned long long acc[kAccSlots];
    int64_t next_row;
};

// The two partition buffers: positions below CAP live in LDS, the rest in a
// per-workgroup global workspace.  LDS is reached through the kernel's
// __shared__ object passed down by reference (never stored in a struct), so
// LDS accesses stay ds_* instructions.
struct GBuf {
    uint64_t *g0, *g1;
    // select, not an indexed array: a runtime-indexed array would live in scratch
    __device__ __forceinline__ uint64_t *at(uint32_t b) const { return b ? g1 : g0; }
};

// The global side uses relaxed workgroup-scope atomic accesses: they cannot be
// merged with the LDS side into one flat access, and barriers order them.
template <int CAP>
__device__ __forceinline__ uint64_t vld(SelSmem<CAP> &sm, const GBuf &gb, uint32_t b, uint32_t p) {
    if (p < CAP) return sm.buf[b][p];
    return __hip_atomic_load(gb.at(b) + (p - CAP), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <int CAP>
__device__ __forceinline__ void vst(SelSmem<CAP> &sm, const GBuf &gb, uint32_t b, uint32_t p, uint64_t v) {
    if (p < CAP) sm.buf[b][p] = v;
    else __hip_atomic_store(gb.at(b) + (p - CAP), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// While a row is streamed, buffer 0 extends through both LDS buffers: positions
// below 2 CAP are LDS (buffer 1 holding [CAP, 2 CAP)), the rest sit in the
// workspace where buffer 0 keeps them (g0[p - CAP]).  normalize_first moves
// [CAP, 2 CAP) of a streamed range to the workspace, restoring buffer 0's own
// layout before anything else uses the buffers.
template <int CAP>
__device__ __forceinline__ void vst_first(SelSmem<CAP> &sm, const GBuf &gb, uint32_t p, uint64_t v) {
    if (p < 2u * CAP) (&sm.buf[0][0])[p] = v;
    else __hip_atomic_store(gb.g0 + (p - CAP), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <int CAP>
__device__ __forceinline__ void normalize_first(SelSmem<CAP> &sm, const GBuf &gb, uint32_t lo, uint32_t hi) {
    const uint32_t a = lo > (uint32_t)CAP ? lo : (uint32_t)CAP, b = hi < 2u * CAP ? hi : 2u * CAP;
    for (uint32_t p = a + threadIdx.x; p < b; p += kSelThreads)
        __hip_atomic_store(gb.g0 + (p - CAP), sm.buf[1][p - CAP], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
}

// Wave-level append of the lanes set in `m` into buffer 0 at the running counter.
template <int CAP>
__device__ __forceinline__ void wave_append(SelSmem<CAP> &sm, const GBuf &gb, uint64_t m, bool mine, float v,
                                            uint32_t j) {
    const uint32_t lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&sm.cnt_lt, (uint32_t)__popcll(m));
    base = wave_bcast0(base);
    if (mine) vst_first(sm, gb, base + lanes_below(m), make_key(v, j));
}

// Generic vote of one entry per lane: key below P, then the wave append of the
// survivors.  Used for masked tails and pivots in the NaN class or at the
// +infinity sentinel.
template <int CAP>
__device__ __forceinline__ void vote_generic(SelSmem<CAP> &sm, const GBuf &gb, float v, uint32_t j, bool valid,
                                             const Pivot &P) {
    bool s = valid & key_below(v, j, P);
    uint64_t m = __ballot(s);
    if (m) wave_append(sm, gb, m, s, v, j);
}

constexpr uint32_t kStreamU = 4;                      // 16-byte loads per lane per tile
constexpr uint32_t kTile4 = kSelThreads * kStreamU;   // float4s per tile

// Votes one full tile (4 x float4 per lane, 16 entries) against a threshold
// value: entries with v <= tv survive (the threshold key (ord(tv), ~0u) sits
// above every key of that value).  One compare and one ballot per entry, one LDS
// atomic per wave for the whole tile, then each non-empty ballot writes its
// survivors at the running offset plus the lane's mbcnt slot (streaming layout
// of buffer 0).  A survivor is never NaN (the compare is false for NaN), so its
// key skips the NaN class, and when the tile's slots all lie in LDS (the usual
// case) the writes skip the per-entry workspace test.
template <int CAP>
__device__ __forceinline__ void vote_tile_le(SelSmem<CAP> &sm, const GBuf &gb, const f32x4 *x, uint32_t t,
                                             float tv) {
    const uint32_t tid = threadIdx.x;
    uint64_t m[kStreamU * 4];
    uint32_t total = 0;
#pragma unroll
    for (uint32_t u = 0; u < kStreamU; ++u) {
        m[4 * u + 0] = __ballot(x[u].x <= tv);
        m[4 * u + 1] = __ballot(x[u].y <= tv);
        m[4 * u + 2] = __ballot(x[u].z <= tv);
        m[4 * u + 3] = __ballot(x[u].w <= tv);
    }
#pragma unroll
    for (uint32_t i = 0; i < kStreamU * 4; ++i) total += (uint32_t)__popcll(m[i]);
    if (total == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&sm.cnt_lt, total);
    base = wave_bcast0(base);
    const bool in_lds = base + total <= 2u * CAP;  // (uniform)
    const uint32_t j0 = (t * kTile4 + tid) * 4;
#pragma unroll
    for (uint32_t u = 0; u < kStreamU; ++u) {
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) {
            const uint64_t mm = m[4 * u + c];
            if (mm) {
                const float v = x[u][c];
                if (v <= tv) {  // this lane's own vote
                    const uint32_t slot = base + lanes_below(mm);
                    const uint64_t key = key_of(ord32_not_nan(v), j0 + (u * kSelThreads * 4 + c));
                    if (in_lds)
                        (&sm.buf[0][0])[slot] = key;
                    else
                        vst_first(sm, gb, slot, key);
                }
                base += (uint32_t)__popcll(mm);
            }
        }
    }
}

// Full tiles of 256 lanes x 4 x 16 bytes against a threshold value, unmasked,
// software-pipelined over two register sets: the loads of one tile are in flight
// while the other is voted on (no copies between the sets, so the wait counts
// only cover the tile being voted on).
template <int CAP>
__device__ __forceinline__ void stream_tiles_le(SelSmem<CAP> &sm, const GBuf &gb, const f32x4 *__restrict__ r4,
                                                uint32_t full, float tv) {
    const f32x4 *p = r4 + threadIdx.x;
    f32x4 A[kStreamU], B[kStreamU];
    auto load = [&](f32x4 *dst, uint32_t t) {
#pragma unroll
        for (uint32_t u = 0; u < kStreamU; ++u) dst[u] = __builtin_nontemporal_load(p + t * kTile4 + u * kSelThreads);
    };
    load(A, 0);
    uint32_t t = 0;
    for (; t + 2 < full; t += 2) {
        load(B, t + 1);
        vote_tile_le(sm, gb, A, t, tv);
        load(A, t + 2);
        vote_tile_le(sm, gb, B, t + 1, tv);
    }
    if (t + 1 < full) {
        load(B, t + 1);
        vote_tile_le(sm, gb, A, t, tv);
        vote_tile_le(sm, gb, B, t + 1, tv);
    } else {
        vote_tile_le(sm, gb, A, t, tv);
    }
}

// One streaming pass over the row, appending to buffer 0 the keys below P.  A
// threshold-form pivot (index ~0u) of a finite value class on 16-byte aligned
// rows takes the tiled fast path for all full tiles; everything else (NaN-class
// pivots, the +infinity sentinel, misaligned rows, the ragged tail) takes the
// generic one-entry-per-lane loop.
template <int CAP>
__device__ __forceinline__ void stream_pass(SelSmem<CAP> &sm, const GBuf &gb, const float *__restrict__ row,
                                            uint32_t N, bool vec, const Pivot &P) {
    const uint32_t tid = threadIdx.x;
    uint32_t done = 0;
    if (vec && !P.nan && !P.inf && P.pidx == 0xFFFFFFFFu) {
        const uint32_t full = (N >> 2) / kTile4;
        if (full > 0) stream_tiles_le(sm, gb, reinterpret_cast<const f32x4 *>(row), full, P.pv);
        done = full * kTile4 * 4;
    }
    for (uint32_t j0 = done; j0 < N; j0 += kSelThreads) {
        uint32_t j = j0 + tid;
        bool valid = j < N;
        float v = valid ? row[j] : 0.f;
        vote_generic<CAP>(sm, gb, v, j, valid, P);
    }
}

// Two-sided partition of segment [s, e) of buffer xb into buffer xb^1 (same
// positions): keys below P from the left end, the others from the right end.
// Returns L, the number of keys below P.
template <int CAP>
__device__ __forceinline__ uint32_t partition_pass(SelSmem<CAP> &sm, const GBuf &gb, uint32_t xb, uint32_t s, uint32_t e,
                                   uint64_t P) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t yb = xb ^ 1u;
    if (tid == 0) {
        sm.cnt_lt = 0;
        sm.cnt_ge = 0;
    }
    __syncthreads();
    for (uint32_t p0 = s + wave * kWave; p0 < e; p0 += kSelWaves * kWave) {
        uint32_t p = p0 + lane;
        bool valid = p < e;
        uint64_t key = valid ? vld(sm, gb, xb, p) : kKeyMax;
        bool lt = valid && key < P;
        bool ge = valid && !lt;
        uint64_t mlt = __ballot(lt), mge = __ballot(ge);
        uint32_t bl = 0, bg = 0;
        if (lane == 0) {
            bl = atomicAdd(&sm.cnt_lt, (uint32_t)__popcll(mlt));
            bg = atomicAdd(&sm.cnt_ge, (uint32_t)__popcll(mge));
        }
        bl = wave_bcast0(bl);
        bg = wave_bcast0(bg);
        if (lt) vst(sm, gb, yb, s + bl + lanes_below(mlt), key);
        if (ge) vst(sm, gb, yb, e - 1 - (bg + lanes_below(mge)), key);
    }
    __syncthreads();
    uint32_t L = sm.cnt_lt;
    __syncthreads();
    return L;
}

// Copies the referenced kept segments into sortbuf[agg...), returns the new agg.
template <int CAP>
__device__ __forceinline__ uint32_t flush_stack(SelSmem<CAP> &sm, const GBuf &gb, uint32_t nstack, uint32_t agg) {
    for (uint32_t i = 0; i < nstack; ++i) {
        uint32_t b = sm.st_b[i], s = sm.st_s[i], e = sm.st_e[i];
        for (uint32_t p = s + threadIdx.x; p < e; p += kSelThreads) sm.sortbuf[agg + (p - s)] = vld(sm, gb, b, p);
        agg += e - s;
    }
    __syncthreads();
    return agg;
}

// Pushes a kept segment reference.  Every thread calls it with the same values
// and tracks nstack / agg identically.
template <int CAP>
__device__ __forceinline__ void push_seg(SelSmem<CAP> &sm, const GBuf &gb, uint32_t b, uint32_t s, uint32_t e, uint32_t &nstack,
                         uint32_t &agg, bool sortbuf_free) {
    if (s == e) return;
    if (nstack == kStackDepth) {
        // Only reachable after the sample is no longer needed (the stream phase
        // pushes at most a handful of segments).
        (void)sortbuf_free;
        agg = flush_stack(sm, gb, nstack, agg);
        nstack = 0;
    }
    if (threadIdx.x == 0) {
        sm.st_b[nstack] = b;
        sm.st_s[nstack] = s;
        sm.st_e[nstack] = e;
    }
    ++nstack;
    __syncthreads();
}

// Index into an ascending sample of S keys whose element lies just above the
// expected position of the K-th smallest of `len` keys (z standard deviations of
// the binomial count plus `add`).
__device__ __forceinline__ uint32_t target_rank(uint32_t S, uint32_t K, uint32_t len, float z, float add) {
    float mu = (float)S * (float)K / (float)len;
    float r = mu + z * sqrtf(mu) + add;
    return r >= (float)(S - 1) ? S - 1 : (uint32_t)r;
}

// Pivot index into an ascending 64-key sample of a segment of `len` keys of
// which Kp are still needed.  When Kp is in the lower half the pivot is aimed
// just above the Kp-th key (so L >= Kp and the segment shrinks to about Kp);
// in the upper half just below it (so L < Kp, the left side is kept and the
// remaining segment is about len - Kp).  The index is in [1, 63], so both sides
// are non-empty and every pass shrinks the segment.
__device__ __forceinline__ uint32_t lds_pivot_rank(uint32_t Kp, uint32_t len) {
    if (2 * Kp <= len) {
        uint32_t r = target_rank(kWave, Kp, len, 2.0f, 1.0f);
        return r < 1 ? 1 : r;
    }
    float mu = (float)kWave * (float)(len - Kp) / (float)len;
    float up = mu + 2.0f * sqrtf(mu) + 1.0f;
    int r = (kWave - 1) - (int)up;
    return r < 1 ? 1u : (uint32_t)r;
}

// 16 strided blocks of 64 contiguous row entries into sortbuf; each block is
// sorted in registers by its wave (four blocks per wave, loads issued first).
template <int CAP>
__device__ __forceinline__ void load_sample_blocks(SelSmem<CAP> &sm, const float *row, uint32_t N) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    constexpr uint32_t per = kSampleBlocks / kSelWaves;
    float v[per];
    uint32_t j[per];
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        uint32_t b = wave + i * kSelWaves;
        uint32_t start = (uint32_t)(((uint64_t)b * (N - kWave)) / (kSampleBlocks - 1));
        j[i] = start + lane;
        v[i] = row[j[i]];
    }
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        uint32_t b = wave + i * kSelWaves;
        sm.sortbuf[b * kWave + lane] = wave_sort64(make_key(v[i], j[i]));
    }
    __syncthreads();
}

// The 64 smallest keys of 16 sorted blocks of 64 in sortbuf, ascending, in the
// lanes of wave 0 (the other waves return kKeyMax): a tree of pairwise merges
// that keep the lower half (the elementwise minimum of one block and the
// reverse of the other holds exactly the 64 smallest of the pair, as a bitonic
// sequence, which six half-cleaning steps sort).  Called by every thread.
template <int CAP>
__device__ __forceinline__ uint64_t lowest64_of_blocks(SelSmem<CAP> &sm) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t m = kKeyMax;
    for (uint32_t w = 1; w < (uint32_t)kSampleBlocks; w <<= 1) {  // merge width in blocks
        for (uint32_t q = wave; q < (uint32_t)kSampleBlocks / (2 * w); q += kSelWaves) {
            const uint32_t a0 = 2 * q * w * kWave, b0 = a0 + w * kWave;
            const uint64_t x = sm.sortbuf[a0 + lane], y = sm.sortbuf[b0 + (kWave - 1 - lane)];
            m = x < y ? x : y;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) {
                const uint64_t o = shfl_xor_u64(m, st);
                m = ((m < o) == ((lane & st) == 0)) ? m : o;
            }
            if (2 * w < (uint32_t)kSampleBlocks) sm.sortbuf[a0 + lane] = m;
        }
        __syncthreads();
    }
    return wave == 0 ? m : kKeyMax;
}

// The r-th smallest (0-based, r < 64) key of 16 sorted blocks of 64 in sortbuf,
// by an r-step 16-way merge in one wave.  Called by wave 0 only.
template <int CAP>
__device__ __forceinline__ uint64_t merge_rank(SelSmem<CAP> &sm, uint32_t r) {
    const uint32_t lane = lane_id();
    uint32_t pos = 0;
    uint64_t head = lane < (uint32_t)kSampleBlocks ? sm.sortbuf[lane * kWave] : kKeyMax;
    uint64_t mn = kKeyMax;
    for (uint32_t step = 0; step <= r; ++step) {
        mn = head;
#pragma unroll
        for (int off = 1; off < kSampleBlocks; off <<= 1) {
            uint64_t o = shfl_xor_u64(mn, off);
            mn = o < mn ? o : mn;
        }
        mn = wave_readlane_u64(mn, 0);
        if (lane < (uint32_t)kSampleBlocks && head == mn) {
            ++pos;
            head = pos < (uint32_t)kWave ? sm.sortbuf[lane * kWave + pos] : kKeyMax;
        }
    }
    return mn;
}

// Finishing by one register sort of the active segment: possible while nothing
// has been kept aside (so the answer is the segment's k smallest); chosen once
// the segment is at most 4 keys per thread, or 8 when so many keys are still
// needed that another partition pass would shrink it by little.  The sort
// exchanges keys through both LDS buffers (2 CAP >= 8 x 256 keys).  Rows with
// k <= 64 finish in one wave instead.
constexpr uint32_t kDirectMinK = kWave;
constexpr uint32_t kDirectWideK = 512;

template <int CAP>
__device__ __forceinline__ bool direct_sort_fits(uint32_t nstack, uint32_t ss, uint32_t se, uint32_t Kp, uint32_t k) {
    static_assert(2 * CAP >= 8 * kSelThreads, "exchange area");
    const uint32_t len = se - ss;
    if (nstack != 0 || ss != 0 || Kp != k || Kp <= kDirectMinK) return false;
    if (len <= 4u * kSelThreads) return true;
    return len <= 8u * kSelThreads && Kp >= kDirectWideK;
}

// The distance-matrix instance (CAP = 1024, about 26 KB of LDS) is held to 96
// registers so that five workgroups share a CU: with every phase of a row but
// the stream latency-bound, more rows in flight per CU pay for the few
// per-row register reloads and for the longer rows that overflow to the
// workspace.  The larger instances serve rows that fit them whole, as many per
// CU as their LDS allows.
template <int CAP, bool KEYS>
__global__ __launch_bounds__(kSelThreads, KEYS ? 1 : (CAP == kSelectCap ? 5 : (CAP == 2048 ? 3 : 2))) void select_rows_kernel(
    SelectArgs a, uint64_t *ws, uint64_t ws_slot) {
    __shared__ SelSmem<CAP> sm;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    GBuf gb{ws + (uint64_t)blockIdx.x * 2 * ws_slot, ws + (uint64_t)blockIdx.x * 2 * ws_slot + ws_slot};

    // per-workgroup totals of the row statistics, in LDS (kept by thread 0)
    if (tid < kAccSlots) sm.acc[tid] = 0;
    __syncthreads();
    // rows: first the workgroup's own, then the next unclaimed one from the
    // launch's row counter (rows differ in cost, so static striding would
    // leave workgroups idle at the end), or strided without a counter
    for (int64_t r = blockIdx.x; r < a.rows;) {
        // this row's matrix: the launch's own, or one segment of several
        const float *dist = a.dist;
        const uint64_t *keys = a.keys;
        const uint32_t *key_cnt = a.key_cnt;
        int64_t ld = a.ld, lr = r, orow = r;
        uint32_t N = a.cols, k = a.k, kout = a.k, col_off = 0;
        float *out_val = a.out_val;
        int32_t *out_idx = a.out_idx;
        if (!KEYS && a.split > 1) {
            // part p of matrix row r / split
            lr = r / a.split;
            col_off = (uint32_t)(r - lr * a.split) * a.cols;
            const uint32_t rest = a.row_cols - col_off;
            N = rest < a.cols ? rest : a.cols;
            k = k < N ? k : N;
        }
        if (a.segs) {
            const SelectSeg sg = uniform_load(a.segs + __builtin_amdgcn_readfirstlane(a.row_seg[r]));
            dist = sg.dist;
            keys = sg.keys;
            key_cnt = sg.key_cnt;
            ld = sg.ld;
            lr = r - sg.row0;
            orow = lr;
            N = sg.cols;
            k = sg.k;
            kout = k;
            out_val = sg.out_val;
            out_idx = sg.out_idx;
        }
        const float *row = dist + lr * ld + col_off;
        const bool vec = ((reinterpret_cast<uintptr_t>(row) & 15u) == 0) && ((ld & 3) == 0);
        uint32_t nstack = 0, agg = 0, passes = 0, stream_passes = 0, spill = 0, first = 0;
        uint32_t wide_lo = 0, wide_hi = 0;  // streamed range of buffer 0 still in the streaming layout
        long long cyc_sample = 0, cyc_stream = 0;
        uint32_t sb, ss, se, Kp;  // active segment (buffer, start, end) and keys still needed

        if (KEYS) {
            // key-list row (at most CAP keys); a list shorter than k (a row
            // whose candidates are re-done later) is padded with the largest
            // key up to k, so that it is exactly the answer
            const uint32_t c = key_cnt ? key_cnt[lr] : N;
            const uint32_t n = c < N ? c : N;
            const uint32_t len = n < k ? k : n;
            const uint64_t *src = keys + lr * ld;
            for (uint32_t p = tid; p < len; p += kSelThreads) sm.buf[0][p] = p < n ? src[p] : kKeyMax;
            __syncthreads();
            sb = 0; ss = 0; se = len; Kp = k;
        } else if (N <= (uint32_t)CAP) {
            for (uint32_t p = tid; p < N; p += kSelThreads) sm.buf[0][p] = make_key(row[p], p);
            __syncthreads();
            sb = 0; ss = 0; se = N; Kp = k;
        } else {
            // 1. first pivot from a strided sample of the row
            long long t0 = clock64();
            uint64_t P;
            bool sample_sorted = false, sample_loaded = false;
            if (a.mode == kPivotPlain) {
                // lower median of 64 strided entries
                if (wave == 0) {
                    uint32_t j = (uint32_t)(((uint64_t)lane * N) >> 6);
                    uint64_t key = wave_sort64(make_key(row[j], j));
                    uint64_t piv = wave_readlane_u64(key, (kWave - 1) / 2);
                    if (lane == 0) sm.pivot = piv;
                }
                __syncthreads();
                P = sm.pivot;
            } else {
                bool from_net = false;
                if (a.mode == kPivotLearned && a.net) {
                    // learned: 4 sample blocks (one per wave) -> features -> network
                    {
                        const uint32_t j = net_sample_start(wave, N) + lane;
                        sm.sortbuf[tid] = make_key(row[j], j);
                    }
                    __syncthreads();
                    block_sort<kSelThreads>(sm.sortbuf, kNetSample);
                    float *vf = reinterpret_cast<float *>(sm.sortbuf + kNetSample);
                    vf[tid] = ord_to_float(key_ord(sm.sortbuf[tid]));
                    __syncthreads();
                    if (wave == 0) {
                        float x[kNetIn], m, s;
                        net_features(vf, N, k, x, m, s);
                        const float y = net_forward_wave(a.net, x);  // BF16 weights, read from global memory
                        if (lane == 0) sm.pivot = (uint64_t)__float_as_uint(fmaf(s, y, m));
                    }
                    __syncthreads();
                    const float pv = __uint_as_float((uint32_t)sm.pivot);
                    if (pv == pv && fabsf(pv) <= 3.0e38f) {  // unusable predictions fall back to the sample rule
                        P = (uint64_t)ord32(pv) << 32;
                        from_net = true;
                    }
                }
                if (!from_net) {
                    load_sample_blocks(sm, row, N);
                    sample_loaded = true;
                    // aimed above the k-th key's expected sample rank mu: by
                    // two standard deviations where the sample holds a few keys
                    // below it (mu >= 4), where fewer survivors mean fewer that
                    // overflow the LDS buffers and a shorter final sort
                    // (16384 x 65536, k = 1024: 0.44 -> 0.12 partition passes
                    // per row); by three and three more keys where it holds
                    // hardly any, so that a row is rarely streamed twice (rows
                    // of 2^20 at k = 1024: mu = 1)
                    const bool few = (uint64_t)kSortN * k < 4ull * N;
                    uint32_t rr0 = few ? target_rank(kSortN, k, N, 3.0f, 3.0f) : target_rank(kSortN, k, N, 2.0f, 1.0f);
                    if (rr0 < 8) {  // a few merge steps
                        if (wave == 0) {
                            uint64_t piv = merge_rank(sm, rr0);
                            if (lane == 0) sm.pivot = piv;
                        }
                        __syncthreads();
                        P = sm.pivot;
                    } else if (rr0 < (uint32_t)kWave) {  // the merge tree of the lowest 64
                        const uint64_t low = lowest64_of_blocks(sm);
                        if (wave == 0) {
                            const uint64_t piv = wave_readlane_u64(low, (int)rr0);
                            if (lane == 0) sm.pivot = piv;
                        }
                        __syncthreads();
                        P = sm.pivot;
                    } else {
                        block_sort<kSelThreads>(sm.sortbuf, kSortN);
                        sample_sorted = true;
                        P = sm.sortbuf[rr0];
                    }
                }
            }
            long long t1 = clock64();
            cyc_sample += t1 - t0;
            // threshold form: every key of the pivot's value class is below it
            P |= 0xFFFFFFFFull;
            // 2. streaming passes until at least k keys are below the pivot.  A
            // pass that keeps fewer is discarded and the row streamed again
            // from the start with a higher pivot: the keys below the old pivot
            // are below the new one too, so the buffer ends up holding what the
            // kept run plus a band above it would hold, but as one active
            // segment (no kept segment to carry, the direct finish stays open)
            // and through the tiled pass.
            Kp = k;
            for (;;) {
                if (tid == 0) sm.cnt_lt = 0;
                __syncthreads();
                const Pivot Pv = make_pivot(P);
                stream_pass<CAP>(sm, gb, row, N, vec, Pv);
                __syncthreads();
                const uint32_t total = sm.cnt_lt;
                __syncthreads();
                ++stream_passes;
                if (stream_passes == 1) first = total;
                if (total > 2u * CAP) spill = 1;
                wide_lo = 0;
                wide_hi = total;
                if (total >= k || P == kKeyMax) {  // (every key is below the sentinel)
                    sb = 0; ss = 0; se = total;
                    break;
                }
                const uint64_t LOk = P;
                if (!sample_loaded) {
                    load_sample_blocks(sm, row, N);
                    sample_loaded = true;
                }
                if (!sample_sorted) {
                    block_sort<kSelThreads>(sm.sortbuf, kSortN);
                    sample_sorted = true;
                }
                // next pivot: about twice as far into the sample as the old one
                uint32_t lo = 0, hi = kSortN;  // first sample key above LOk
                while (lo < hi) {
                    uint32_t mid = (lo + hi) / 2;
                    if (sm.sortbuf[mid] <= LOk) lo = mid + 1;
                    else hi = mid;
                }
                if (lo >= (uint32_t)kSortN) {
                    P = kKeyMax;
                } else {
                    uint32_t rr = 2 * lo + 8 < (uint32_t)kSortN - 1 ? 2 * lo + 8 : (uint32_t)kSortN - 1;
                    P = sm.sortbuf[rr] | 0xFFFFFFFFull;
                }
            }
            cyc_stream += clock64() - t1;
        }

        // 3. quickselect passes over the active segment, until it is short
        // enough to be sorted where it lies
        long long t2 = clock64();
        uint32_t nfinal = 0;
        bool direct = false;
        for (;;) {
            uint32_t len = se - ss;
            if (direct_sort_fits<CAP>(nstack, ss, se, Kp, k)) {
                direct = true;
                break;
            }
            if (wide_hi > (uint32_t)CAP) normalize_first(sm, gb, wide_lo, wide_hi);
            wide_hi = 0;
            if (Kp == len) {
                push_seg(sm, gb, sb, ss, se, nstack, agg, true);
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
                    uint64_t key = lane < len ? vld(sm, gb, sb, ss + lane) : kKeyMax;
                    key = wave_sort64(key);
                    if (lane < Kp) sm.finals[lane] = key;
                }
                nfinal = Kp;
                __syncthreads();
                break;
            }
            if (wave == 0) {
                uint32_t p = ss + (uint32_t)(((uint64_t)lane * len) >> 6);
                uint64_t key = wave_sort64(vld(sm, gb, sb, p));
                uint32_t rk = (a.mode == kPivotPlain) ? (uint32_t)(kWave - 1) / 2 : lds_pivot_rank(Kp, len);
                uint64_t piv = wave_readlane_u64(key, rk);
                if (lane == 0) sm.pivot = piv;
            }
            __syncthreads();
            uint64_t P = sm.pivot;
            uint32_t L = partition_pass(sm, gb, sb, ss, se, P);
            ++passes;
            uint32_t yb = sb ^ 1u;
            if (Kp < L) {
                sb = yb; se = ss + L;
            } else if (Kp > L) {
                push_seg(sm, gb, yb, ss, ss + L, nstack, agg, true);
                sb = yb; ss = ss + L; Kp -= L;
            } else {
                push_seg(sm, gb, yb, ss, ss + L, nstack, agg, true);
                break;
            }
        }

        // 4. gather kept keys, sort, write out; the next row is claimed now, so
        // that the atomic's round trip overlaps this last phase
        long long t3 = clock64();
        unsigned long long claimed = 0;
        if (tid == 0 && a.next_row) claimed = atomicAdd(a.next_row, 1ull);
        if (!direct) {
            agg = flush_stack(sm, gb, nstack, agg);
            for (uint32_t t = tid; t < nfinal; t += kSelThreads) sm.sortbuf[agg + t] = sm.finals[t];
            agg += nfinal;
            __syncthreads();
        }
        // (agg == k on every normal exit)
        auto emit = [&](uint32_t t, uint64_t key) {
            const int64_t o_at = orow * (int64_t)kout + t;
            if (a.out_keys) {
                // kKeyMax (internal-error path) stays the largest key
                a.out_keys[o_at] = key == kKeyMax ? kKeyMax : key + col_off;
                return;
            }
            uint32_t idx = key_idx(key), o = key_ord(key);
            float v;
            if (key == kKeyMax) {  // only on the reported internal-error path
                v = __uint_as_float(0x7fc00000u);
                idx = 0xFFFFFFFFu;
            } else if (o == kOrdZero || o == kOrdNaN) {
                // the key holds the class, the input its bits
                v = !KEYS ? row[idx] : (a.src ? a.src[lr * a.src_ld + idx] : ord_to_float(o));
            } else {
                v = ord_to_float(o);
            }
            out_val[o_at] = v;
            if (out_idx) out_idx[o_at] = (int32_t)(idx + col_off);
        };
        // a part shorter than k: its missing slots hold the largest key
        if (!KEYS && a.out_keys)
            for (uint32_t t = k + tid; t < kout; t += kSelThreads) a.out_keys[orow * (int64_t)kout + t] = kKeyMax;
        if (direct) {
            // no kept segments: the active segment [0, se) of buffer sb (its
            // tail possibly in the workspace) holds every key below its upper
            // end, and its first k after sorting are the answer; both LDS
            // buffers together are the sort's exchange area
            uint64_t *xb = &sm.buf[0][0];
            const uint32_t len = se;
            if (wide_hi > (uint32_t)CAP) {
                // still in the streaming layout (sb == 0): more than CAP and at
                // most 2 CAP keys, wholly in LDS, sorted in place
                auto load = [&](uint32_t p) { return p < len ? xb[p] : kKeyMax; };
                block_sort_regs_from<kSelThreads, 8, false>(xb, load);
            } else {
                auto load = [&](uint32_t p) { return p < len ? vld(sm, gb, sb, p) : kKeyMax; };
                if (len <= (uint32_t)kSelThreads)
                    block_sort_regs_from<kSelThreads, 1, true>(xb, load);
                else if (len <= 2u * kSelThreads)
                    block_sort_regs_from<kSelThreads, 2, true>(xb, load);
                else if (len <= 4u * kSelThreads)
                    block_sort_regs_from<kSelThreads, 4, true>(xb, load);
                else
                    block_sort_regs_from<kSelThreads, 8, true>(xb, load);
            }
            for (uint32_t t = tid; t < k; t += kSelThreads) emit(t, xb[t]);
        } else if (k <= (uint32_t)kWave) {
            if (wave == 0) {
                uint64_t key = wave_sort64(lane < agg ? sm.sortbuf[lane] : kKeyMax);
                if (lane < k) emit(lane, key);
            }
        } else {
            block_sort<kSelThreads>(sm.sortbuf, agg);
            for (uint32_t t = tid; t < k; t += kSelThreads) emit(t, sm.sortbuf[t]);
        }
        long long t4 = clock64();
        // per-workgroup totals, published once after the last row (all rows'
        // counters share one cache line: per-row atomics would serialise there)
        if (tid == 0) {
            sm.acc[0] += 1;
            sm.acc[1] += passes;
            sm.acc[2] = passes > sm.acc[2] ? passes : sm.acc[2];
            sm.acc[3] += stream_passes;
            sm.acc[4] += spill;
            sm.acc[5] += first;
            sm.acc[6] += (unsigned long long)cyc_sample;
            sm.acc[7] += (unsigned long long)cyc_stream;
            sm.acc[8] += (unsigned long long)(t3 - t2);
            sm.acc[9] += (unsigned long long)(t4 - t3);
            sm.next_row = a.next_row ? (int64_t)claimed + gridDim.x : r + gridDim.x;
        }
        __syncthreads();
        r = sm.next_row;
    }
    if (tid == 0 && a.stats && sm.acc[0]) {
        atomicAdd(&a.stats[kStatRows], sm.acc[0]);
        atomicAdd(&a.stats[kStatPasses], sm.acc[1]);
        atomicMax(&a.stats[kStatPassesMax], sm.acc[2]);
        atomicAdd(&a.stats[kStatStreamPasses], sm.acc[3]);
        atomicAdd(&a.stats[kStatSpillRows], sm.acc[4]);
        atomicAdd(&a.stats[kStatFirstSurvivors], sm.acc[5]);
        atomicAdd(&a.stats[kStatCycSample], sm.acc[6]);
        atomicAdd(&a.stats[kStatCycStream], sm.acc[7]);
        atomicAdd(&a.stats[kStatCycSelect], sm.acc[8]);
        atomicAdd(&a.stats[kStatCycFinal], sm.acc[9]);
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

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Adds the sum of n uint32 values to *out (one atomic per workgroup).
__global__ __launch_bounds__(256) void sum_u32_kernel(const uint32_t *p, int64_t n, unsigned long long *out) {
    __shared__ unsigned long long part[4];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += p[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---- host side --------------------------------------------------------------
int select_cap_for_k(uint32_t k) {
    // 1024 keys per buffer for every k: the first pass keeps about 2k of a long
    // row, and the part beyond the LDS buffer goes to the workspace (mostly L2
    // hits); that costs less than the fifth to half of the workgroups per CU
    // that larger buffers would take away
    (void)k;
    return kSelectCap;
}

template <int CAP>
static int blocks_per_cu() {
    static int cached = 0;  // the library targets one architecture, so one value per kernel
    if (cached == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, select_rows_kernel<CAP, false>, kSelThreads, 0) != hipSuccess ||
            n < 1)
            n = 1;
        cached = n;
    }
    return cached;
}

int select_grid(int cap, int64_t rows, int num_cu) {
    int per = cap == 2048 ? blocks_per_cu<2048>() : cap == 4096 ? blocks_per_cu<4096>() : blocks_per_cu<kSelectCap>();
    int64_t g = (int64_t)per * num_cu;
    if (g > rows) g = rows;
    return g < 1 ? 1 : (int)g;
}

// Workspace: the launch's row counter (in its own 256-byte block), then per
// workgroup two overflow buffers of (cols - cap) keys.
constexpr size_t kSelWsHeader = 256;

size_t select_ws_bytes(int cap, uint32_t cols, int grid) {
    uint64_t slot = cols > (uint32_t)cap ? (uint64_t)cols - cap : 0;
    return kSelWsHeader + (size_t)grid * 2 * slot * sizeof(uint64_t);
}

hipError_t launch_select(const SelectArgs &args, int cap, int grid, void *ws, hipStream_t stream) {
    if (!ws) return hipErrorInvalidValue;
    uint64_t slot = args.cols > (uint32_t)cap ? (uint64_t)args.cols - cap : 0;
    SelectArgs a = args;
    uint64_t *w = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kSelWsHeader);
    // rows claimed from a counter where row costs vary (several matrices; k >
    // 64: overflowing rows and longer finishing sorts; network or plain
    // pivots: extra passes); rows of one matrix with k <= 64 and sample pivots
    // cost about the same and are strided (measured 3 % faster)
    if (a.segs || a.k > (uint32_t)kWave || a.mode != kPivotSample) {
        a.next_row = static_cast<unsigned long long *>(ws);
        // the counter starts at zero in every launch (a kernel, so that
        // captured graphs clear it on every replay)
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, stream, a.next_row, 1);
    }
    switch (cap) {
        case kSelectCap:
            hipLaunchKernelGGL((select_rows_kernel<kSelectCap, false>), dim3(grid), dim3(kSelThreads), 0, stream, a, w,
                               slot);
            break;
        case 2048: hipLaunchKernelGGL((select_rows_kernel<2048, false>), dim3(grid), dim3(kSelThreads), 0, stream, a, w, slot); break;
        case 4096: hipLaunchKernelGGL((select_rows_kernel<4096, false>), dim3(grid), dim3(kSelThreads), 0, stream, a, w, slot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_select_keys(const SelectArgs &args, void *counter, int64_t rows_grid_limit, int num_cu,
                              hipStream_t stream) {
    if (args.cols > (uint32_t)kSelectKeysCap || args.k > (uint32_t)kSelectMaxK) return hipErrorInvalidValue;
    SelectArgs a = args;
    a.next_row = static_cast<unsigned long long *>(counter);
    if (a.next_row) hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, stream, a.next_row, 1);
    static int per = 0;
    if (per == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, select_rows_kernel<kSelectKeysCap, true>, kSelThreads, 0) !=
                hipSuccess ||
            n < 1)
            n = 1;
        per = n;
    }
    int64_t g = (int64_t)per * num_cu;
    if (g > a.rows) g = a.rows;
    if (g > rows_grid_limit) g = rows_grid_limit;
    if (g < 1) g = 1;
    hipLaunchKernelGGL((select_rows_kernel<kSelectKeysCap, true>), dim3((unsigned)g), dim3(kSelThreads), 0, stream, a,
                       (uint64_t *)nullptr, (uint64_t)0);
    return hipGetLastError();
}

// ---- rows split across workgroups -------------------------------------------
// A part is worth its own workgroup once it is long against the work that does
// not scale with its length (the pivot sample, the final sort of about k keys
// and the merge of its k keys).  Smallest part: 32 k columns (a part's k keys stay a small fraction of it) and
// at least 64 Ki columns when the split is chosen here: every part pays a fixed
// cost (sample, sort, its list in the merge) that 16 KiB parts do not amortise
// (8 rows of 2^20, k = 32: 181 us with 4 Ki-column parts, 56 us with 64 Ki).
// A forced split goes down to 4 Ki columns.
static uint64_t split_min_chunk(uint32_t k, bool force) {
    const uint64_t floor = force ? 4096ull : 65536ull;
    return k * 32ull > floor ? k * 32ull : floor;
}

SplitPlan select_split_plan(int64_t rows, uint32_t cols, uint32_t k, int num_cu, bool force) {
    SplitPlan sp{1, 1, cols, 0};
    const int64_t resident = (int64_t)blocks_per_cu<kSelectCap>() * num_cu;
    // enough rows to keep every resident workgroup busy: nothing to gain
    if (rows < 1 || (!force && rows * 2 > resident)) return sp;
    uint32_t group = 2;
    while (2ull * group * k <= (uint64_t)kSelectKeysCap) group *= 2;
    const uint64_t min_chunk = split_min_chunk(k, force);
    // parts for half the resident workgroups: fewer, longer parts measured
    // faster than filling every slot (their streams are latency-bound, and each
    // part's fixed cost grows the merge)
    const int64_t want = force ? INT64_MAX : resident / 2;
    uint32_t parts = 1;
    while (parts < 4096u && rows * (int64_t)parts < want && (uint64_t)cols >= 2ull * parts * min_chunk) parts *= 2;
    for (; parts > 1; parts /= 2) {
        // every part keeps at least one column (the last one may be short)
        const uint64_t chunk = (((uint64_t)cols + parts - 1) / parts + 3) / 4 * 4;
        if ((uint64_t)(parts - 1) * chunk < cols) {
            sp.chunk = (uint32_t)chunk;
            break;
        }
    }
    if (parts < 2) return sp;
    sp.parts = parts;
    sp.group = group;
    sp.grid = select_grid(kSelectCap, rows * parts, num_cu);
    return sp;
}

// Workspace of a split call: the part selection's (header with its row counter,
// overflow buffers), a 256-byte block with the merges' row counter, then two
// key arrays: the parts' lists and the first merge level's.
static size_t split_keys_a(const SplitPlan &sp, int64_t rows, uint32_t k) { return (size_t)rows * sp.parts * k; }
static size_t split_keys_b(const SplitPlan &sp, int64_t rows, uint32_t k) {
    const uint32_t g = sp.group < sp.parts ? sp.group : sp.parts;
    return (size_t)rows * (sp.parts / g) * k;
}

size_t select_split_ws_bytes(const SplitPlan &sp, int64_t rows, uint32_t k) {
    const size_t sel = (select_ws_bytes(kSelectCap, sp.chunk, sp.grid) + 255) / 256 * 256;
    return sel + 256 + (split_keys_a(sp, rows, k) + split_keys_b(sp, rows, k)) * sizeof(uint64_t);
}

hipError_t launch_select_split(const SelectArgs &a, const SplitPlan &sp, void *ws, int num_cu, hipStream_t stream) {
    if (!ws || sp.parts < 2 || a.k > (uint32_t)kSelectMaxK || (uint64_t)sp.group * a.k > (uint64_t)kSelectKeysCap)
        return hipErrorInvalidValue;
    char *w = static_cast<char *>(ws);
    const size_t sel = (select_ws_bytes(kSelectCap, sp.chunk, sp.grid) + 255) / 256 * 256;
    void *counter = w + sel;
    uint64_t *ka = reinterpret_cast<uint64_t *>(w + sel + 256);
    uint64_t *kb = ka + split_keys_a(sp, a.rows, a.k);
    // 1. every part's k smallest keys, global column indices
    SelectArgs pa = a;
    pa.rows = a.rows * sp.parts;
    pa.cols = sp.chunk;
    pa.row_cols = a.cols;
    pa.split = sp.parts;
    pa.out_keys = ka;
    pa.out_val = nullptr;
    pa.out_idx = nullptr;
    hipError_t e = launch_select(pa, kSelectCap, sp.grid, ws, stream);
    if (e != hipSuccess) return e;
    // 2. merge levels: `group` lists of k keys per merged row
    uint64_t *in = ka, *out = kb;
    for (uint32_t cur = sp.parts; cur > 1;) {
        const uint32_t g = sp.group < cur ? sp.group : cur, next = cur / g;
        SelectArgs m{};
        m.keys = in;
        m.rows = a.rows * next;
        m.cols = g * a.k;
        m.ld = (int64_t)g * a.k;
        m.k = a.k;
        m.mode = kPivotSample;
        if (next == 1) {
            m.out_val = a.out_val;
            m.out_idx = a.out_idx;
            m.src = a.dist;
            m.src_ld = a.ld;
        } else {
            m.out_keys = out;
        }
        if ((e = launch_select_keys(m, counter, m.rows, num_cu, stream)) != hipSuccess) return e;
        uint64_t *t = in;
        in = out;
        out = t;
        cur = next;
    }
    return hipSuccess;
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

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_sum_u32(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(sum_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, out);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace knn
