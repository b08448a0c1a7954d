// Host/device interface of the distance kernels (dist.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

enum : int { kEpiDense = 0, kEpiFilter = 1 };

struct DistArgs {
    const float *Q;        // m x d queries
    int64_t m;
    const float *C;        // n x d corpus
    int64_t n;
    int d;
    const float *cnorm;    // n squared norms of the corpus rows
    const float *qnorm;    // kEpiDense only: if set, ||q_i||^2 is added (full squared distance)
    // self exclusion: when self_offset >= 0, query row i has global id
    // self_offset + (row_ids ? row_ids[i] : i) and corpus column j == that id is excluded
    int64_t self_offset;
    const int32_t *row_ids;
    // kEpiDense: d' into out (row stride ldo); excluded entries get +inf
    float *out;
    int64_t ldo;
    // kEpiFilter: keep d' <= tau[i * tau_stride]; append keys to cand[i * cap + ...]
    const float *tau;
    int64_t tau_stride;
    uint32_t *cnt;
    uint64_t *cand;
    int cap;
    // filled by the launcher
    uint32_t tiles_m, tiles_n;
};

struct RerankArgs {
    const float *Q;         // m x d
    int64_t m;
    const float *C;         // corpus, n x d
    int64_t n;
    int d;
    const int32_t *cidx;    // m x kk candidate corpus indices
    uint32_t kk;
    int k;
    float *out_dist;        // m x k
    int32_t *out_idx;       // m x k
};

hipError_t launch_dist_gemm(const DistArgs &a, int epi, hipStream_t stream);
hipError_t launch_sqnorm(const float *X, int64_t n, int d, float *out, hipStream_t stream);
hipError_t launch_gather_rows(const float *src, int64_t n, int d, const int32_t *idx, int64_t rows, float *dst,
                              const float *norms, float *dst_norms, hipStream_t stream);
hipError_t launch_flag_rows(const uint32_t *cnt, int64_t m, uint32_t need, uint32_t cap, int force, uint32_t *nflag,
                            int32_t *flags, hipStream_t stream);
hipError_t launch_scatter_fallback(const int32_t *rows, int64_t nrows, const float *val, const int32_t *idx, int kk,
                                   uint64_t *cand, uint32_t *cnt, int cap, hipStream_t stream);
hipError_t launch_rerank(const RerankArgs &a, hipStream_t stream);

}  // namespace knn
