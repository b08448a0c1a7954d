// Host/device interface of the distance kernels (dist.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

enum : int { kEpiDense = 0, kEpiFilter = 1 };
enum : int { kPrecF32 = 0, kPrecBF16 = 1, kPrecFP8 = 2 };
enum : int { kTileSmall = 0, kTileWide = 1, kTileBig = 2, kTileSmall1 = 3 };

// Quantised operands (BF16 / FP8): rows padded with zeros to a multiple of
// kQuantPad elements, so every 128-byte k-chunk load is in bounds.
constexpr int kQuantPad = 128;

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
    // operand precision; for BF16 / FP8 the product reads Qq / Cq (row stride
    // ldq bytes) and, for FP8, undoes the per-row power-of-two scales
    // qscale_i * cscale_j in the epilogue
    int prec;
    const void *Qq;
    const void *Cq;
    int64_t ldq;
    const float *qscale;
    const float *cscale;
    // tile shape (kTile*), or -1 for the default choice of gemm_tile_choice
    int tile = -1;
    // FILTER with the resident-corpus product only (optional): stage_bytes of
    // device memory where each wave appends its kept keys without atomics; a
    // second pass then appends them to the rows (cnt / cand as above).  Null:
    // every kept key is appended to its row in the product itself.
    void *stage = nullptr;
    int64_t stage_bytes = 0;
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
    int64_t self_offset = -1;  // >= 0: row i's own corpus index self_offset + i is never returned
    float out_scale = 1.0f;    // returned distance = out_scale * the direct-form sum (a power of two)
};

hipError_t launch_dist_gemm(const DistArgs &a, int epi, hipStream_t stream);

// ---- grouped product (batches) ---------------------------------------------
struct GemmItem {
    uint32_t job, tm, tn;
};
// Rows x columns of a tile shape (kTile*).
void gemm_tile_dims(int tile, int *bm, int *bn);
// One workgroup per item: jobs is a device array of DistArgs (tiles_m /
// tiles_n / tile unused), items a device array of nitems tiles of the shape
// `tile`, in dispatch order (item b runs on XCD b % 8).  FP32 jobs need
// d % 4 == 0.  The DENSE epilogue only with the small tile.
hipError_t launch_dist_gemm_grouped(const DistArgs *jobs, const GemmItem *items, int64_t nitems, int prec, int tile,
                                    hipStream_t stream, int epi = kEpiFilter);
// The same items (FILTER epilogue) taken by a resident grid from eight per-XCD
// atomic queues instead of one workgroup per item; `queues` is 8 uint32 of
// device memory (cleared by the launch).
hipError_t launch_dist_gemm_queue(const DistArgs *jobs, const GemmItem *items, int64_t nitems, int prec, int tile,
                                  uint32_t *queues, int num_cu, hipStream_t stream);
// The resident-corpus product for short BF16 / FP8 rows with the FILTER
// epilogue (gemm_sk.hip): whether it serves `a` (KNN_GEMM_SK=0 turns it off),
// and its launch.  launch_dist_gemm uses it where it applies.
bool gemm_sk_applies(const DistArgs &a, int epi);
hipError_t launch_dist_gemm_sk(const DistArgs &a, hipStream_t stream);
// Tile shape launch_dist_gemm uses for `a` (kTile*).
int gemm_tile_choice(const DistArgs &a);
// Squared norms of n rows of d floats into out; with max_bits (non-null, zero or
// a smaller value at launch) the largest norm's FP32 bits are folded in too.
hipError_t launch_sqnorm(const float *X, int64_t n, int d, float *out, unsigned int *max_bits, hipStream_t stream);
hipError_t launch_gather_rows(const float *src, int64_t n, int d, const int32_t *idx, int64_t rows, float *dst,
                              const float *norms, float *dst_norms, hipStream_t stream);
hipError_t launch_flag_rows(const uint32_t *cnt, int64_t m, uint32_t need, uint32_t cap, int force, uint32_t *nflag,
                            int32_t *flags, hipStream_t stream);
hipError_t launch_scatter_fallback(const int32_t *rows, int64_t nrows, const float *val, const int32_t *idx, int kk,
                                   uint64_t *cand, uint32_t *cnt, int cap, hipStream_t stream);
hipError_t launch_rerank(const RerankArgs &a, hipStream_t stream);
// Quantises n x d FP32 rows to BF16 (prec 1) or OCP e4m3 with a per-row
// power-of-two scale (prec 2) into rows of dq = round_up(d, kQuantPad)
// elements; scale_out (FP8 only) receives 2^-e per row.
hipError_t launch_quantize(const float *X, int64_t n, int d, int prec, void *out, float *scale_out,
                           hipStream_t stream);
// Per-row certificate of a candidate list.  The reduced key of column j,
// ||c_j||^2 - 2 q_i.c_j, is computed with an error of at most
//   E_i = (gamma + 2u) max ||c||^2 + 2 (rel + 2u) ||q_i|| max ||c||
// (gamma: the FP32 norm reduction over d terms; rel: the relative error of the
// dot product in the operand precision; 2u: the final fused multiply-add).  A row
// is certified when the gap between its kk-th and k-th candidate keys exceeds
// 2 E_i: then every point outside the candidates has a larger exact key than the
// k-th candidate, so the exact top k lie among the candidates.  Uncertified rows
// are counted into *count and, when `list` is set, appended to list (count in
// *nlist) with the threshold key_k + 2 E_i in tfix[i], which bounds the reduced
// key of every exact top-k point of the row (NaN or infinite when no bound
// exists).
struct CertifyArgs {
    const float *sorted_keys;  // m x kk, ascending
    int64_t m;
    int kk, k;
    const float *qnorm2;       // m squared query norms
    const unsigned int *cmax2_bits;
    float rel, gamma;
    unsigned long long *count;
    int32_t *list;             // or null
    uint32_t *nlist;
    float *tfix;               // m thresholds (only uncertified rows written)
    int force;                 // treat every row as uncertified
};
hipError_t launch_certify(const CertifyArgs &a, hipStream_t stream);

// Exact re-run of listed rows (uncertified FP32 rows) from their materialised
// reduced-key rows: every column whose key is at most the row's threshold tfix
// is re-ranked by its exact FP32 direct-form distance (the same arithmetic as
// the re-rank), and the k smallest (distance, index) pairs are written to the
// row's output.  Rows without a finite threshold re-rank every column.
struct FixupArgs {
    const float *D;          // reduced keys, row stride ldd: row f holds listed row rows[f], or
    int64_t ldd;             // with by_row, row i holds row id i (a materialised block)
    bool by_row;
    const int32_t *rows;     // nrows row ids within the block
    int64_t nrows;
    const float *tfix;       // thresholds by row id
    const float *Q;          // block queries, row-major (row id i at Q + i d)
    const float *C;          // corpus n x d
    int64_t n;
    int d, k;
    int64_t self_offset;     // >= 0: row i's own corpus index self_offset + i is excluded
    float *out_dist;         // block outputs, row id i at out + i k
    int32_t *out_idx;
    float out_scale = 1.0f;  // as RerankArgs::out_scale
};
hipError_t launch_fixup(const FixupArgs &a, hipStream_t stream);

// Unit vectors for the cosine (centre = false) and Pearson (centre = true)
// distances: each row of X minus its mean (Pearson), divided by its Euclidean
// norm, into out (n x d FP32).  A row without a direction (zero or non-finite
// norm after centring; a constant row for Pearson) becomes all NaN.
hipError_t launch_unit_rows(const float *X, int64_t n, int d, bool centre, float *out, hipStream_t stream);

}  // namespace knn
