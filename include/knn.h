/*
 * knn.h -- C ABI of libknn.so: brute-force k-NN / k-NN graph construction by
 * GPU quick multi-select on AMD Instinct MI355X (gfx950).
 *
 * Method: Komarov, Dashti & D'Souza, "Fast k-NNG construction with GPU-based
 * quick multi-select" (arXiv:1309.5478).  The distance part is a matrix product
 * plus norm corrections (Methods, "Distance calculation"); the selection part
 * is the paper's two-level quick multi-select (Methods, "GPU-based quick
 * multi-select").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller (for example
 *    the storage of a torch tensor on ROCm).  The library never frees, retains
 *    or writes through an input pointer; inputs are const.  Outputs are written
 *    only when the call returns KNN_SUCCESS.
 *  - Layout is row-major.  Point sets are n x d with row stride d floats.  A
 *    distance matrix has row stride `ld` >= cols floats.  Outputs are rows x k,
 *    contiguous.
 *  - Each output row is in ascending order of (value, index): the selected set
 *    and its order are those of a stable sort of the row, so equal values
 *    resolve to the lower column index.  FP32 values are ordered by a total
 *    order: -0 == +0, all NaNs equal and above +inf.
 *  - Indices are int32; any count of columns / corpus points above INT32_MAX is
 *    rejected.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously on it.  Arguments are validated on the host before anything
 *    is enqueued; on an error nothing is launched and the outputs are untouched.
 *  - A handle owns a device workspace that grows on demand and is reused by
 *    later calls.  Calls on one handle must be issued from one host thread at a
 *    time and ordered on one stream (or otherwise ordered by the caller).
 *  - Device-side faults surface as KNN_ERROR_DEVICE from the failing launch or
 *    from knn_get_stats, which synchronises the stream.
 */
#ifndef KNN_H_
#define KNN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct knn_handle_s *knn_handle_t;

typedef enum {
    KNN_SUCCESS = 0,
    KNN_ERROR_INVALID_VALUE = 1, /* bad pointer, size, k, stride or option      */
    KNN_ERROR_OUT_OF_MEMORY = 2, /* workspace allocation failed                 */
    KNN_ERROR_UNSUPPORTED = 3,   /* device is not gfx950, or a size limit is hit */
    KNN_ERROR_DEVICE = 4,        /* a HIP runtime call or a kernel failed        */
    KNN_ERROR_IO = 5             /* a file could not be read or written          */
} knn_status_t;

/* How the first pivot of each row is chosen.  The output never depends on it. */
typedef enum {
    /* lower median of a strided sample of the segment, at every pass: the
     * paper's quickselect with the pivot rule it leaves open */
    KNN_PIVOT_PLAIN = 0,
    /* the sample order statistic just above the expected rank of the k-th key */
    KNN_PIVOT_SAMPLE = 1,
    /* the pivot network's estimate of the k-th value; rows where it is unusable
     * fall back to KNN_PIVOT_SAMPLE */
    KNN_PIVOT_LEARNED = 2
} knn_pivot_t;

/* Operand precision of the distance product in knn_search / knn_graph.  The
 * candidates it ranks are always re-ranked with exact FP32 distances. */
typedef enum {
    KNN_PREC_FP32 = 0,      /* FP32 inputs on the FP32 matrix cores                */
    KNN_PREC_BF16 = 1,      /* BF16 (round to nearest even) inputs, FP32 accumulation */
    KNN_PREC_FP8_E4M3 = 2   /* OCP e4m3 (round to nearest even, saturating) after a   */
                            /* per-point power-of-two scale 2^e, e the largest with   */
                            /* max|x| 2^e <= 448; FP32 accumulation, scales undone    */
                            /* exactly in the epilogue                                */
} knn_precision_t;

/* Distance of knn_search / knn_graph / knn_batch_search (Methods, "Distance
 * calculation": Euclidean distance, cosine similarity, and Pearson's
 * correlation as the cosine similarity of the mean-centred vectors). */
typedef enum {
    KNN_METRIC_SQEUCLIDEAN = 0, /* |x - y|^2                                             */
    KNN_METRIC_COSINE = 1,      /* 1 - x.y / (|x| |y|)                                   */
    KNN_METRIC_PEARSON = 2      /* 1 - r(x, y): the cosine distance of x - mean(x) and   */
                                /* y - mean(y)                                           */
    /* Cosine and Pearson run the Euclidean path on unit vectors u = x / |x|
     * (centred first for Pearson) and return |u - v|^2 / 2, which equals
     * 1 - similarity and has no cancellation near 0.  A vector without a
     * direction (zero norm after centring, a constant vector for Pearson, or a
     * non-finite element) has NaN distances, which sort after every number. */
} knn_metric_t;

typedef struct {
    int32_t pivot;      /* knn_pivot_t; default KNN_PIVOT_SAMPLE                      */
    int32_t precision;  /* knn_precision_t; default KNN_PREC_FP32 (search / graph)    */
    int32_t oversample; /* candidates kept before the exact re-rank = oversample * k; */
                        /* default 4, at least 1                                      */
    int32_t flags;      /* KNN_FLAG_* bits                                            */
    int32_t metric;     /* knn_metric_t; default KNN_METRIC_SQEUCLIDEAN               */
} knn_options_t;

/* Force the exact-fallback path of search / graph for every row that takes
 * the filtering path, i.e. every row of a corpus larger than its threshold
 * sample (tests). */
#define KNN_FLAG_FORCE_FALLBACK 0x1
/* Materialise distance tiles and select from them instead of the fused kernel. */
#define KNN_FLAG_UNFUSED 0x2
/* Time every launch of the distance product with HIP events on the call's
 * stream and report it in knn_stats_t (product_ms, product_launches). */
#define KNN_FLAG_TIMING 0x4
/* knn_batch_search: run every step eagerly instead of capturing and replaying
 * HIP graphs. */
#define KNN_FLAG_NO_GRAPH 0x8
/* Choose the tile shape of the distance product by timing the candidate shapes
 * on the call's own operands the first time a shape class is seen (cached per
 * handle, and in the JSON file named by KNN_AUTOTUNE_CACHE when that is set).
 * Also enabled by the environment variable KNN_AUTOTUNE=1. */
#define KNN_FLAG_AUTOTUNE 0x10
/* search / graph / batch with FP32 products: treat every row as uncertified, so
 * that each row is re-run exactly from its materialised reduced-key row (tests). */
#define KNN_FLAG_FORCE_RERUN 0x20
/* knn_select_k: never split rows across workgroups (see knn_select_k). */
#define KNN_FLAG_NO_SPLIT 0x40
/* knn_select_k: split every row that is at least two minimal parts of
 * max(4096, 32 k) columns long, whatever the row count (tests). */
#define KNN_FLAG_FORCE_SPLIT 0x80

typedef struct {
    int64_t rows;                 /* rows processed by the last call; with        */
                                  /* split_parts > 1 the counters below sum (and  */
                                  /* passes_max maximises) over the parts         */
    int64_t passes_total;         /* partition passes summed over rows            */
    int32_t passes_max;           /* most partition passes on one row             */
    int32_t split_parts;          /* select_k: parts each row was cut into (1:    */
                                  /* whole rows, one workgroup each)              */
    int64_t stream_passes_total;  /* full reads of an input row (select_k)        */
    int64_t spill_rows;           /* rows whose candidates left on-chip memory    */
    int64_t first_pass_survivors; /* keys kept by the first pass, summed          */
    int64_t fallback_rows;        /* search / graph rows re-run on the exact path */
    int64_t candidates_total;     /* search / graph candidates, summed            */
    int64_t phase_cycles[4];      /* shader clocks summed over rows: first pivot, */
                                  /* streaming passes, on-chip passes, final sort */
    double product_ms;            /* KNN_FLAG_TIMING: summed duration of the main  */
    int64_t product_launches;     /* distance-product launches (fused or dense),   */
    double product_flops;         /* their count, and their algorithmic flops      */
                                  /* (2 * rows * cols * d each)                    */
    int64_t rows_uncertified;     /* search / graph rows whose candidate margin    */
                                  /* does not exceed twice the key error bound     */
    int64_t rows_rerun;           /* FP32 rows among them re-run exactly: every    */
                                  /* point whose reduced key is within the bound   */
                                  /* of the k-th candidate re-ranked by its exact  */
                                  /* distance                                      */
} knn_stats_t;

/* Create a handle bound to HIP device `device` (must be gfx950). */
knn_status_t knn_create(knn_handle_t *out, int device);
/* Release a handle and its workspace.  NULL is accepted. */
knn_status_t knn_destroy(knn_handle_t h);
/* Static description of a status code. */
const char *knn_status_string(knn_status_t s);
/* Detail string for the last failing call on `h` (or on no handle, if NULL). */
const char *knn_last_error(knn_handle_t h);

/*
 * knn_select_k -- the k smallest entries of every row of a distance matrix
 * (Introduction: brute-force selection from each row of the M x N matrix;
 * Methods, "GPU-based quick multi-select": two-level quickselect, one workgroup
 * per row, ballot-based partition, K-versus-L recursion with a stack of segment
 * references).
 *
 * Few long rows: the paper's GPU is only saturated with enough rows in flight
 * (Results, Figure 8; Discussion).  When the rows are too few to give every
 * resident workgroup one, each row is cut into parts of at least
 * max(65536, 32 k) columns (a power of two of them; max(4096, 32 k) when
 * forced), every part's k smallest keys are selected by its own workgroup, and
 * the parts' lists are merged by key-list selections; the result is the same,
 * bit for bit.  The flags KNN_FLAG_NO_SPLIT / KNN_FLAG_FORCE_SPLIT turn this
 * off / force it.
 *
 *   dist     rows x cols FP32, row stride ld (>= cols)            [in, device]
 *   k        1 <= k <= min(cols, 1024)
 *   out_val  rows x k FP32: the selected entries, bit-for-bit copies [out]
 *   out_idx  rows x k int32: their column indices, or NULL for values only
 *            (Results: the selection measured on values alone)     [out]
 *   opt      NULL for defaults; `pivot` and the split flags are used
 * Errors: INVALID_VALUE for null dist / out_val, rows < 0, cols < 1, ld < cols,
 * k < 1, k > cols, or both split flags; UNSUPPORTED for k > 1024 or
 * cols > INT32_MAX.
 */
knn_status_t knn_select_k(knn_handle_t h, const float *dist, int64_t rows, int64_t cols,
                          int64_t ld, int32_t k, float *out_val, int32_t *out_idx,
                          void *stream, const knn_options_t *opt);

/*
 * knn_select_k_noalloc -- knn_select_k for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, checks and results as knn_select_k
 * (values only with out_idx NULL), but it allocates nothing: its workspace is
 * a static 64 MiB device array that the library holds on every device it runs
 * on until the process ends.  Rows are never split across workgroups; rows
 * longer than 8192 columns run with fewer workgroups at once so that their
 * overflow buffers (2 (cols - 1024) keys of 8 bytes per workgroup) fit the
 * array.  Every call on one device shares that device's array: calls that
 * overlap in time on one device (on different streams, or from different
 * handles or threads) race and give undefined results; order them.
 * Errors: as knn_select_k, plus UNSUPPORTED for cols above 4195312 (one
 * workgroup's overflow buffers would not fit) or a device ordinal >= 64.
 */
knn_status_t knn_select_k_noalloc(knn_handle_t h, const float *dist, int64_t rows, int64_t cols,
                                  int64_t ld, int32_t k, float *out_val, int32_t *out_idx,
                                  void *stream, const knn_options_t *opt);

/*
 * knn_partition -- one partition pass per row, as the paper describes it for one
 * warp per row (Methods, "GPU-based quick multi-select", and Figures 1-3): the
 * row is read in 64-element segments, a wavefront ballot on "key below pivot"
 * gives every lane its slot through a population count of the lanes below it,
 * keys below the pivot are written from the left end of the output row in input
 * order and the others from the right end (so they appear in reverse input
 * order).  Keys are (value, column index) under the total order above.
 *
 *   in        rows x cols FP32, row stride ld                       [in, device]
 *   piv_val   rows FP32 pivot values                                [in, device]
 *   piv_idx   rows int32 pivot column indices (ties of value: a key is below
 *             the pivot when its index is lower)                     [in, device]
 *   out_val   rows x cols FP32 partitioned values                    [out]
 *   out_idx   rows x cols int32 their column indices                 [out]
 *   out_left  rows int32: L, the number of keys below the pivot      [out]
 * Errors: INVALID_VALUE for null pointers, rows < 0, cols < 1, ld < cols.
 */
knn_status_t knn_partition(knn_handle_t h, const float *in, int64_t rows, int64_t cols,
                           int64_t ld, const float *piv_val, const int32_t *piv_idx,
                           float *out_val, int32_t *out_idx, int32_t *out_left, void *stream);

/*
 * knn_search -- for each of m queries, its k nearest corpus points by squared
 * Euclidean distance (Methods, "Distance calculation": squared distance
 * ||x||^2 + ||y||^2 - 2 x.y, ranked on ||y||^2 - 2 x.y since ||x||^2 is common
 * to a row).  Candidates (oversample * k per row) are ranked on that reduced
 * key from the matrix-core product, then re-ranked by the exact FP32 direct
 * form sum_t (q_t - c_t)^2, which is what out_dist returns.
 *
 *   queries   m x d FP32                                           [in, device]
 *   corpus    n x d FP32                                           [in, device]
 *   k         1 <= k <= min(n, 1024)
 *   out_dist  m x k FP32 squared distances (cosine / Pearson: 1 - similarity,
 *             see knn_metric_t)                                     [out]
 *   out_idx   m x k int32 corpus indices                            [out]
 * Errors: INVALID_VALUE for null pointers, m < 0, n < 1, d < 1, k < 1, k > n,
 * a bad option; UNSUPPORTED for k > 1024 or n > INT32_MAX.  With a cosine or
 * Pearson metric the handle keeps a second buffer of (m + n) d floats (n d for
 * knn_graph) for the unit vectors.
 */
knn_status_t knn_search(knn_handle_t h, const float *queries, int64_t m, const float *corpus,
                        int64_t n, int32_t d, int32_t k, float *out_dist, int32_t *out_idx,
                        void *stream, const knn_options_t *opt);

/*
 * knn_search_host_corpus -- knn_search with the corpus in host memory, for
 * corpora beyond (or not resident in) device memory.  The paper names the
 * device memory as the limit of its method and partitioning of the data as the
 * way past it (Discussion).  The corpus is copied to the device in partitions
 * of part_rows points, two partition buffers deep: the copy of partition p + 1
 * runs on a copy stream of the handle while partition p is searched on
 * `stream`, and each partition's k nearest per query are merged into the
 * running k nearest by (distance, global index).  The result is knn_search's on
 * the whole corpus, bit for bit, whenever knn_search's rows are exact (FP32
 * products: always); options as knn_search.
 *   queries      m x d FP32                                        [in, device]
 *   corpus_host  n x d FP32 in host memory; copies overlap the search only
 *                when it is pinned (hipHostMalloc); it must stay valid until
 *                the work enqueued on `stream` has completed           [in, host]
 *   part_rows    points per partition (0: about 1 GiB of points, at least k)
 *   out_dist, out_idx  m x k, as knn_search                        [out, device]
 * The handle keeps two partition buffers and three m x k result buffers.
 * Errors: as knn_search, plus INVALID_VALUE for part_rows < 0.
 */
knn_status_t knn_search_host_corpus(knn_handle_t h, const float *queries, int64_t m, const float *corpus_host,
                                    int64_t n, int32_t d, int32_t k, int64_t part_rows, float *out_dist,
                                    int32_t *out_idx, void *stream, const knn_options_t *opt);

/*
 * knn_graph -- the k-NN graph of n points (Introduction: every corpus point is
 * also a query).  Same as knn_search(points, n, points, n, ...) except that each
 * point's own index is excluded; duplicates at distance 0 remain neighbours.
 *   points    n x d FP32                                           [in, device]
 *   k         1 <= k <= min(n - 1, 1024)
 * Errors: as knn_search, with k > n - 1 rejected.
 */
knn_status_t knn_graph(knn_handle_t h, const float *points, int64_t n, int32_t d, int32_t k,
                       float *out_dist, int32_t *out_idx, void *stream,
                       const knn_options_t *opt);

/*
 * One job of knn_batch_search: the k nearest corpus points of each query, or,
 * with queries == NULL, the k-NN graph of the corpus (m must equal n; each
 * point's own index excluded).  All pointers are device pointers owned by the
 * caller; rows are dense (stride d).
 */
typedef struct {
    const float *queries;   /* m x d FP32, or NULL for the k-NN graph of corpus;     */
                            /* unused when m == 0                                    */
    int64_t m;              /* query count (>= 0)                                    */
    const float *corpus;    /* n x d FP32                                            */
    int64_t n;              /* corpus size (>= 1; >= 2 for a graph job)              */
    int32_t d;              /* dimension (>= 1)                                      */
    int32_t k;              /* 1 <= k <= 1024; k may exceed the corpus (less the own */
                            /* point for a graph job): the missing entries of a row  */
                            /* are +inf with index -1                                */
    float *out_dist;        /* m x k FP32 exact squared distances           [out]    */
    int32_t *out_idx;       /* m x k int32 corpus indices                   [out]    */
} knn_job_t;

/*
 * knn_batch_search -- many independent k-NN problems of uneven sizes in one
 * call (Introduction and Discussion: many simultaneous queries, each a row
 * selection, are the coarse level of parallelism; here whole problems of
 * different corpus sizes, dimensions and k are pooled the same way).  Each job
 * computes exactly what knn_search (or knn_graph) computes for it, with the same
 * output bits.  The distance products of all jobs run in one launch of
 * (job, tile) items, one per workgroup, ordered longest job first for the
 * round-robin dispatch of workgroups over the XCDs; the per-job threshold,
 * flagging, selection and re-rank steps are captured into
 * HIP graphs on the first call and replayed by later calls with the same job
 * table, options and handle state (KNN_FLAG_NO_GRAPH runs them eagerly).
 *
 *   jobs     njobs job descriptions (host array, read during the call)     [in]
 *   njobs    >= 0
 *   stream   HIP stream of the call; the call returns after the last step is
 *            enqueued, once the rows needing the exact fallback are known
 *            (one host synchronisation, as knn_search)
 *   opt      NULL for defaults; pivot, precision, oversample and the flags
 *            FORCE_FALLBACK, UNFUSED (jobs run one by one as knn_search),
 *            TIMING, NO_GRAPH and AUTOTUNE are honoured
 * Errors: INVALID_VALUE for a null jobs array with njobs > 0, njobs < 0, a job
 * with a null pointer, m < 0, n < 1, d < 1, k < 1, a graph job (null queries,
 * m > 0) with m != n or n < 2, or a bad option; UNSUPPORTED for k > 1024 or n > INT32_MAX; the
 * message names the first offending job.  OUT_OF_MEMORY when the batch's
 * workspace (kept by the handle for replays) cannot be allocated.
 */
knn_status_t knn_batch_search(knn_handle_t h, const knn_job_t *jobs, int32_t njobs, void *stream,
                              const knn_options_t *opt);

/*
 * knn_distances -- the m x n matrix of squared Euclidean distances between the
 * rows of `queries` and `corpus` by the norm expansion
 * ||q||^2 + ||c||^2 - 2 q.c (Methods, "Distance calculation": norms by a
 * reduction, dot products as one matrix product on the FP32 matrix cores).
 * Together with knn_select_k this is the paper's two-step pipeline with the
 * matrix stored.  Values carry the cancellation error of the expansion and can
 * be slightly negative for near-duplicate points.
 *
 *   queries  m x d FP32                                            [in, device]
 *   corpus   n x d FP32                                            [in, device]
 *   out      m x n FP32, row stride ldo (>= n)                     [out]
 * Errors: INVALID_VALUE for null pointers, m < 0, n < 1, d < 1, ldo < n;
 * UNSUPPORTED for n > INT32_MAX.
 */
knn_status_t knn_distances(knn_handle_t h, const float *queries, int64_t m, const float *corpus,
                           int64_t n, int32_t d, float *out, int64_t ldo, void *stream);

/*
 * knn_quantize -- the reduced-precision operands that knn_search / knn_graph
 * feed to the matrix cores for KNN_PREC_BF16 and KNN_PREC_FP8_E4M3 (the paper
 * computes in FP32; lower operand precision is this library's addition, with
 * every candidate re-ranked in FP32).  Exported so that the conversion can be
 * checked element by element.
 *   X      n x d FP32 points                                      [in, device]
 *   prec   KNN_PREC_BF16: BF16 codes (uint16), round to nearest even; a NaN
 *          stays a quiet NaN with its sign.
 *          KNN_PREC_FP8_E4M3: OCP e4m3 codes (uint8) of x * 2^e, where e is per
 *          point the largest integer with amax 2^e <= 448 (amax: the largest
 *          finite magnitude of the point; e = 0 without a finite non-zero
 *          element; e limited to [-100, 100]); round to nearest even,
 *          saturating at +-448 (infinities too); a NaN becomes the NaN code
 *          S.1111.111.
 *   out    n rows of ldo codes, ldo = d rounded up to a multiple of 128; the
 *          padding codes are zero                                  [out, device]
 *   scale  n FP32 scales 2^-e (FP8; NULL allowed for BF16)         [out, device]
 * Errors: INVALID_VALUE for null pointers, n < 0, d < 1 or another precision.
 */
knn_status_t knn_quantize(knn_handle_t h, const float *X, int64_t n, int32_t d, int32_t prec, void *out,
                          float *scale, void *stream);

/*
 * Pivot network (learned first pivot of the quick multi-select).
 *
 * The paper leaves the pivot rule of its method open (Methods, "GPU-based quick
 * multi-select": only the cited quicksort's random pivot is described).  This
 * network predicts, from statistics of a 256-entry strided sample of a row
 * (4 blocks of 64 contiguous entries), the standardised value of the row's
 * k-th smallest entry, y = (v_k - m) / s (m: sample lower median, s: sample
 * interquartile range / 1.349), so that the first partition pass keeps just
 * over k keys.  8 features -> 64 -> 64 -> 1, ReLU, BF16 weights with FP32
 * accumulation; trained with a pinball (quantile) loss by the kernels below.
 * Features, in order: log2(N)/16, log2(k)/10, and (v - m)/s for the sample
 * minimum, the sample entries at ranks r and r+1 with r = ceil(256 k / N) - 1,
 * the entry at rank 25 and the sample mean, then log(s / (|m| + s)).
 * Parameter layout (KNN_PIVOT_NPARAM floats): W1 (64 x 8, row-major), b1 (64),
 * W2 (64 x 64), b2 (64), w3 (64), b3.
 * When no network is loaded, KNN_PIVOT_LEARNED behaves as KNN_PIVOT_SAMPLE; an
 * unusable prediction (NaN, infinite) falls back to the sample rule per row.
 */
#define KNN_PIVOT_NPARAM 4801

/* FP32 master weights from a host array of KNN_PIVOT_NPARAM finite floats;
 * resets the optimiser state.  Synchronous. */
knn_status_t knn_pivot_set_weights(knn_handle_t h, const float *host_params, int32_t n);
/* FP32 master weights into a host array.  Synchronises the device. */
knn_status_t knn_pivot_get_weights(knn_handle_t h, float *host_params, int32_t n);
/* Writes / reads a weights file: "KNNPIV01", version, sizes, optimiser step,
 * training quantile, FP32 master weights.  IO on failure. */
knn_status_t knn_pivot_save(knn_handle_t h, const char *path);
knn_status_t knn_pivot_load(knn_handle_t h, const char *path);
/*
 * The 8 features of every row of a distance matrix for a given k.
 *   dist       rows x cols FP32, row stride ld, cols >= 256          [in, device]
 *   feats      rows x 8 FP32                                         [out, device]
 *   loc_scale  rows x 2 FP32 (m, s), or NULL                         [out, device]
 * Errors: INVALID_VALUE for bad sizes or null pointers; UNSUPPORTED for
 * cols < 256 or cols > INT32_MAX.
 */
knn_status_t knn_pivot_features(knn_handle_t h, const float *dist, int64_t rows, int64_t cols,
                                int64_t ld, int32_t k, float *feats, float *loc_scale, void *stream);
/* Standardised predictions y_hat (rows) for feature rows (rows x 8), with the
 * BF16 weights.  INVALID_VALUE if no network is loaded. */
knn_status_t knn_pivot_predict(knn_handle_t h, const float *feats, int64_t rows, float *y_hat,
                               void *stream);
/*
 * Mean pinball loss at `quantile` (0 < q < 1) of a batch and its gradient with
 * respect to the (BF16-rounded) weights, FP32, summed over the batch in order.
 *   feats (B x 8), targets (B), grad (KNN_PIVOT_NPARAM), loss (1)   [device]
 */
knn_status_t knn_pivot_grad(knn_handle_t h, const float *feats, const float *targets, int64_t B,
                            float quantile, float *grad, float *loss, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on the FP32
 * master weights with the gradient above; refreshes the BF16 copy.  loss may
 * be NULL. */
knn_status_t knn_pivot_train_step(knn_handle_t h, const float *feats, const float *targets,
                                  int64_t B, float quantile, float lr, float *loss, void *stream);

/*
 * Training the pivot network on rows the method itself generates.
 *
 * knn_pivot_add_examples appends one training example per row of a distance
 * matrix: the row's 8 features for `k` and the target y = (v_k - m) / s, the
 * row's exact k-th smallest value (by knn_select_k) standardised with the
 * sample location m and scale s the features use.  Rows whose features or
 * target are not finite are skipped; the kept rows are appended in row order.
 * The examples live on the device, owned by the handle, until
 * knn_pivot_clear_examples.  Synchronous (returns once they are stored).
 *   dist   rows x cols FP32, row stride ld, cols >= 256             [in, device]
 *   k      1 <= k <= min(cols, 1024)
 * Errors: INVALID_VALUE for bad sizes or a null pointer; UNSUPPORTED for
 * cols < 256, cols > INT32_MAX or k > 1024; OUT_OF_MEMORY.
 *
 * knn_pivot_train trains the network from scratch on the stored examples and,
 * when out_path is not NULL, writes it with knn_pivot_save.  Every step runs on
 * the device: weights drawn from `seed` (He initialisation: normal weights of
 * variance 2 / fan-in for the hidden layers and 1 / 64 for the output, zero
 * biases, the output bias at the lower median of a strided sample of at most
 * 2048 targets), then `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8) on
 * batches of min(4096, examples) drawn uniformly with replacement by a
 * counter-based generator of (seed, step), pinball loss at quantile 0.99,
 * learning rate 2e-3 decaying exponentially to 2e-4.  The result depends only
 * on the examples, the seed and the step count.  Synchronous.
 * Errors: INVALID_VALUE without examples or with steps < 0; IO if the file
 * cannot be written.
 */
knn_status_t knn_pivot_add_examples(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld,
                                    int32_t k, void *stream);
knn_status_t knn_pivot_clear_examples(knn_handle_t h);
knn_status_t knn_pivot_example_count(knn_handle_t h, int64_t *count);
/* Copies the stored examples (count x 8 features, count targets) into device
 * arrays of at least max_rows rows.  Synchronous. */
knn_status_t knn_pivot_get_examples(knn_handle_t h, float *feats, float *targets, int64_t max_rows);
knn_status_t knn_pivot_train(knn_handle_t h, const char *out_path, uint64_t seed, int32_t steps);

/* Counters of the last select / search / graph call on `h`.  Synchronises the
 * stream that call used. */
knn_status_t knn_get_stats(knn_handle_t h, knn_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* KNN_H_ */
