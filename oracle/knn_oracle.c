/*
 * CPU oracle for brute-force k-NN / k-NNG by per-row selection of the k smallest
 * entries (Komarov, Dashti & D'Souza, "Fast k-NNG construction with GPU-based
 * quick multi-select", arXiv:1309.5478).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP path.
 *
 * What it computes is the plain definition the paper's method reaches exactly:
 *
 *  - Selection (Introduction, brute-force description: sort each row of the
 *    M x N distance matrix and keep the indices of the k smallest).  Quickselect
 *    is exact, so the oracle is the definition itself: a full stable sort of each
 *    row followed by taking the first k.  Stability resolves equal values to the
 *    lower column index.  Values are ordered by a total order on FP32: -0 and +0
 *    are equal, all NaNs are equal to each other and above +inf, otherwise IEEE
 *    order.  Selected values are copied verbatim (bit for bit) from the input.
 *
 *  - Cosine and Pearson distances (Methods, "Distance calculation": cosine
 *    similarity of two vectors, and Pearson correlation as the cosine similarity
 *    of the vectors minus their means), as the distance 1 - similarity, in FP64
 *    from the FP32 inputs; a vector of zero norm (after centring) has no
 *    direction, and its distances are NaN.
 *
 *  - k-NN / k-NNG distances (Methods, "Distance calculation": squared Euclidean
 *    distance is what the neighbour comparison uses).  The oracle evaluates the
 *    direct difference form sum_t (q_t - c_t)^2 in FP64 from FP32 inputs (exactly
 *    converted), not the norm expansion, which cancels.  For the k-NNG the query
 *    set is the corpus and only the query's own index is excluded; duplicates at
 *    distance 0 remain neighbours.  Rows are stable-sorted by distance (ties to the
 *    lower corpus index) and the first k are returned.
 *
 * Built with -ffp-contract=off so every FP64 operation rounds on its own.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---- total order on FP32 values ---------------------------------------- */
static int f32_total_cmp(float a, float b) {
    int an = isnan(a) ? 1 : 0, bn = isnan(b) ? 1 : 0;
    if (an || bn) return an - bn;          /* NaN above everything, NaN == NaN */
    if (a < b) return -1;                  /* IEEE: -0 == +0 */
    if (a > b) return 1;
    return 0;
}

static int f64_total_cmp(double a, double b) {
    int an = isnan(a) ? 1 : 0, bn = isnan(b) ? 1 : 0;
    if (an || bn) return an - bn;
    if (a < b) return -1;
    if (a > b) return 1;
    return 0;
}

/* ---- stable bottom-up merge sort of an index array by a key array ------ */
typedef struct {
    const float *f32;  /* exactly one of these is set */
    const double *f64;
} keys_t;

static int key_cmp(const keys_t *k, int32_t a, int32_t b) {
    return k->f32 ? f32_total_cmp(k->f32[a], k->f32[b]) : f64_total_cmp(k->f64[a], k->f64[b]);
}

/* Sorts idx[0..n) so that keys are non-decreasing; equal keys keep their input
 * order (stability), which with idx initialised to 0..n-1 puts the lower index first. */
static void stable_sort_idx(int32_t *idx, int32_t *tmp, int64_t n, const keys_t *keys) {
    int32_t *src = idx, *dst = tmp;
    for (int64_t width = 1; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            int64_t mid = lo + width < n ? lo + width : n;
            int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int64_t i = lo, j = mid, o = lo;
            while (i < mid && j < hi) {
                /* take from the right run only if strictly smaller: stability */
                if (key_cmp(keys, src[j], src[i]) < 0) dst[o++] = src[j++];
                else dst[o++] = src[i++];
            }
            while (i < mid) dst[o++] = src[i++];
            while (j < hi) dst[o++] = src[j++];
        }
        int32_t *t = src; src = dst; dst = t;
    }
    if (src != idx) memcpy(idx, src, (size_t)n * sizeof(int32_t));
}

static int resolve_threads(int32_t nthreads) {
    if (nthreads > 0) return nthreads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* ---- selection ------------------------------------------------------------ */
typedef struct {
    const float *D; int64_t cols, ld; int32_t k;
    const int64_t *row_ids; int64_t nrows;
    float *out_val; int32_t *out_idx;
    int tid, nthreads; int status;
} sel_job_t;

static void *sel_worker(void *arg) {
    sel_job_t *j = (sel_job_t *)arg;
    int32_t *idx = (int32_t *)malloc((size_t)j->cols * sizeof(int32_t));
    int32_t *tmp = (int32_t *)malloc((size_t)j->cols * sizeof(int32_t));
    if (!idx || !tmp) { j->status = 2; free(idx); free(tmp); return NULL; }
    for (int64_t p = j->tid; p < j->nrows; p += j->nthreads) {
        int64_t r = j->row_ids ? j->row_ids[p] : p;
        const float *row = j->D + r * j->ld;
        for (int64_t c = 0; c < j->cols; ++c) idx[c] = (int32_t)c;
        keys_t keys = {row, NULL};
        stable_sort_idx(idx, tmp, j->cols, &keys);
        for (int32_t t = 0; t < j->k; ++t) {
            j->out_idx[p * j->k + t] = idx[t];
            memcpy(&j->out_val[p * j->k + t], &row[idx[t]], sizeof(float)); /* verbatim bits */
        }
    }
    free(idx); free(tmp);
    return NULL;
}

/* For each listed row r of the row-major matrix D (row stride ld), the k entries
 * that come first in a stable sort by the FP32 total order.  row_ids == NULL means
 * rows 0..nrows-1.  Outputs are nrows x k, row p holding row row_ids[p].
 * Returns 0 on success, 1 on invalid arguments, 2 on allocation failure. */
int oracle_select_k(const float *D, int64_t nrows, const int64_t *row_ids, int64_t cols,
                    int64_t ld, int32_t k, float *out_val, int32_t *out_idx, int32_t nthreads) {
    if (!D || !out_val || !out_idx || cols < 1 || ld < cols || k < 1 || k > cols || nrows < 0 ||
        cols > INT32_MAX)
        return 1;
    int nt = resolve_threads(nthreads);
    if (nt > nrows) nt = nrows > 0 ? (int)nrows : 1;
    pthread_t th[256]; sel_job_t jobs[256];
    if (nt > 256) nt = 256;
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (sel_job_t){D, cols, ld, k, row_ids, nrows, out_val, out_idx, t, nt, 0};
        pthread_create(&th[t], NULL, sel_worker, &jobs[t]);
    }
    int status = 0;
    for (int t = 0; t < nt; ++t) { pthread_join(th[t], NULL); if (jobs[t].status) status = jobs[t].status; }
    return status;
}

/* ---- k-NN with FP64 direct distances ------------------------------------- */
typedef struct {
    const float *Q; int64_t m; const float *C; int64_t n; int32_t d; int32_t kout;
    const int64_t *self_ids;
    double *out_dist; int32_t *out_idx;
    int tid, nthreads; int status;
    int32_t metric;                  /* 0 squared Euclidean, 1 cosine, 2 Pearson */
    const double *cmean, *cnorm;     /* per corpus vector (metrics 1 and 2) */
} knn_job_t;

/* Mean (Pearson only; 0 otherwise) and Euclidean norm of the centred vector, FP64. */
static void centre_norm(const float *x, int32_t d, int32_t metric, double *mean, double *norm) {
    double mu = 0.0;
    if (metric == 2) {
        for (int32_t t = 0; t < d; ++t) mu += (double)x[t];
        mu /= (double)d;
    }
    double s = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        double v = (double)x[t] - mu;
        s += v * v;
    }
    *mean = mu;
    *norm = sqrt(s);
}

/* Distance between query q and corpus vector y under the job's metric. */
static double pair_distance(const knn_job_t *j, const float *q, double qmean, double qnorm, int64_t c) {
    const float *y = j->C + c * (int64_t)j->d;
    if (j->metric == 0) {
        double s = 0.0;
        for (int32_t t = 0; t < j->d; ++t) {
            double diff = (double)q[t] - (double)y[t];
            s += diff * diff;
        }
        return s;
    }
    /* cosine distance 1 - x.y / (|x| |y|) of the (centred) vectors; undefined
     * (NaN) when either has zero norm */
    const double ym = j->cmean[c], yn = j->cnorm[c];
    if (qnorm == 0.0 || yn == 0.0) return NAN;
    double dot = 0.0;
    for (int32_t t = 0; t < j->d; ++t) dot += ((double)q[t] - qmean) * ((double)y[t] - ym);
    return 1.0 - dot / (qnorm * yn);
}

static void *knn_worker(void *arg) {
    knn_job_t *j = (knn_job_t *)arg;
    double *dist = (double *)malloc((size_t)j->n * sizeof(double));
    int32_t *idx = (int32_t *)malloc((size_t)j->n * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc((size_t)j->n * sizeof(int32_t));
    int32_t *scratch = (int32_t *)malloc((size_t)j->n * sizeof(int32_t));
    if (!dist || !idx || !order || !scratch) {
        j->status = 2; free(dist); free(idx); free(order); free(scratch); return NULL;
    }
    for (int64_t i = j->tid; i < j->m; i += j->nthreads) {
        const float *q = j->Q + i * (int64_t)j->d;
        int64_t self = j->self_ids ? j->self_ids[i] : -1;
        int64_t cnt = 0;
        double qmean = 0.0, qnorm = 0.0;
        if (j->metric != 0) centre_norm(q, j->d, j->metric, &qmean, &qnorm);
        for (int64_t c = 0; c < j->n; ++c) {
            if (c == self) continue;           /* k-NNG: exclude only the query itself */
            dist[cnt] = pair_distance(j, q, qmean, qnorm, c);
            idx[cnt] = (int32_t)c;
            ++cnt;
        }
        /* positions are in increasing corpus-index order, so the stable sort breaks
         * distance ties toward the lower corpus index */
        for (int64_t c = 0; c < cnt; ++c) order[c] = (int32_t)c;
        keys_t keys = {NULL, dist};
        stable_sort_idx(order, scratch, cnt, &keys);
        for (int32_t t = 0; t < j->kout; ++t) {
            if (t < cnt) {
                j->out_dist[i * j->kout + t] = dist[order[t]];
                j->out_idx[i * j->kout + t] = idx[order[t]];
            } else {
                j->out_dist[i * j->kout + t] = INFINITY;
                j->out_idx[i * j->kout + t] = -1;
            }
        }
    }
    free(dist); free(idx); free(order); free(scratch);
    return NULL;
}

/* The kout nearest corpus points (rows of C, n x d) to each query (rows of Q,
 * m x d), by FP64 squared Euclidean distance in direct form; ties to the lower
 * corpus index.  self_ids == NULL: no exclusion; otherwise corpus index
 * self_ids[i] is excluded for query i (k-NNG).  Positions beyond the number of
 * eligible corpus points are filled with (+inf, -1).
 * Returns 0 on success, 1 on invalid arguments, 2 on allocation failure. */
int oracle_knn_metric(const float *Q, int64_t m, const float *C, int64_t n, int32_t d, int32_t kout,
                      const int64_t *self_ids, double *out_dist, int32_t *out_idx, int32_t nthreads,
                      int32_t metric) {
    if (!Q || !C || !out_dist || !out_idx || m < 0 || n < 1 || d < 1 || kout < 1 || n > INT32_MAX ||
        metric < 0 || metric > 2)
        return 1;
    double *cmean = NULL, *cnorm = NULL;
    if (metric != 0) {
        cmean = (double *)malloc((size_t)n * sizeof(double));
        cnorm = (double *)malloc((size_t)n * sizeof(double));
        if (!cmean || !cnorm) { free(cmean); free(cnorm); return 2; }
        for (int64_t c = 0; c < n; ++c) centre_norm(C + c * (int64_t)d, d, metric, &cmean[c], &cnorm[c]);
    }
    int nt = resolve_threads(nthreads);
    if (nt > m) nt = m > 0 ? (int)m : 1;
    if (nt > 256) nt = 256;
    pthread_t th[256]; knn_job_t jobs[256];
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (knn_job_t){Q, m, C, n, d, kout, self_ids, out_dist, out_idx, t, nt, 0, metric, cmean, cnorm};
        pthread_create(&th[t], NULL, knn_worker, &jobs[t]);
    }
    int status = 0;
    for (int t = 0; t < nt; ++t) { pthread_join(th[t], NULL); if (jobs[t].status) status = jobs[t].status; }
    free(cmean); free(cnorm);
    return status;
}

/* Squared Euclidean k-NN (metric 0 of oracle_knn_metric). */
int oracle_knn(const float *Q, int64_t m, const float *C, int64_t n, int32_t d, int32_t kout,
               const int64_t *self_ids, double *out_dist, int32_t *out_idx, int32_t nthreads) {
    return oracle_knn_metric(Q, m, C, n, d, kout, self_ids, out_dist, out_idx, nthreads, 0);
}

/* Number of worker threads a call with nthreads <= 0 uses. */
int oracle_default_threads(void) { return resolve_threads(0); }
