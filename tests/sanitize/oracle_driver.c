/* Drives every entry point of the C oracle (oracle/knn_oracle.c) on small
 * seeded inputs, including the edge
 * cases (k = 1, k = n, NaN and signed-zero values, rows shorter than k,
 * zero-norm vectors for the cosine and Pearson distances, one and many
 * threads), so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py) checks the oracle's memory accesses and
 * arithmetic for undefined behaviour.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_select_k(const float *D, int64_t nrows, const int64_t *row_ids, int64_t cols, int64_t ld, int32_t k,
                    float *out_val, int32_t *out_idx, int32_t nthreads);
int oracle_knn_metric(const float *Q, int64_t m, const float *C, int64_t n, int32_t d, int32_t kout,
                      const int64_t *self_ids, double *out_dist, int32_t *out_idx, int32_t nthreads, int32_t metric);
int oracle_knn(const float *Q, int64_t m, const float *C, int64_t n, int32_t d, int32_t kout,
               const int64_t *self_ids, double *out_dist, int32_t *out_idx, int32_t nthreads);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static float next_uniform(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (float)((state >> 40) * (1.0 / 16777216.0));
}

static int check(int st, const char *what) {
    if (st != 0) {
        fprintf(stderr, "%s returned %d\n", what, st);
        return 1;
    }
    return 0;
}

int main(void) {
    int bad = 0;
    /* selection: ragged sizes, every k, special values, one and several threads */
    for (int cols = 1; cols <= 70; cols += 23) {
        const int rows = 7;
        float *D = malloc(sizeof(float) * rows * cols);
        for (int i = 0; i < rows * cols; ++i) D[i] = floorf(next_uniform() * 5.0f);
        if (cols > 3) {
            D[0] = NAN;
            D[1] = -0.0f;
            D[2] = INFINITY;
            D[3] = -INFINITY;
        }
        int64_t ids[3] = {0, rows - 1, 2};
        for (int k = 1; k <= cols; k += (cols > 10 ? 9 : 1)) {
            float *v = malloc(sizeof(float) * rows * k);
            int32_t *ix = malloc(sizeof(int32_t) * rows * k);
            for (int nt = 1; nt <= 3; nt += 2) {
                bad |= check(oracle_select_k(D, rows, NULL, cols, cols, k, v, ix, nt), "oracle_select_k");
                bad |= check(oracle_select_k(D, 3, ids, cols, cols, k, v, ix, nt), "oracle_select_k rows");
            }
            free(v);
            free(ix);
        }
        free(D);
    }
    /* k-NN: every metric, self exclusion, kout beyond the eligible points, zero vectors */
    for (int metric = 0; metric <= 2; ++metric) {
        const int n = 40, m = 9, d = 5;
        float *C = malloc(sizeof(float) * n * d), *Q = malloc(sizeof(float) * m * d);
        for (int i = 0; i < n * d; ++i) C[i] = next_uniform();
        for (int i = 0; i < m * d; ++i) Q[i] = next_uniform();
        for (int t = 0; t < d; ++t) {
            C[3 * d + t] = 0.0f;   /* zero vector */
            C[4 * d + t] = 2.0f;   /* constant vector */
            Q[1 * d + t] = 0.0f;
        }
        int64_t self[9];
        for (int i = 0; i < m; ++i) self[i] = i;
        for (int kout = 1; kout <= n + 2; kout += 7) {
            double *od = malloc(sizeof(double) * m * kout);
            int32_t *oi = malloc(sizeof(int32_t) * m * kout);
            for (int nt = 1; nt <= 4; nt += 3) {
                bad |= check(oracle_knn_metric(Q, m, C, n, d, kout, NULL, od, oi, nt, metric), "oracle_knn_metric");
                bad |= check(oracle_knn_metric(C, m, C, n, d, kout, self, od, oi, nt, metric), "oracle_knn_metric self");
            }
            if (metric == 0) bad |= check(oracle_knn(Q, m, C, n, d, kout, NULL, od, oi, 2), "oracle_knn");
            free(od);
            free(oi);
        }
        free(C);
        free(Q);
    }
    /* argument errors are reported, not acted on */
    if (oracle_select_k(NULL, 1, NULL, 1, 1, 1, NULL, NULL, 1) == 0) bad = 1;
    if (oracle_knn_metric(NULL, 1, NULL, 1, 1, 1, NULL, NULL, NULL, 1, 0) == 0) bad = 1;
    if (bad) return 1;
    puts("oracle sanitizer driver: ok");
    return 0;
}
