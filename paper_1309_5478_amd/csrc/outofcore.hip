// k-NN search over a corpus held in host memory (Discussion: the data and the
// distance matrix beyond the device's memory bound the method; partitioning the
// data is the remedy it proposes).  The corpus is streamed to the device in
// partitions, two buffers deep: the copy of the next partition (on a copy
// stream of the handle) overlaps the search of the current one, and each
// partition's k nearest per query are merged into the running k nearest by
// (distance, global index).  Because keys form a total order and the k nearest
// of the whole corpus lie among the union of every partition's k nearest, the
// result is the one knn_search gives on the whole corpus.
#include <hip/hip_runtime.h>

#include <string>

#include "handle.hpp"
#include "internal.hpp"
#include "keys.hpp"
#include "knn.h"

namespace knn {

knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg);
knn_status_t run_search(knn_handle_t h, const float *Q, int64_t m, const float *C, int64_t n, int d, int k, bool graph,
                        float *out_dist, int32_t *out_idx, hipStream_t stream, const knn_options_t *opt);
knn_status_t ensure_ooc_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
void set_host_rows(knn_handle_t h, int64_t rows);

// Key of a result entry: its distance class, then its global index; an absent
// entry (index -1) is the largest key, after every real one (NaN included).
__device__ __forceinline__ uint64_t entry_key(float dist, int32_t idx, int64_t off) {
    return idx < 0 ? kKeyMax : make_key(dist, (uint32_t)(idx + off));
}

// Row r: the k smallest entries of a (ka per row, global indices) and b (kb per
// row, indices local to a partition starting at b_off), both ascending by key,
// into out (k per row, global indices).  One thread per row, a two-pointer
// merge; entries are copied verbatim.
__global__ __launch_bounds__(256) void merge_topk_kernel(const float *__restrict__ ad, const int32_t *__restrict__ ai,
                                                         int ka, const float *__restrict__ bd,
                                                         const int32_t *__restrict__ bi, int kb, int64_t b_off,
                                                         int64_t m, int k, float *__restrict__ od,
                                                         int32_t *__restrict__ oi) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= m) return;
    const float *pa = ad + r * ka, *pb = bd + r * kb;
    const int32_t *qa = ai + r * ka, *qb = bi + r * kb;
    int x = 0, y = 0;
    uint64_t kx = x < ka ? entry_key(pa[0], qa[0], 0) : kKeyMax;
    uint64_t ky = y < kb ? entry_key(pb[0], qb[0], b_off) : kKeyMax;
    for (int t = 0; t < k; ++t) {
        float dv;
        int32_t iv;
        if (kx <= ky) {
            if (kx == kKeyMax) {  // both exhausted or absent
                dv = __uint_as_float(0x7f800000u);
                iv = -1;
            } else {
                dv = pa[x];
                iv = qa[x];
            }
            ++x;
            kx = x < ka ? entry_key(pa[x], qa[x], 0) : kKeyMax;
        } else {
            dv = pb[y];
            iv = (int32_t)(qb[y] + b_off);
            ++y;
            ky = y < kb ? entry_key(pb[y], qb[y], b_off) : kKeyMax;
        }
        od[r * k + t] = dv;
        oi[r * k + t] = iv;
    }
}

static hipError_t launch_merge(const float *ad, const int32_t *ai, int ka, const float *bd, const int32_t *bi, int kb,
                               int64_t b_off, int64_t m, int k, float *od, int32_t *oi, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(merge_topk_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ad, ai, ka, bd, bi, kb,
                       b_off, m, k, od, oi);
    return hipGetLastError();
}

knn_status_t run_search_host_corpus(knn_handle_t h, const float *Q, int64_t m, const float *C_host, int64_t n, int d,
                                    int k, int64_t part_rows, float *out_dist, int32_t *out_idx, hipStream_t stream,
                                    const knn_options_t *opt) {
    hipError_t e;
#define OTRY(call)                                                                                      \
    do {                                                                                                \
        if ((e = (call)) != hipSuccess) return fail_msg(h, KNN_ERROR_DEVICE, std::string(#call) + ": " + \
                                                                                 hipGetErrorString(e)); \
    } while (0)
    if (!h->copy_stream) {
        OTRY(hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking));
        for (int i = 0; i < 4; ++i) OTRY(hipEventCreateWithFlags(&h->ooc_ev[i], hipEventDisableTiming));
    }
    const int64_t R = part_rows < n ? part_rows : n;
    const int64_t parts = (n + R - 1) / R;
    // two partition buffers, then the partition result and two running results
    const size_t pbuf = (size_t)R * d * sizeof(float);
    const size_t res = (size_t)m * k * (sizeof(float) + sizeof(int32_t));
    void *ws = nullptr;
    knn_status_t st = ensure_ooc_ws(h, 2 * pbuf + 3 * res + 1024, stream, &ws);
    if (st != KNN_SUCCESS) return st;
    char *w = static_cast<char *>(ws);
    float *buf[2] = {reinterpret_cast<float *>(w), reinterpret_cast<float *>(w + pbuf)};
    auto res_at = [&](int i, float **dd, int32_t **ii) {
        char *b = w + 2 * pbuf + (size_t)i * res;
        *dd = reinterpret_cast<float *>(b);
        *ii = reinterpret_cast<int32_t *>(b + (size_t)m * k * sizeof(float));
    };
    float *pd, *rd[2];
    int32_t *pi, *ri[2];
    res_at(0, &pd, &pi);
    res_at(1, &rd[0], &ri[0]);
    res_at(2, &rd[1], &ri[1]);
    hipEvent_t *copied = h->ooc_ev, *freed = h->ooc_ev + 2;

    auto issue_copy = [&](int64_t p) -> hipError_t {
        const int64_t r0 = p * R, rows = n - r0 < R ? n - r0 : R;
        hipError_t ce = hipSuccess;
        if (p >= 2) ce = hipStreamWaitEvent(h->copy_stream, freed[p % 2], 0);
        if (ce == hipSuccess)
            ce = hipMemcpyAsync(buf[p % 2], C_host + r0 * d, (size_t)rows * d * sizeof(float), hipMemcpyHostToDevice,
                                h->copy_stream);
        if (ce == hipSuccess) ce = hipEventRecord(copied[p % 2], h->copy_stream);
        return ce;
    };
    // the copy stream starts after the work already enqueued on `stream` (the
    // buffers may still be read by an earlier call)
    OTRY(hipEventRecord(freed[0], stream));
    OTRY(hipStreamWaitEvent(h->copy_stream, freed[0], 0));
    OTRY(issue_copy(0));
    if (parts > 1) OTRY(issue_copy(1));
    int cur = 0;       // running result in rd[cur] / ri[cur], kcur entries per row
    int kcur = 0;
    for (int64_t p = 0; p < parts; ++p) {
        const int64_t r0 = p * R, rows = n - r0 < R ? n - r0 : R;
        const int kp = (int)(k < rows ? k : rows);
        const bool last = p + 1 == parts;
        OTRY(hipStreamWaitEvent(stream, copied[p % 2], 0));
        // a single partition writes the output directly; the first of several
        // becomes the running result (its indices are already global)
        float *sd = parts == 1 ? out_dist : (p == 0 ? rd[cur] : pd);
        int32_t *si = parts == 1 ? out_idx : (p == 0 ? ri[cur] : pi);
        st = run_search(h, Q, m, buf[p % 2], rows, d, kp, false, sd, si, stream, opt);
        if (st != KNN_SUCCESS) return st;
        OTRY(hipEventRecord(freed[p % 2], stream));
        if (p + 2 < parts) OTRY(issue_copy(p + 2));
        if (p == 0) {
            kcur = kp;
            continue;
        }
        const int kout = (int)(k < r0 + rows ? k : r0 + rows);
        float *od = last ? out_dist : rd[cur ^ 1];
        int32_t *oi = last ? out_idx : ri[cur ^ 1];
        OTRY(launch_merge(rd[cur], ri[cur], kcur, pd, pi, kp, r0, m, kout, od, oi, stream));
        cur ^= 1;
        kcur = kout;
    }
    set_host_rows(h, m);
#undef OTRY
    return KNN_SUCCESS;
}

}  // namespace knn
