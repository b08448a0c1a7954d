// C ABI of libknn (declared in include/knn.h): handles, argument validation,
// workspace management, statistics and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "dist.hpp"
#include "handle.hpp"
#include "internal.hpp"
#include "knn.h"

using namespace knn;

static thread_local std::string g_err;  // errors with no handle

namespace knn {
// Workspace of knn_select_k_noalloc: one array per device, reserved when the
// library's code object is loaded there and held until the process ends.  In
// host code `scratch` only names the symbol; its device address on each device
// comes from hipGetSymbolAddress, looked up once per device (knn_create).
constexpr size_t kScratchBytes = 64ull << 20;
// longest rows whose overflow buffers (2 (cols - 1024) keys) fit one workgroup
constexpr int64_t kScratchMaxCols = 1024 + (int64_t)((kScratchBytes - 256) / 16);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device `device`.
static hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipSuccess;  // none: the entry point reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace knn

static knn_status_t fail(knn_handle_t h, knn_status_t s, const std::string &msg) {
    if (h) h->err = msg;
    else g_err = msg;
    return s;
}

static knn_status_t hip_fail(knn_handle_t h, hipError_t e, const char *what) {
    return fail(h, KNN_ERROR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace knn {
knn_status_t run_search(knn_handle_t h, const float *Q, int64_t m, const float *C, int64_t n, int d, int k, bool graph,
                        float *out_dist, int32_t *out_idx, hipStream_t stream, const knn_options_t *opt);

knn_status_t run_batch(knn_handle_t h, const knn_job_t *jobs, int32_t njobs, hipStream_t stream,
                       const knn_options_t *opt);
knn_status_t run_search_host_corpus(knn_handle_t h, const float *Q, int64_t m, const float *C_host, int64_t n, int d,
                                    int k, int64_t part_rows, float *out_dist, int32_t *out_idx, hipStream_t stream,
                                    const knn_options_t *opt);
void batch_release(knn_handle_t h);
knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg) { return fail(h, s, msg); }
uint32_t *host_counter(knn_handle_t h) { return h->pinned; }
unsigned long long *stats_ptr(knn_handle_t h) { return h->stats_dev; }
int handle_num_cu(knn_handle_t h) { return h->num_cu; }
const uint16_t *handle_net(knn_handle_t h) { return h->has_net ? h->net_bf16 : nullptr; }
void add_host_stats(knn_handle_t h, int64_t rows, int64_t fallback_rows) {
    h->host_rows += rows;
    h->host_fallback += fallback_rows;
}
void add_host_rerun(knn_handle_t h, int64_t rows) { h->host_rerun += rows; }
void add_product_time(knn_handle_t h, double ms, double flops) {
    h->host_product_ms += ms;
    h->host_product_flops += flops;
    h->host_product_launches += 1;
}

// Ensures the handle buffer (*buf, *cap bytes) holds at least `bytes`; returns its pointer.
static knn_status_t ensure_buf(knn_handle_t h, void **buf, size_t *cap, size_t bytes, hipStream_t stream, void **out) {
    if (bytes <= *cap) {
        *out = *buf;
        return KNN_SUCCESS;
    }
    // earlier work on the previous stream may still use the old buffer
    if (*buf) {
        hipError_t e = hipStreamSynchronize(h->last_stream);
        if (e == hipSuccess && stream != h->last_stream) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    size_t want = bytes + bytes / 4;  // headroom to avoid regrowing
    hipError_t e = hipMalloc(buf, want);
    if (e != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return fail(h, KNN_ERROR_OUT_OF_MEMORY, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    *cap = want;
    *out = *buf;
    return KNN_SUCCESS;
}

// The handle's general workspace.
knn_status_t ensure_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out) {
    return ensure_buf(h, &h->ws, &h->ws_bytes, bytes, stream, out);
}

// The partition buffers and running results of knn_search_host_corpus.
knn_status_t ensure_ooc_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out) {
    return ensure_buf(h, &h->ooc, &h->ooc_bytes, bytes, stream, out);
}
void set_host_rows(knn_handle_t h, int64_t rows) { h->host_rows = rows; }

// The unit-vector copies of the cosine and Pearson distances (kept apart from
// the general workspace, which the Euclidean path on them may regrow).
knn_status_t ensure_unit_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out) {
    return ensure_buf(h, &h->uws, &h->uws_bytes, bytes, stream, out);
}
}  // namespace knn

extern "C" {

const char *knn_status_string(knn_status_t s) {
    switch (s) {
        case KNN_SUCCESS: return "success";
        case KNN_ERROR_INVALID_VALUE: return "invalid value";
        case KNN_ERROR_OUT_OF_MEMORY: return "out of device memory";
        case KNN_ERROR_UNSUPPORTED: return "unsupported";
        case KNN_ERROR_DEVICE: return "device error";
        case KNN_ERROR_IO: return "i/o error";
    }
    return "unknown status";
}

const char *knn_last_error(knn_handle_t h) { return h ? h->err.c_str() : g_err.c_str(); }

knn_status_t knn_create(knn_handle_t *out, int device) {
    if (!out) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_create: out is null");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return fail(nullptr, KNN_ERROR_DEVICE, "knn_create: no HIP device available");
    }
    if (device < 0 || device >= count) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_create: bad device ordinal");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fail(nullptr, KNN_ERROR_UNSUPPORTED, "knn_create: device is " + arch + ", libknn is built for gfx950 only");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    void *scr = nullptr;
    if ((e = scratch_address(device, &scr)) != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    knn_handle_t h = new knn_handle_s();
    h->device = device;
    h->scratch = scr;
    h->num_cu = prop.multiProcessorCount;
    h->arch = arch;
    if ((e = hipMalloc(&h->stats_dev, kStatCount * sizeof(unsigned long long))) != hipSuccess) {
        delete h;
        return hip_fail(nullptr, e, "hipMalloc(stats)");
    }
    if ((e = hipHostMalloc(&h->pinned, sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess) {
        hipFree(h->stats_dev);
        delete h;
        return hip_fail(nullptr, e, "hipHostMalloc");
    }
    *out = h;
    return KNN_SUCCESS;
}

knn_status_t knn_destroy(knn_handle_t h) {
    if (!h) return KNN_SUCCESS;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    batch_release(h);
    if (h->ws) hipFree(h->ws);
    if (h->uws) hipFree(h->uws);
    if (h->ooc) hipFree(h->ooc);
    for (hipEvent_t ev : h->ooc_ev)
        if (ev) hipEventDestroy(ev);
    if (h->copy_stream) hipStreamDestroy(h->copy_stream);
    if (h->stats_dev) hipFree(h->stats_dev);
    if (h->pinned) hipHostFree(h->pinned);
    for (void *p : {(void *)h->net_theta, (void *)h->net_theta_r, (void *)h->net_m, (void *)h->net_v,
                    (void *)h->net_grad, (void *)h->net_bf16, (void *)h->ex_x, (void *)h->ex_y})
        if (p) hipFree(p);
    delete h;
    return KNN_SUCCESS;
}

static knn_status_t begin_stats(knn_handle_t h, hipStream_t stream) {
    hipError_t e = launch_zero_u64(h->stats_dev, kStatCount, stream);
    if (e != hipSuccess) return hip_fail(h, e, "stats reset");
    h->last_stream = stream;
    h->stats_pending = true;
    h->host_rows = 0;
    h->host_fallback = 0;
    h->host_rerun = 0;
    h->host_product_ms = 0;
    h->host_product_flops = 0;
    h->host_product_launches = 0;
    h->last_split_parts = 1;
    return KNN_SUCCESS;
}

// Argument checks shared by knn_select_k and knn_select_k_noalloc.
static knn_status_t check_select(knn_handle_t h, const char *fn, const float *dist, int64_t rows, int64_t cols,
                                 int64_t ld, int32_t k, const float *out_val, const knn_options_t *opt) {
    const std::string f(fn);
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, f + ": handle is null");
    if (rows < 0) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": rows < 0");
    if (cols < 1) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": cols < 1");
    if (ld < cols) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": ld < cols");
    if (k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": k < 1");
    if (k > cols) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": k > cols");
    if (cols > INT32_MAX) return fail(h, KNN_ERROR_UNSUPPORTED, f + ": cols > INT32_MAX");
    if (k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, f + ": k > 1024");
    const int mode = opt ? opt->pivot : kPivotSample;
    if (mode < kPivotPlain || mode > kPivotLearned) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": bad pivot mode");
    if (rows > 0 && (!dist || !out_val)) return fail(h, KNN_ERROR_INVALID_VALUE, f + ": null pointer");
    return KNN_SUCCESS;
}

knn_status_t knn_select_k(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld, int32_t k,
                          float *out_val, int32_t *out_idx, void *stream_, const knn_options_t *opt) {
    knn_status_t cs = check_select(h, "knn_select_k", dist, rows, cols, ld, k, out_val, opt);
    if (cs != KNN_SUCCESS) return cs;
    if (rows == 0) return KNN_SUCCESS;
    int mode = opt ? opt->pivot : kPivotSample;
    const int flags = opt ? opt->flags : 0;
    if ((flags & KNN_FLAG_NO_SPLIT) && (flags & KNN_FLAG_FORCE_SPLIT))
        return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: NO_SPLIT and FORCE_SPLIT together");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if (mode == kPivotLearned && !h->has_net) mode = kPivotSample;  // no pivot network loaded: sample rule
    int cap = select_cap_for_k((uint32_t)k);
    SplitPlan sp{1, 1, (uint32_t)cols, 0};
    if (!(flags & KNN_FLAG_NO_SPLIT))
        sp = select_split_plan(rows, (uint32_t)cols, (uint32_t)k, h->num_cu, (flags & KNN_FLAG_FORCE_SPLIT) != 0);
    int grid = sp.parts > 1 ? sp.grid : select_grid(cap, rows, h->num_cu);
    void *ws = nullptr;
    size_t need = sp.parts > 1 ? select_split_ws_bytes(sp, rows, (uint32_t)k) : select_ws_bytes(cap, (uint32_t)cols, grid);
    knn_status_t st = ensure_ws(h, need < 256 ? 256 : need, stream, &ws);
    if (st != KNN_SUCCESS) return st;
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    h->last_split_parts = sp.parts;
    SelectArgs a{};
    a.dist = dist;
    a.rows = rows;
    a.cols = (uint32_t)cols;
    a.ld = ld;
    a.k = (uint32_t)k;
    a.out_val = out_val;
    a.out_idx = out_idx;
    a.net = mode == kPivotLearned ? h->net_bf16 : nullptr;
    a.mode = mode;
    a.stats = h->stats_dev;
    hipError_t e = sp.parts > 1 ? launch_select_split(a, sp, ws, h->num_cu, stream) : launch_select(a, cap, grid, ws, stream);
    if (e != hipSuccess) return hip_fail(h, e, "select kernel launch");
    return KNN_SUCCESS;
}

knn_status_t knn_select_k_noalloc(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld,
                                  int32_t k, float *out_val, int32_t *out_idx, void *stream_,
                                  const knn_options_t *opt) {
    knn_status_t cs = check_select(h, "knn_select_k_noalloc", dist, rows, cols, ld, k, out_val, opt);
    if (cs != KNN_SUCCESS) return cs;
    if (!h->scratch) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_select_k_noalloc: no scratch array on this device");
    const int cap = select_cap_for_k((uint32_t)k);
    // workgroups whose overflow buffers fit the array (all of them unless rows
    // are long: each needs 2 (cols - 1024) keys)
    const size_t one = select_ws_bytes(cap, (uint32_t)cols, 1), hdr = select_ws_bytes(cap, (uint32_t)cols, 0);
    if (one > kScratchBytes)
        return fail(h, KNN_ERROR_UNSUPPORTED,
                    "knn_select_k_noalloc: rows of " + std::to_string(cols) + " columns need " + std::to_string(one) +
                        " bytes of scratch per workgroup, above the " + std::to_string(kScratchBytes) +
                        "-byte array (at most " + std::to_string(kScratchMaxCols) + " columns)");
    if (rows == 0) return KNN_SUCCESS;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    int grid = select_grid(cap, rows, h->num_cu);
    if (one > hdr) {
        const int64_t fit = (int64_t)((kScratchBytes - hdr) / (one - hdr));
        if (grid > fit) grid = (int)fit;
    }
    knn_status_t st = begin_stats(h, stream);
    if (st != KNN_SUCCESS) return st;
    int mode = opt ? opt->pivot : kPivotSample;
    if (mode == kPivotLearned && !h->has_net) mode = kPivotSample;
    SelectArgs a{};
    a.dist = dist;
    a.rows = rows;
    a.cols = (uint32_t)cols;
    a.ld = ld;
    a.k = (uint32_t)k;
    a.out_val = out_val;
    a.out_idx = out_idx;
    a.net = mode == kPivotLearned ? h->net_bf16 : nullptr;
    a.mode = mode;
    a.stats = h->stats_dev;
    hipError_t e = launch_select(a, cap, grid, h->scratch, stream);
    if (e != hipSuccess) return hip_fail(h, e, "select kernel launch");
    return KNN_SUCCESS;
}

knn_status_t knn_partition(knn_handle_t h, const float *in, int64_t rows, int64_t cols, int64_t ld,
                           const float *piv_val, const int32_t *piv_idx, float *out_val, int32_t *out_idx,
                           int32_t *out_left, void *stream_) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_partition: handle is null");
    if (rows < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_partition: rows < 0");
    if (cols < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_partition: cols < 1");
    if (ld < cols) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_partition: ld < cols");
    if (cols > INT32_MAX) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_partition: cols > INT32_MAX");
    if (rows == 0) return KNN_SUCCESS;
    if (!in || !piv_val || !piv_idx || !out_val || !out_idx || !out_left)
        return fail(h, KNN_ERROR_INVALID_VALUE, "knn_partition: null pointer");
    hipSetDevice(h->device);
    hipError_t e = launch_partition(in, rows, (uint32_t)cols, ld, piv_val, piv_idx, out_val, out_idx, out_left,
                                    static_cast<hipStream_t>(stream_));
    if (e != hipSuccess) return hip_fail(h, e, "partition kernel launch");
    return KNN_SUCCESS;
}

static knn_status_t check_points(knn_handle_t h, const char *fn, const float *p, int64_t n, int32_t d) {
    if (n < 1) return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": corpus size < 1");
    if (d < 1) return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": d < 1");
    if (!p) return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": null pointer");
    if (n > INT32_MAX) return fail(h, KNN_ERROR_UNSUPPORTED, std::string(fn) + ": corpus larger than INT32_MAX");
    return KNN_SUCCESS;
}

static knn_status_t check_options(knn_handle_t h, const char *fn, const knn_options_t *opt) {
    if (!opt) return KNN_SUCCESS;
    if (opt->pivot < KNN_PIVOT_PLAIN || opt->pivot > KNN_PIVOT_LEARNED)
        return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": bad pivot mode");
    if (opt->oversample < 0) return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": oversample < 0");
    if (opt->precision < KNN_PREC_FP32 || opt->precision > KNN_PREC_FP8_E4M3)
        return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": bad precision");
    if (opt->metric < KNN_METRIC_SQEUCLIDEAN || opt->metric > KNN_METRIC_PEARSON)
        return fail(h, KNN_ERROR_INVALID_VALUE, std::string(fn) + ": bad metric");
    return KNN_SUCCESS;
}

knn_status_t knn_search(knn_handle_t h, const float *queries, int64_t m, const float *corpus, int64_t n, int32_t d,
                        int32_t k, float *out_dist, int32_t *out_idx, void *stream_, const knn_options_t *opt) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_search: handle is null");
    if (m < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search: m < 0");
    knn_status_t st = check_points(h, "knn_search", corpus, n, d);
    if (st != KNN_SUCCESS) return st;
    if (k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search: k < 1");
    if (k > n) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search: k > n");
    if (k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_search: k > 1024");
    if ((st = check_options(h, "knn_search", opt)) != KNN_SUCCESS) return st;
    if (m == 0) return KNN_SUCCESS;
    if (!queries || !out_dist || !out_idx) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search: null pointer");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    return run_search(h, queries, m, corpus, n, d, k, false, out_dist, out_idx, stream, opt);
}

knn_status_t knn_search_host_corpus(knn_handle_t h, const float *queries, int64_t m, const float *corpus_host,
                                    int64_t n, int32_t d, int32_t k, int64_t part_rows, float *out_dist,
                                    int32_t *out_idx, void *stream_, const knn_options_t *opt) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: handle is null");
    if (m < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: m < 0");
    knn_status_t st = check_points(h, "knn_search_host_corpus", corpus_host, n, d);
    if (st != KNN_SUCCESS) return st;
    if (k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: k < 1");
    if (k > n) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: k > n");
    if (k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_search_host_corpus: k > 1024");
    if (part_rows < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: part_rows < 0");
    if ((st = check_options(h, "knn_search_host_corpus", opt)) != KNN_SUCCESS) return st;
    if (m == 0) return KNN_SUCCESS;
    if (!queries || !out_dist || !out_idx) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_search_host_corpus: null pointer");
    if (part_rows == 0) {
        // partitions of about 1 GiB, never below k points
        part_rows = (int64_t)((1ull << 30) / ((size_t)d * sizeof(float)));
        if (part_rows < k) part_rows = k;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    return run_search_host_corpus(h, queries, m, corpus_host, n, d, k, part_rows, out_dist, out_idx, stream, opt);
}

knn_status_t knn_graph(knn_handle_t h, const float *points, int64_t n, int32_t d, int32_t k, float *out_dist,
                       int32_t *out_idx, void *stream_, const knn_options_t *opt) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_graph: handle is null");
    knn_status_t st = check_points(h, "knn_graph", points, n, d);
    if (st != KNN_SUCCESS) return st;
    if (k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_graph: k < 1");
    if (k > n - 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_graph: k > n - 1");
    if (k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_graph: k > 1024");
    if ((st = check_options(h, "knn_graph", opt)) != KNN_SUCCESS) return st;
    if (!out_dist || !out_idx) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_graph: null pointer");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    return run_search(h, points, n, points, n, d, k, true, out_dist, out_idx, stream, opt);
}

knn_status_t knn_batch_search(knn_handle_t h, const knn_job_t *jobs, int32_t njobs, void *stream_,
                              const knn_options_t *opt) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_batch_search: handle is null");
    if (njobs < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_batch_search: njobs < 0");
    if (njobs > 0 && !jobs) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_batch_search: jobs is null");
    knn_status_t st = check_options(h, "knn_batch_search", opt);
    if (st != KNN_SUCCESS) return st;
    for (int32_t j = 0; j < njobs; ++j) {
        const knn_job_t &b = jobs[j];
        const std::string fn = "knn_batch_search: job " + std::to_string(j);
        if ((st = check_points(h, fn.c_str(), b.corpus, b.n, b.d)) != KNN_SUCCESS) return st;
        if (b.m < 0) return fail(h, KNN_ERROR_INVALID_VALUE, fn + ": m < 0");
        if (b.k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, fn + ": k < 1");
        if (b.k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, fn + ": k > 1024");
        if (b.m > 0 && !b.queries && (b.m != b.n || b.n < 2))
            return fail(h, KNN_ERROR_INVALID_VALUE, fn + ": a graph job (null queries) needs m == n >= 2");
        if (b.m > 0 && (!b.out_dist || !b.out_idx)) return fail(h, KNN_ERROR_INVALID_VALUE, fn + ": null pointer");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    return run_batch(h, jobs, njobs, stream, opt);
}

knn_status_t knn_distances(knn_handle_t h, const float *queries, int64_t m, const float *corpus, int64_t n, int32_t d,
                           float *out, int64_t ldo, void *stream_) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_distances: handle is null");
    if (m < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_distances: m < 0");
    knn_status_t st = check_points(h, "knn_distances", corpus, n, d);
    if (st != KNN_SUCCESS) return st;
    if (ldo < n) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_distances: ldo < n");
    if (m == 0) return KNN_SUCCESS;
    if (!queries || !out) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_distances: null pointer");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    void *ws = nullptr;
    size_t need = (size_t)(m + n) * sizeof(float) + 512;
    if ((st = ensure_ws(h, need, stream, &ws)) != KNN_SUCCESS) return st;
    float *qn = static_cast<float *>(ws);
    float *cn = qn + ((m + 63) / 64) * 64;
    hipError_t e;
    if ((e = launch_sqnorm(queries, m, d, qn, nullptr, stream)) != hipSuccess) return hip_fail(h, e, "norm kernel");
    if ((e = launch_sqnorm(corpus, n, d, cn, nullptr, stream)) != hipSuccess) return hip_fail(h, e, "norm kernel");
    DistArgs a{};
    a.Q = queries;
    a.m = m;
    a.C = corpus;
    a.n = n;
    a.d = d;
    a.cnorm = cn;
    a.qnorm = qn;
    a.self_offset = -1;
    a.out = out;
    a.ldo = ldo;
    if ((e = launch_dist_gemm(a, kEpiDense, stream)) != hipSuccess) return hip_fail(h, e, "distance kernel");
    return KNN_SUCCESS;
}

knn_status_t knn_quantize(knn_handle_t h, const float *X, int64_t n, int32_t d, int32_t prec, void *out, float *scale,
                          void *stream_) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_quantize: handle is null");
    if (n < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_quantize: n < 0");
    if (d < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_quantize: d < 1");
    if (prec != KNN_PREC_BF16 && prec != KNN_PREC_FP8_E4M3)
        return fail(h, KNN_ERROR_INVALID_VALUE, "knn_quantize: precision must be BF16 or FP8 e4m3");
    if (n == 0) return KNN_SUCCESS;
    if (!X || !out || (prec == KNN_PREC_FP8_E4M3 && !scale))
        return fail(h, KNN_ERROR_INVALID_VALUE, "knn_quantize: null pointer");
    hipSetDevice(h->device);
    hipError_t e = launch_quantize(X, n, d, prec, out, scale, static_cast<hipStream_t>(stream_));
    if (e != hipSuccess) return hip_fail(h, e, "quantize kernel");
    return KNN_SUCCESS;
}

knn_status_t knn_get_stats(knn_handle_t h, knn_stats_t *out) {
    if (!h || !out) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_get_stats: null argument");
    hipSetDevice(h->device);
    if (h->stats_pending) {
        unsigned long long s[kStatCount];
        hipError_t e = hipStreamSynchronize(h->last_stream);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        e = hipMemcpy(s, h->stats_dev, sizeof(s), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(h, e, "hipMemcpy(stats)");
        if (s[kStatErrors] != 0)
            return fail(h, KNN_ERROR_DEVICE, "a kernel reported an internal error on " + std::to_string(s[kStatErrors]) + " rows");
        knn_stats_t t{};
        // a split row's parts count one row each
        t.rows = (int64_t)s[kStatRows] / (h->last_split_parts > 1 ? h->last_split_parts : 1);
        t.passes_total = (int64_t)s[kStatPasses];
        t.passes_max = (int32_t)s[kStatPassesMax];
        t.split_parts = h->last_split_parts;
        t.stream_passes_total = (int64_t)s[kStatStreamPasses];
        t.spill_rows = (int64_t)s[kStatSpillRows];
        t.first_pass_survivors = (int64_t)s[kStatFirstSurvivors];
        t.fallback_rows = (int64_t)s[kStatFallbackRows] + h->host_fallback;
        if (t.rows == 0) t.rows = h->host_rows;
        t.product_ms = h->host_product_ms;
        t.product_flops = h->host_product_flops;
        t.product_launches = h->host_product_launches;
        t.rows_uncertified = (int64_t)s[kStatUncertified];
        t.rows_rerun = h->host_rerun;
        t.candidates_total = (int64_t)s[kStatCandidates];
        t.phase_cycles[0] = (int64_t)s[kStatCycSample];
        t.phase_cycles[1] = (int64_t)s[kStatCycStream];
        t.phase_cycles[2] = (int64_t)s[kStatCycSelect];
        t.phase_cycles[3] = (int64_t)s[kStatCycFinal];
        h->last = t;
        h->stats_pending = false;
    }
    *out = h->last;
    return KNN_SUCCESS;
}

}  // extern "C"
