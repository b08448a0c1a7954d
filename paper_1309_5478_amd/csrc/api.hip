// C ABI of libknn (declared in include/knn.h): handles, argument validation,
// workspace management, statistics and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "knn.h"

using namespace knn;

struct knn_handle_s {
    int device = 0;
    int num_cu = 0;
    std::string arch;
    void *ws = nullptr;        // general workspace, grows on demand
    size_t ws_bytes = 0;
    unsigned long long *stats_dev = nullptr;  // kStatCount counters
    hipStream_t last_stream = nullptr;
    knn_stats_t last{};
    bool stats_pending = false;
    std::string err;
    int grid_cache[3] = {0, 0, 0};  // blocks per CU per select capacity class
};

static thread_local std::string g_err;  // errors with no handle

static knn_status_t fail(knn_handle_t h, knn_status_t s, const std::string &msg) {
    if (h) h->err = msg;
    else g_err = msg;
    return s;
}

static knn_status_t hip_fail(knn_handle_t h, hipError_t e, const char *what) {
    return fail(h, KNN_ERROR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace knn {
// Ensures the handle's workspace holds at least `bytes`; returns its pointer.
knn_status_t ensure_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out) {
    if (bytes <= h->ws_bytes) {
        *out = h->ws;
        return KNN_SUCCESS;
    }
    // earlier work on the previous stream may still use the old buffer
    if (h->ws) {
        hipError_t e = hipStreamSynchronize(h->last_stream);
        if (e == hipSuccess && stream != h->last_stream) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t want = bytes + bytes / 4;  // headroom to avoid regrowing
    hipError_t e = hipMalloc(&h->ws, want);
    if (e != hipSuccess) {
        h->ws = nullptr;
        (void)hipGetLastError();
        return fail(h, KNN_ERROR_OUT_OF_MEMORY, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    h->ws_bytes = want;
    *out = h->ws;
    return KNN_SUCCESS;
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
    knn_handle_t h = new knn_handle_s();
    h->device = device;
    h->num_cu = prop.multiProcessorCount;
    h->arch = arch;
    if ((e = hipMalloc(&h->stats_dev, kStatCount * sizeof(unsigned long long))) != hipSuccess) {
        delete h;
        return hip_fail(nullptr, e, "hipMalloc(stats)");
    }
    *out = h;
    return KNN_SUCCESS;
}

knn_status_t knn_destroy(knn_handle_t h) {
    if (!h) return KNN_SUCCESS;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    if (h->ws) hipFree(h->ws);
    if (h->stats_dev) hipFree(h->stats_dev);
    delete h;
    return KNN_SUCCESS;
}

static knn_status_t begin_stats(knn_handle_t h, hipStream_t stream) {
    hipError_t e = launch_zero_u64(h->stats_dev, kStatCount, stream);
    if (e != hipSuccess) return hip_fail(h, e, "stats reset");
    h->last_stream = stream;
    h->stats_pending = true;
    return KNN_SUCCESS;
}

knn_status_t knn_select_k(knn_handle_t h, const float *dist, int64_t rows, int64_t cols, int64_t ld, int32_t k,
                          float *out_val, int32_t *out_idx, void *stream_, const knn_options_t *opt) {
    if (!h) return fail(nullptr, KNN_ERROR_INVALID_VALUE, "knn_select_k: handle is null");
    if (rows < 0) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: rows < 0");
    if (cols < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: cols < 1");
    if (ld < cols) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: ld < cols");
    if (k < 1) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: k < 1");
    if (k > cols) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: k > cols");
    if (cols > INT32_MAX) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_select_k: cols > INT32_MAX");
    if (k > kSelectMaxK) return fail(h, KNN_ERROR_UNSUPPORTED, "knn_select_k: k > 1024");
    int mode = opt ? opt->pivot : kPivotSample;
    if (mode < kPivotPlain || mode > kPivotLearned) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: bad pivot mode");
    if (rows == 0) return KNN_SUCCESS;
    if (!dist || !out_val || !out_idx) return fail(h, KNN_ERROR_INVALID_VALUE, "knn_select_k: null pointer");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipSetDevice(h->device);
    if (mode == kPivotLearned) mode = kPivotSample;  // no pivot network loaded: sample rule
    int cap = select_cap_for_k((uint32_t)k);
    int grid = select_grid(cap, rows, h->num_cu);
    void *ws = nullptr;
    size_t need = select_ws_bytes(cap, (uint32_t)cols, grid);
    knn_status_t st = ensure_ws(h, need < 256 ? 256 : need, stream, &ws);
    if (st != KNN_SUCCESS) return st;
    if ((st = begin_stats(h, stream)) != KNN_SUCCESS) return st;
    SelectArgs a{};
    a.dist = dist;
    a.rows = rows;
    a.cols = (uint32_t)cols;
    a.ld = ld;
    a.k = (uint32_t)k;
    a.out_val = out_val;
    a.out_idx = out_idx;
    a.pivot_hint = nullptr;
    a.mode = mode;
    a.stats = h->stats_dev;
    hipError_t e = launch_select(a, cap, grid, ws, stream);
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
        t.rows = (int64_t)s[kStatRows];
        t.passes_total = (int64_t)s[kStatPasses];
        t.passes_max = (int32_t)s[kStatPassesMax];
        t.stream_passes_total = (int64_t)s[kStatStreamPasses];
        t.spill_rows = (int64_t)s[kStatSpillRows];
        t.first_pass_survivors = (int64_t)s[kStatFirstSurvivors];
        t.fallback_rows = (int64_t)s[kStatFallbackRows];
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
