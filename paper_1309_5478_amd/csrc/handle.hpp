// The libknn handle (shared by the C ABI translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "knn.h"

namespace knn {
struct BatchState;  // batch.hip
}

struct knn_handle_s {
    int device = 0;
    int num_cu = 0;
    std::string arch;
    void *ws = nullptr;        // general workspace, grows on demand
    void *uws = nullptr;       // unit-vector copies (cosine / Pearson), grows on demand
    size_t uws_bytes = 0;
    void *ooc = nullptr;       // host-corpus search: partition buffers and running results
    size_t ooc_bytes = 0;
    hipStream_t copy_stream = nullptr;       // host-to-device copies of corpus partitions
    hipEvent_t ooc_ev[4] = {nullptr, nullptr, nullptr, nullptr};  // copied[2], freed[2]
    void *scratch = nullptr;   // device address of this device's static scratch array
    size_t ws_bytes = 0;
    unsigned long long *stats_dev = nullptr;  // kStatCount counters
    hipStream_t last_stream = nullptr;
    knn_stats_t last{};
    bool stats_pending = false;
    int64_t host_rows = 0, host_fallback = 0, host_rerun = 0;  // host-side counters of the last call
    double host_product_ms = 0, host_product_flops = 0;
    int64_t host_product_launches = 0;
    int32_t last_split_parts = 1;              // parts per row of the last knn_select_k
    uint32_t *pinned = nullptr;                 // one pinned word for device-to-host counts
    std::string err;
    // pivot network: FP32 master weights, their BF16-rounded values (as FP32 for
    // training, as BF16 for inference) and the Adam moments
    float *net_theta = nullptr, *net_theta_r = nullptr, *net_m = nullptr, *net_v = nullptr, *net_grad = nullptr;
    uint16_t *net_bf16 = nullptr;
    int64_t net_step = 0;
    bool has_net = false;
    float net_quantile = 0.9f;
    // training examples of the pivot network (features rows x 8, targets)
    float *ex_x = nullptr, *ex_y = nullptr;
    int64_t ex_n = 0, ex_cap = 0;
    // plan, workspace and graphs of the last knn_batch_search
    knn::BatchState *batch = nullptr;
};

