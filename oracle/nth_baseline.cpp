// CPU comparison baseline for per-row k-smallest selection, the kind of CPU
// method the paper times its GPU selection against (Results: the standard
// library's nth_element on one CPU core).  Per row: (value, column) keys under
// the FP32 total order (-0 == +0, NaN == NaN above +inf), std::nth_element at
// k - 1, then std::sort of the first k; threaded over rows.
//
// TEST INFRASTRUCTURE ONLY: timed beside knn_select_k by the benchmark and
// checked against the oracle by the tests.  It shares no code with the HIP path
// and is not a reference for it (the oracle's stable sort is).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// Order-preserving integer image of an FP32 value under the total order.
uint32_t total_order_bits(float v) {
    if (std::isnan(v)) return 0xFFFFFFFFu;
    if (v == 0.0f) v = 0.0f;  // -0 == +0
    uint32_t u;
    std::memcpy(&u, &v, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

void select_rows(const float *D, int64_t r0, int64_t r1, int64_t cols, int64_t ld, int32_t k, float *ov,
                 int32_t *oi) {
    std::vector<uint64_t> keys((size_t)cols);
    for (int64_t r = r0; r < r1; ++r) {
        const float *row = D + r * ld;
        for (int64_t j = 0; j < cols; ++j) keys[(size_t)j] = ((uint64_t)total_order_bits(row[j]) << 32) | (uint64_t)j;
        std::nth_element(keys.begin(), keys.begin() + (k - 1), keys.end());
        std::sort(keys.begin(), keys.begin() + k);
        for (int32_t t = 0; t < k; ++t) {
            const uint32_t j = (uint32_t)keys[(size_t)t];
            ov[r * k + t] = row[j];
            oi[r * k + t] = (int32_t)j;
        }
    }
}

}  // namespace

extern "C" int nth_select_k(const float *D, int64_t rows, int64_t cols, int64_t ld, int32_t k, float *ov,
                            int32_t *oi, int32_t nthreads) {
    if (!D || !ov || !oi || rows < 0 || cols < 1 || ld < cols || k < 1 || k > cols) return 1;
    int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if ((int64_t)nt > rows) nt = rows > 0 ? (int)rows : 1;
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) {
        const int64_t a = rows * t / nt, b = rows * (t + 1) / nt;
        pool.emplace_back(select_rows, D, a, b, cols, ld, k, ov, oi);
    }
    for (auto &th : pool) th.join();
    return 0;
}
