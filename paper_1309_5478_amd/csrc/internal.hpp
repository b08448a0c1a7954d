// Host-side declarations shared between the C ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

enum PivotMode : int { kPivotPlain = 0, kPivotSample = 1, kPivotLearned = 2 };

// Device counters filled by the kernels of one call (uint64 each).
enum StatSlot : int {
    kStatRows = 0,
    kStatPasses = 1,
    kStatPassesMax = 2,
    kStatStreamPasses = 3,
    kStatSpillRows = 4,
    kStatFirstSurvivors = 5,
    kStatFallbackRows = 6,
    kStatCandidates = 7,
    kStatErrors = 8,
    kStatCycSample = 9,
    kStatCycStream = 10,
    kStatCycSelect = 11,
    kStatCycFinal = 12,
    kStatUncertified = 13,
    kStatCount = 14
};

// ---- selection over a given FP32 matrix ------------------------------------
// One matrix of a multi-matrix selection: its rows are rows row0 .. of the
// launch.  Either dense rows (dist, row stride ld) or key-list rows (keys,
// key_cnt, row stride ld), as in SelectArgs.
struct SelectSeg {
    const float *dist;
    const uint64_t *keys;
    const uint32_t *key_cnt;
    int64_t ld;
    int64_t row0;
    uint32_t cols, k;
    float *out_val;        // rows x k
    int32_t *out_idx;      // rows x k
};

struct SelectArgs {
    const float *dist;     // rows x cols, row stride ld
    int64_t rows;
    uint32_t cols;
    int64_t ld;
    uint32_t k;
    float *out_val;        // rows x k
    int32_t *out_idx;      // rows x k
    const uint16_t *net;   // pivot-network BF16 weights (learned mode), or null
    // key-list rows instead of `dist`: row r holds min(key_cnt[r], cols) keys at
    // keys + r * ld (cols must not exceed the kernel capacity)
    const uint64_t *keys;
    const uint32_t *key_cnt;
    int mode;              // PivotMode
    unsigned long long *stats;  // kStatCount counters, or null
    // several matrices in one launch: row r belongs to segs[row_seg[r]]; then
    // rows is the total, cols and k the largest of the segments (they size the
    // workspace and the capacity class), and dist / keys / outputs come from
    // the segments
    const SelectSeg *segs;
    const uint32_t *row_seg;
    // row counter for dynamic row claiming (set by launch_select), or null
    unsigned long long *next_row;
    // Rows split into parts (split > 1, dense rows only): launch row r is part
    // r % split of matrix row r / split, columns [p cols, min((p + 1) cols,
    // row_cols)); its min(k, part length) smallest keys, with the part's column
    // offset added to their indices, go to out_keys + r k and the rest of the
    // k slots are padded with the largest key.
    uint32_t split;
    uint32_t row_cols;
    // When set, every row's selected keys go here (rows x k, ascending) instead
    // of out_val / out_idx.
    uint64_t *out_keys;
    // Key-list rows whose keys index the columns of a given matrix: values of the
    // zero and NaN classes are copied from src + r * src_ld + index, so that they
    // keep their bits (sign of zero, NaN payload).
    const float *src;
    int64_t src_ld;
};

// Largest k a selection call supports.
constexpr int kSelectMaxK = 1024;
// LDS partition buffer size (keys) of the distance-matrix selection
constexpr int kSelectCap = 1024;

// Capacity class (keys held on chip per buffer) used for a given k.
int select_cap_for_k(uint32_t k);
// Workgroups to launch for `rows` rows (persistent grid) on a device with `num_cu` CUs.
int select_grid(int cap, int64_t rows, int num_cu);
// Global workspace bytes for a launch with `grid` workgroups over rows of `cols`.
size_t select_ws_bytes(int cap, uint32_t cols, int grid);
// Launch; `ws` must hold select_ws_bytes(...) bytes.
hipError_t launch_select(const SelectArgs &a, int cap, int grid, void *ws, hipStream_t stream);
// Selection over key-list rows (a.keys / a.key_cnt set, a.cols <= kSelectKeysCap).
constexpr int kSelectKeysCap = 4096;
// `counter` (8 bytes of device memory, or null for strided rows) holds the
// launch's row counter.
hipError_t launch_select_keys(const SelectArgs &a, void *counter, int64_t rows_grid_limit, int num_cu,
                              hipStream_t stream);

// ---- rows split across workgroups -----------------------------------------------
// Few long rows leave most of the device idle with one workgroup per row.  Each
// row is then cut into `parts` parts (a power of two) selected independently,
// and the parts' key lists are merged by key-list selections, up to `group`
// lists of k keys per merged row and level (a power of two with group k <=
// kSelectKeysCap), until one list per row remains: exact, since keys form a
// total order and the k smallest of a row lie among the k smallest of its parts.
struct SplitPlan {
    uint32_t parts, group, chunk;  // chunk: columns per part (a multiple of 4)
    int grid;                      // workgroups of the part selection
};
// parts = 1 when splitting is not worth it; `force` splits whenever the row is
// at least two minimal parts long.
SplitPlan select_split_plan(int64_t rows, uint32_t cols, uint32_t k, int num_cu, bool force);
size_t select_split_ws_bytes(const SplitPlan &sp, int64_t rows, uint32_t k);
// a: the whole call as for launch_select (dist, rows, cols, ld, k, outputs,
// mode, net, stats; out_idx may be null).
hipError_t launch_select_split(const SelectArgs &a, const SplitPlan &sp, void *ws, int num_cu, hipStream_t stream);

// ---- one partition pass, one wavefront per row ------------------------------
hipError_t launch_partition(const float *in, int64_t rows, uint32_t cols, int64_t ld,
                            const float *piv_val, const int32_t *piv_idx, float *out_val,
                            int32_t *out_idx, int32_t *out_left, hipStream_t stream);

// ---- utilities ------------------------------------------------------------------
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t stream);

}  // namespace knn
