// Measured choice of the distance product's tile shape.
//
// A choice is keyed by a string that names the device and the shape class of
// the work (precision, dimension, size buckets).  The first time a key is seen
// with autotuning enabled, every candidate is timed with HIP events on the
// caller's operands (a side-effect-free launch, see the callers) and the fastest
// is kept: in a process-wide table and, when the environment variable
// KNN_AUTOTUNE_CACHE names a file, in that JSON file ({"key": choice, ...}),
// which later processes read back.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "knn.h"

namespace knn {

// Autotuning requested by the options (KNN_FLAG_AUTOTUNE) or by KNN_AUTOTUNE=1.
bool autotune_enabled(const knn_options_t *opt);

// Cached choice for `key`, or -1.
int autotune_lookup(const std::string &key);

// Times run(c) for every candidate c on `stream` (one warm-up launch, then the
// best of `reps` timed launches) and returns the fastest in *choice, recording
// it under `key`; the first candidate (the preferred one) is kept unless
// another is faster by more than the fraction `margin`.  The stream is
// synchronised.
hipError_t autotune_pick(const std::string &key, const std::vector<int> &candidates,
                         const std::function<hipError_t(int)> &run, hipStream_t stream, int reps, int *choice,
                         float margin = 0.f);

// log2 bucket of a positive size (floor).
int size_bucket(int64_t x);

}  // namespace knn
