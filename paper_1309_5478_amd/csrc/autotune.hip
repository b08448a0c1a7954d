// Measured tile-shape choice with a process-wide table and an optional JSON
// cache file (see autotune.hpp).
#include "autotune.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

namespace knn {

namespace {

std::mutex g_mu;
std::map<std::string, int> g_table;
bool g_file_read = false;

const char *cache_path() {
    const char *p = std::getenv("KNN_AUTOTUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Reads a flat JSON object of string keys and integer values.  Keys written by
// this module hold no quotes or backslashes; anything else ends the parse.
void read_file_locked() {
    g_file_read = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    size_t i = 0;
    while (true) {
        size_t q0 = text.find('"', i);
        if (q0 == std::string::npos) break;
        size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        size_t colon = text.find(':', q1 + 1);
        if (colon == std::string::npos) break;
        char *end = nullptr;
        long v = std::strtol(text.c_str() + colon + 1, &end, 10);
        if (end == text.c_str() + colon + 1) break;
        g_table.emplace(text.substr(q0 + 1, q1 - q0 - 1), (int)v);
        i = (size_t)(end - text.c_str());
    }
}

void write_file_locked() {
    const char *path = cache_path();
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fputs("{\n", f);
    size_t n = 0;
    for (const auto &kv : g_table) {
        std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++n < g_table.size() ? "," : "");
    }
    std::fputs("}\n", f);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

bool autotune_enabled(const knn_options_t *opt) {
    if (opt && (opt->flags & KNN_FLAG_AUTOTUNE)) return true;
    const char *e = std::getenv("KNN_AUTOTUNE");
    return e && std::strcmp(e, "1") == 0;
}

int autotune_lookup(const std::string &key) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_file_read) read_file_locked();
    auto it = g_table.find(key);
    return it == g_table.end() ? -1 : it->second;
}

int size_bucket(int64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

hipError_t autotune_pick(const std::string &key, const std::vector<int> &candidates,
                         const std::function<hipError_t(int)> &run, hipStream_t stream, int reps, int *choice,
                         float margin) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = candidates.empty() ? -1 : candidates[0];
    float best_ms = 0.f, first_ms = 0.f;
    for (size_t ci = 0; e == hipSuccess && ci < candidates.size(); ++ci) {
        const int c = candidates[ci];
        e = run(c);  // warm-up
        float cand_ms = 0.f;
        for (int r = 0; e == hipSuccess && r < reps; ++r) {
            e = hipEventRecord(e0, stream);
            if (e == hipSuccess) e = run(c);
            if (e == hipSuccess) e = hipEventRecord(e1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (r == 0 || ms < cand_ms)) cand_ms = ms;
        }
        if (e == hipSuccess && ci == 0) first_ms = cand_ms;
        if (e == hipSuccess && (ci == 0 || cand_ms < best_ms)) {
            best_ms = cand_ms;
            best = c;
        }
    }
    if (!candidates.empty() && best != candidates[0] && best_ms > first_ms * (1.f - margin)) best = candidates[0];
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_file_read) read_file_locked();
        g_table[key] = best;
        write_file_locked();
    }
    *choice = best;
    return hipSuccess;
}

}  // namespace knn
