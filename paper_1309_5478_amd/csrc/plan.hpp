// Per-call plan and workspace layout of the search / graph path (shared by the
// single-call and the batched entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdint>

#include "dist.hpp"
#include "internal.hpp"
#include "knn.h"

namespace knn {

void add_product_time(knn_handle_t h, double ms, double flops);

// Bump allocator over one workspace buffer (sizing pass with base == nullptr).
struct Carve {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

constexpr int kSampleCols = 2048;
constexpr int kSampleColsMax = 16384;
constexpr int64_t kRowBlock = 32768;
constexpr size_t kDenseBytes = size_t(1) << 30;  // materialised distance block budget

struct Plan {
    int64_t m, n, n_eff;
    int d, k, kk;
    int prec;          // kPrecF32 / kPrecBF16 / kPrecFP8
    int64_t ldq;       // bytes per quantised row
    float rel;         // relative dot-product error bound of the precision
    float gamma;       // relative error bound of an FP32 reduction over d terms
    bool graph, unfused;
    int force;
    int force_rerun;
    // fused
    int S;
    bool gathered;
    int r;
    int cap;
    int64_t Mb;
    int64_t Fb;
    // unfused
    int64_t Mu;
};

struct Bufs {
    float *cnorm = nullptr;
    float *qn2 = nullptr;
    unsigned int *cmax2 = nullptr;
    void *Cq = nullptr, *Qq = nullptr, *Csq = nullptr, *Qfq = nullptr;
    float *cs = nullptr, *qs = nullptr, *css = nullptr, *qfs = nullptr;
    float *Cs = nullptr, *csn = nullptr;
    float *Ds = nullptr, *tv = nullptr;
    int32_t *ti = nullptr;
    uint32_t *cnt = nullptr;
    uint64_t *cand = nullptr;
    int32_t *flags = nullptr;
    uint32_t *nflag = nullptr;
    float *sv = nullptr;
    int32_t *si = nullptr;
    float *Qf = nullptr, *Df = nullptr, *fv = nullptr;
    int32_t *fi = nullptr;
    float *Dm = nullptr;
    int32_t *ulist = nullptr;  // uncertified rows of the current block (FP32 re-run)
    uint32_t *nu = nullptr;
    float *tfix = nullptr;
    void *selws = nullptr;
    float *ninf = nullptr;  // one -inf: threshold of the tile-timing launches
    void *stage = nullptr;  // kept-key staging of the resident-corpus product
    size_t stage_bytes = 0;
};

inline size_t carve(Carve &c, const Plan &p, Bufs &b, int num_cu) {
    b.cnorm = c.take<float>(p.n);
    b.qn2 = c.take<float>(p.m);
    b.cmax2 = c.take<unsigned int>(1);
    if (p.prec != kPrecF32) {
        b.Cq = c.take<char>((size_t)p.n * p.ldq);
        b.cs = c.take<float>(p.n);
        if (!p.graph) {
            b.Qq = c.take<char>((size_t)p.m * p.ldq);
            b.qs = c.take<float>(p.m);
        }
        if (!p.unfused) {
            b.Csq = c.take<char>((size_t)p.S * p.ldq);
            b.css = c.take<float>(p.S);
            b.Qfq = c.take<char>((size_t)p.Fb * p.ldq);
            b.qfs = c.take<float>(p.Fb);
        }
    }
    size_t selws = 0;
    {
        const int64_t rows = p.unfused ? p.Mu : p.Mb;
        b.ulist = c.take<int32_t>((size_t)rows);
        b.tfix = c.take<float>((size_t)rows);
        b.nu = c.take<uint32_t>(1);
    }
    if (p.unfused) {
        b.Dm = c.take<float>((size_t)p.Mu * p.n);
        b.sv = c.take<float>((size_t)p.Mu * p.kk);
        b.si = c.take<int32_t>((size_t)p.Mu * p.kk);
        int cap = select_cap_for_k(p.kk);
        selws = select_ws_bytes(cap, (uint32_t)p.n, select_grid(cap, p.Mu, num_cu));
    } else {
        if (p.gathered) {
            b.Cs = c.take<float>((size_t)p.S * p.d);
            b.csn = c.take<float>(p.S);
        }
        b.Ds = c.take<float>((size_t)p.Mb * p.S);
        b.tv = c.take<float>((size_t)p.Mb * (p.r + 1));
        b.ti = c.take<int32_t>((size_t)p.Mb * (p.r + 1));
        b.cnt = c.take<uint32_t>(p.Mb);
        b.cand = c.take<uint64_t>((size_t)p.Mb * p.cap);
        if (p.prec != kPrecF32 && p.ldq <= 512) {
            // room for every row's full candidate list (key and row), plus one
            // count per wave of the resident-corpus grid (at most 8 waves per
            // 256 columns per 512 rows)
            const size_t waves = (size_t)((p.n + 255) / 256) * (size_t)(p.Mb / 512 + 2) * 8;
            b.stage_bytes = (size_t)p.Mb * p.cap * 12 + waves * 4 + 256;
            b.stage = c.take<char>(b.stage_bytes);
        }
        b.flags = c.take<int32_t>(p.Mb);
        b.nflag = c.take<uint32_t>(1);
        b.sv = c.take<float>((size_t)p.Mb * p.kk);
        b.si = c.take<int32_t>((size_t)p.Mb * p.kk);
        b.Qf = c.take<float>((size_t)p.Fb * p.d);
        b.Df = c.take<float>((size_t)p.Fb * p.n);
        b.fv = c.take<float>((size_t)p.Fb * p.kk);
        b.fi = c.take<int32_t>((size_t)p.Fb * p.kk);
        int cap1 = select_cap_for_k(p.r + 1);
        size_t w1 = select_ws_bytes(cap1, (uint32_t)p.S, select_grid(cap1, p.Mb, num_cu));
        int cap2 = select_cap_for_k(p.kk);
        size_t w2 = select_ws_bytes(cap2, (uint32_t)p.n, select_grid(cap2, p.Fb, num_cu));
        selws = w1 > w2 ? w1 : w2;
    }
    b.selws = c.take<char>(selws < 256 ? 256 : selws);
    b.ninf = c.take<float>(1);
    return c.off;
}

// Optional HIP-event timing of the main distance-product launches.
struct ProductTimer {
    bool on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double flops = 0;
    bool pending = false;
    ~ProductTimer() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    }
    hipError_t init(bool enable) {
        on = enable;
        if (!on) return hipSuccess;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        return e;
    }
    hipError_t begin(hipStream_t s, double f) {
        if (!on) return hipSuccess;
        flops = f;
        pending = true;
        return hipEventRecord(e0, s);
    }
    hipError_t end(hipStream_t s) { return on ? hipEventRecord(e1, s) : hipSuccess; }
    // after the stream has been synchronised past end()
    hipError_t collect(knn_handle_t h) {
        if (!on || !pending) return hipSuccess;
        float ms = 0;
        hipError_t e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) add_product_time(h, ms, flops);
        pending = false;
        return e;
    }
};

inline hipError_t select_dense(const float *D, int64_t rows, int64_t cols, int64_t ld, int k, float *ov, int32_t *oi,
                               void *ws, int num_cu, int mode, const uint16_t *net, hipStream_t stream) {
    SelectArgs a{};
    a.dist = D;
    a.rows = rows;
    a.cols = (uint32_t)cols;
    a.ld = ld;
    a.k = (uint32_t)k;
    a.out_val = ov;
    a.out_idx = oi;
    a.mode = mode;
    a.net = mode == kPivotLearned ? net : nullptr;
    int cap = select_cap_for_k((uint32_t)k);
    return launch_select(a, cap, select_grid(cap, rows, num_cu), ws, stream);
}

// The plan of one search / graph call: candidate oversampling, threshold sample,
// list capacity, row blocking.  Mb_limit caps the rows per block.
inline Plan make_plan(int64_t m, int64_t n, int d, int k, bool graph, const knn_options_t *opt, int64_t Mb_limit) {
    Plan p{};
    p.m = m;
    p.n = n;
    p.n_eff = graph ? n - 1 : n;
    p.d = d;
    p.k = k;
    p.graph = graph;
    int over = opt && opt->oversample > 0 ? opt->oversample : 4;
    int64_t kk = (int64_t)k * over;
    if (kk > kSelectMaxK) kk = kSelectMaxK;
    if (kk < k) kk = k;
    if (kk > p.n_eff) kk = p.n_eff;
    p.kk = (int)kk;
    p.unfused = opt && (opt->flags & KNN_FLAG_UNFUSED);
    p.force = (opt && (opt->flags & KNN_FLAG_FORCE_FALLBACK)) ? 1 : 0;
    p.force_rerun = (opt && (opt->flags & KNN_FLAG_FORCE_RERUN)) ? 1 : 0;
    p.prec = opt ? opt->precision : KNN_PREC_FP32;
    {
        const int dq = (d + kQuantPad - 1) / kQuantPad * kQuantPad;
        p.ldq = (int64_t)dq * (p.prec == kPrecBF16 ? 2 : 1);
        const double gamma = d * std::ldexp(1.0, -24) / (1.0 - d * std::ldexp(1.0, -24));
        const double u = p.prec == kPrecBF16 ? std::ldexp(1.0, -8) : (p.prec == kPrecFP8 ? std::ldexp(1.0, -4) : 0.0);
        p.rel = (float)(2 * u + u * u + gamma);
        p.gamma = (float)gamma;
    }
    if (p.unfused) {
        int64_t mu = (int64_t)(kDenseBytes / sizeof(float) / (size_t)n);
        p.Mu = mu < 1 ? 1 : (mu > m ? m : mu);
    } else {
        // sample columns: at least 2 n / kk (from 2048 up to 16384), and more while the
        // expected survivors of the threshold would exceed half the largest list
        // capacity, so that the candidate lists stay a few kk long and rarely overflow
        auto rank_for = [&](int64_t S, double &expected) -> int {
            if (n <= S) {
                expected = (double)p.kk;
                return p.kk - 1;  // the sample is the whole corpus (own index excluded)
            }
            const double mu = (double)S * p.kk / (double)p.n_eff;
            int64_t ri = (int64_t)std::ceil(mu + 3.0 * std::sqrt(mu) + 4.0);
            if (ri > S - 1) ri = S - 1;
            if (ri > kSelectMaxK - 1) ri = kSelectMaxK - 1;
            expected = (double)(ri + 1) * (double)p.n_eff / (double)S;
            return (int)ri;
        };
        int64_t S = kSampleCols;
        double expected = 0;
        for (;;) {
            rank_for(S, expected);
            const bool enough = S * p.kk >= 2 * n && 2.0 * expected <= kSelectKeysCap;
            if (enough || S >= kSampleColsMax || S >= n) break;
            S *= 2;
        }
        // then more sample columns while they cost less than the candidates
        // they save: with a small expected sample rank the margin above it lets
        // several kk through.  A kept candidate (its slot reservation and key
        // write in the product, its share of the candidate selection) costs
        // about 0.19 ns of the device (measured on the 2^20 x 256 BF16 graph);
        // a sample column costs, per row, its share of the sample product
        // (2 d flops) and a written and re-read distance.  Short reduced-
        // precision rows gain (2^20 x 256 BF16, kk = 256: 8192 -> 16384
        // columns, 1536 -> 1024 candidates per row expected, 1544 -> 1038
        // measured); long FP32 rows keep theirs.
        {
            const double t_keep = 1.9e-10;
            const double t_col = 2.0 * d / (p.prec == kPrecF32 ? 1.25e14 : 6.0e14) + 2.0e-12;
            while (2 * S <= kSampleColsMax && 2 * S < n) {
                double e2 = 0;
                rank_for(2 * S, e2);
                if (2.0 * e2 > kSelectKeysCap) break;
                if ((expected - e2) * t_keep <= (double)S * t_col) break;
                S *= 2;
                expected = e2;
            }
        }
        if (const char *e = std::getenv("KNN_SAMPLE_COLS")) {
            const long v = std::atol(e);
            if (v >= 64 && v <= 65536) S = v;
        }
        p.S = n < S ? (int)n : (int)S;
        p.gathered = n > p.S;
        p.r = rank_for(p.S, expected);
        // the survivor count varies with the sample's order statistic (relative
        // spread about 1 / sqrt(r + 1)): three times the expectation keeps
        // overflows (rows re-done exactly) rare
        int64_t cap = (int64_t)(3.0 * expected);
        if (cap < p.kk + 64) cap = p.kk + 64;
        cap = (cap + 63) / 64 * 64;
        if (cap > kSelectKeysCap) cap = kSelectKeysCap;
        p.cap = (int)cap;
        p.Mb = m < kRowBlock ? m : kRowBlock;
        if (p.Mb > Mb_limit) p.Mb = Mb_limit;
        int64_t fb = (int64_t)((size_t(256) << 20) / sizeof(float) / (size_t)n);
        p.Fb = fb < 1 ? 1 : (fb > p.Mb ? p.Mb : fb);
    }
    return p;
}

}  // namespace knn
