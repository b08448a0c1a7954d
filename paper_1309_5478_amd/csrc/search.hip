// Host orchestration of knn_search / knn_graph: brute-force k-NN by a distance
// matrix product fused with per-row selection (Methods: "Distance calculation"
// and "GPU-based quick multi-select"), on one device.
//
// Fused path, per block of query rows:
//  1. threshold: d' to S strided corpus samples (a small dense product), then
//     tau_i = the sample order statistic just above the expected rank of the
//     kk-th candidate (kk = oversample * k), by quick multi-select over the
//     sample row.  When the sample is the whole corpus, tau_i is the exact kk-th.
//  2. fused product: the full Q x C product with the FILTER epilogue, which
//     keeps d' <= tau_i in per-row candidate lists; the M x N matrix is never
//     stored.
//  3. rows with fewer than kk candidates (tau too low) or more than the list
//     capacity are listed and re-done exactly: their distance rows are
//     materialised and selected in full.
//  4. quick multi-select of the kk smallest reduced keys among each row's
//     candidates, then the exact FP32 direct-form re-rank of those kk and the
//     final k, in (distance, index) order.
// Unfused path (KNN_FLAG_UNFUSED): blocks of the distance matrix are
// materialised and selected directly, then re-ranked the same way.
#include <cmath>
#include <string>

#include "dist.hpp"
#include "internal.hpp"
#include "knn.h"

namespace knn {

knn_status_t ensure_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg);
uint32_t *host_counter(knn_handle_t h);
unsigned long long *stats_ptr(knn_handle_t h);
void add_host_stats(knn_handle_t h, int64_t rows, int64_t fallback_rows);
void add_product_time(knn_handle_t h, double ms, double flops);
int handle_num_cu(knn_handle_t h);
const uint16_t *handle_net(knn_handle_t h);

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_sum_u32(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t stream);

namespace {

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
    bool graph, unfused;
    int force;
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
    void *selws = nullptr;
};

size_t carve(Carve &c, const Plan &p, Bufs &b, int num_cu) {
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

hipError_t select_dense(const float *D, int64_t rows, int64_t cols, int64_t ld, int k, float *ov, int32_t *oi,
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

}  // namespace

knn_status_t run_search(knn_handle_t h, const float *Q, int64_t m, const float *C, int64_t n, int d, int k, bool graph,
                        float *out_dist, int32_t *out_idx, hipStream_t stream, const knn_options_t *opt) {
    const int num_cu = handle_num_cu(h);
    // pivot rule of every quick multi-select in the path (the learned rule needs
    // a loaded pivot network; without one it is the sample rule)
    const uint16_t *net = handle_net(h);
    int smode = opt ? opt->pivot : kPivotSample;
    if (smode == kPivotLearned && !net) smode = kPivotSample;
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
    p.prec = opt ? opt->precision : KNN_PREC_FP32;
    {
        const int dq = (d + kQuantPad - 1) / kQuantPad * kQuantPad;
        p.ldq = (int64_t)dq * (p.prec == kPrecBF16 ? 2 : 1);
        const double gamma = d * std::ldexp(1.0, -24) / (1.0 - d * std::ldexp(1.0, -24));
        const double u = p.prec == kPrecBF16 ? std::ldexp(1.0, -8) : (p.prec == kPrecFP8 ? std::ldexp(1.0, -4) : 0.0);
        p.rel = (float)(2 * u + u * u + gamma);
    }

    if (p.unfused) {
        int64_t mu = (int64_t)(kDenseBytes / sizeof(float) / (size_t)n);
        p.Mu = mu < 1 ? 1 : (mu > m ? m : mu);
    } else {
        // sample columns: about 2 n / kk (at least 2048, at most 16384), so that the
        // expected survivors of the threshold stay a few kk and within the list capacity
        int64_t S = kSampleCols;
        while (S < kSampleColsMax && S * p.kk < 2 * n) S *= 2;
        p.S = n < S ? (int)n : (int)S;
        p.gathered = n > p.S;
        if (!p.gathered) {
            p.r = p.kk - 1;  // the sample is the whole corpus (own index excluded)
        } else {
            double mu = (double)p.S * p.kk / (double)p.n_eff;
            double r = std::ceil(mu + 3.0 * std::sqrt(mu) + 4.0);
            int64_t ri = (int64_t)r;
            if (ri > p.S - 1) ri = p.S - 1;
            if (ri > kSelectMaxK - 1) ri = kSelectMaxK - 1;
            p.r = (int)ri;
        }
        double expected = p.gathered ? (double)(p.r + 1) * (double)p.n_eff / p.S : (double)p.kk;
        int64_t cap = (int64_t)(2.0 * expected);
        if (cap < p.kk + 64) cap = p.kk + 64;
        cap = (cap + 63) / 64 * 64;
        if (cap > kSelectKeysCap) cap = kSelectKeysCap;
        p.cap = (int)cap;
        p.Mb = m < kRowBlock ? m : kRowBlock;
        int64_t fb = (int64_t)((size_t(256) << 20) / sizeof(float) / (size_t)n);
        p.Fb = fb < 1 ? 1 : (fb > p.Mb ? p.Mb : fb);
    }

    Bufs b;
    Carve sizing{nullptr};
    size_t bytes = carve(sizing, p, b, num_cu);
    void *ws = nullptr;
    knn_status_t st = ensure_ws(h, bytes, stream, &ws);
    if (st != KNN_SUCCESS) return st;
    Carve real{static_cast<char *>(ws)};
    carve(real, p, b, num_cu);

    hipError_t e;
#define KNN_TRY(call)                                                                                   \
    do {                                                                                                \
        if ((e = (call)) != hipSuccess) return fail_msg(h, KNN_ERROR_DEVICE, std::string(#call) + ": " + \
                                                                                 hipGetErrorString(e)); \
    } while (0)

    KNN_TRY(launch_sqnorm(C, n, d, b.cnorm, stream));
    KNN_TRY(launch_sqnorm(Q, m, d, b.qn2, stream));
    KNN_TRY(launch_fill_u32(b.cmax2, 1, 0u, stream));
    KNN_TRY(launch_max_nonneg(b.cnorm, n, b.cmax2, stream));
    const void *Qq = nullptr, *Cq = nullptr;
    const float *qsc = nullptr, *csc = nullptr;
    if (p.prec != kPrecF32) {
        KNN_TRY(launch_quantize(C, n, d, p.prec, b.Cq, b.cs, stream));
        Cq = b.Cq;
        csc = b.cs;
        if (graph) {
            Qq = b.Cq;
            qsc = b.cs;
        } else {
            KNN_TRY(launch_quantize(Q, m, d, p.prec, b.Qq, b.qs, stream));
            Qq = b.Qq;
            qsc = b.qs;
        }
    }
    auto set_prec = [&](DistArgs &a, const void *qq, const float *qs, const void *cq, const float *cs) {
        a.prec = p.prec;
        a.Qq = qq;
        a.Cq = cq;
        a.ldq = p.ldq;
        a.qscale = qs;
        a.cscale = cs;
    };
    auto qrow = [&](int64_t i0) -> const void * {
        return Qq ? static_cast<const char *>(Qq) + i0 * p.ldq : nullptr;
    };
    auto qsrow = [&](int64_t i0) -> const float * { return qsc ? qsc + i0 : nullptr; };
    const bool certify = p.kk < p.n_eff;
    int64_t fallback_total = 0;
    ProductTimer timer;
    KNN_TRY(timer.init(opt && (opt->flags & KNN_FLAG_TIMING)));

    if (p.unfused) {
        for (int64_t i0 = 0; i0 < m; i0 += p.Mu) {
            const int64_t mb = m - i0 < p.Mu ? m - i0 : p.Mu;
            DistArgs a{};
            a.Q = Q + i0 * d;
            a.m = mb;
            a.C = C;
            a.n = n;
            a.d = d;
            a.cnorm = b.cnorm;
            a.self_offset = graph ? i0 : -1;
            a.out = b.Dm;
            a.ldo = n;
            set_prec(a, qrow(i0), qsrow(i0), Cq, csc);
            KNN_TRY(timer.begin(stream, 2.0 * (double)mb * (double)n * d));
            KNN_TRY(launch_dist_gemm(a, kEpiDense, stream));
            KNN_TRY(timer.end(stream));
            KNN_TRY(select_dense(b.Dm, mb, n, n, p.kk, b.sv, b.si, b.selws, num_cu, smode, net, stream));
            if (certify)
                KNN_TRY(launch_certify(b.sv, mb, p.kk, k, b.qn2 + i0, b.cmax2, p.rel, stats_ptr(h) + kStatUncertified,
                                       stream));
            RerankArgs rr{Q + i0 * d, mb, C, n, d, b.si, (uint32_t)p.kk, k, out_dist + i0 * k, out_idx + i0 * k};
            KNN_TRY(launch_rerank(rr, stream));
            if (timer.on) {
                KNN_TRY(hipStreamSynchronize(stream));
                KNN_TRY(timer.collect(h));
            }
        }
        add_host_stats(h, m, 0);
        return KNN_SUCCESS;
    }

    const float *Cs = C, *csn = b.cnorm;
    const void *Csq = Cq;
    const float *css = csc;
    if (p.gathered) {
        KNN_TRY(launch_gather_rows(C, n, d, nullptr, p.S, b.Cs, b.cnorm, b.csn, stream));
        Cs = b.Cs;
        csn = b.csn;
        if (p.prec != kPrecF32) {
            KNN_TRY(launch_quantize(b.Cs, p.S, d, p.prec, b.Csq, b.css, stream));
            Csq = b.Csq;
            css = b.css;
        }
    }
    uint32_t *hcount = host_counter(h);
    for (int64_t i0 = 0; i0 < m; i0 += p.Mb) {
        const int64_t mb = m - i0 < p.Mb ? m - i0 : p.Mb;
        const float *Qb = Q + i0 * d;
        // 1. thresholds from the sample
        DistArgs sa{};
        sa.Q = Qb;
        sa.m = mb;
        sa.C = Cs;
        sa.n = p.S;
        sa.d = d;
        sa.cnorm = csn;
        sa.self_offset = (graph && !p.gathered) ? i0 : -1;
        sa.out = b.Ds;
        sa.ldo = p.S;
        set_prec(sa, qrow(i0), qsrow(i0), Csq, css);
        KNN_TRY(launch_dist_gemm(sa, kEpiDense, stream));
        KNN_TRY(select_dense(b.Ds, mb, p.S, p.S, p.r + 1, b.tv, b.ti, b.selws, num_cu, smode, net, stream));
        // 2. fused product + filter
        KNN_TRY(launch_fill_u32(b.cnt, mb, 0u, stream));
        DistArgs fa{};
        fa.Q = Qb;
        fa.m = mb;
        fa.C = C;
        fa.n = n;
        fa.d = d;
        fa.cnorm = b.cnorm;
        fa.self_offset = graph ? i0 : -1;
        fa.tau = b.tv + p.r;
        fa.tau_stride = p.r + 1;
        fa.cnt = b.cnt;
        fa.cand = b.cand;
        fa.cap = p.cap;
        set_prec(fa, qrow(i0), qsrow(i0), Cq, csc);
        KNN_TRY(timer.begin(stream, 2.0 * (double)mb * (double)n * d));
        KNN_TRY(launch_dist_gemm(fa, kEpiFilter, stream));
        KNN_TRY(timer.end(stream));
        KNN_TRY(launch_sum_u32(b.cnt, mb, stats_ptr(h) + kStatCandidates, stream));
        // 3. exact re-do of rows whose candidate list is unusable
        KNN_TRY(launch_fill_u32(b.nflag, 1, 0u, stream));
        KNN_TRY(launch_flag_rows(b.cnt, mb, (uint32_t)p.kk, (uint32_t)p.cap, p.force, b.nflag, b.flags, stream));
        KNN_TRY(hipMemcpyAsync(hcount, b.nflag, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        KNN_TRY(hipStreamSynchronize(stream));
        KNN_TRY(timer.collect(h));
        const int64_t nf = *hcount;
        fallback_total += nf;
        for (int64_t f0 = 0; f0 < nf; f0 += p.Fb) {
            const int64_t fb = nf - f0 < p.Fb ? nf - f0 : p.Fb;
            KNN_TRY(launch_gather_rows(Qb, mb, d, b.flags + f0, fb, b.Qf, nullptr, nullptr, stream));
            if (p.prec != kPrecF32) KNN_TRY(launch_quantize(b.Qf, fb, d, p.prec, b.Qfq, b.qfs, stream));
            DistArgs da{};
            da.Q = b.Qf;
            da.m = fb;
            da.C = C;
            da.n = n;
            da.d = d;
            da.cnorm = b.cnorm;
            da.self_offset = graph ? i0 : -1;
            da.row_ids = b.flags + f0;
            da.out = b.Df;
            da.ldo = n;
            set_prec(da, b.Qfq, b.qfs, Cq, csc);
            KNN_TRY(launch_dist_gemm(da, kEpiDense, stream));
            KNN_TRY(select_dense(b.Df, fb, n, n, p.kk, b.fv, b.fi, b.selws, num_cu, smode, net, stream));
            KNN_TRY(launch_scatter_fallback(b.flags + f0, fb, b.fv, b.fi, p.kk, b.cand, b.cnt, p.cap, stream));
        }
        // 4. kk smallest candidates, exact re-rank, final k
        SelectArgs ka{};
        ka.keys = b.cand;
        ka.key_cnt = b.cnt;
        ka.rows = mb;
        ka.cols = (uint32_t)p.cap;
        ka.ld = p.cap;
        ka.k = (uint32_t)p.kk;
        ka.out_val = b.sv;
        ka.out_idx = b.si;
        ka.mode = smode;
        KNN_TRY(launch_select_keys(ka, mb, num_cu, stream));
        if (certify)
            KNN_TRY(launch_certify(b.sv, mb, p.kk, k, b.qn2 + i0, b.cmax2, p.rel, stats_ptr(h) + kStatUncertified,
                                   stream));
        RerankArgs rr{Qb, mb, C, n, d, b.si, (uint32_t)p.kk, k, out_dist + i0 * k, out_idx + i0 * k};
        KNN_TRY(launch_rerank(rr, stream));
    }
#undef KNN_TRY
    add_host_stats(h, m, fallback_total);
    return KNN_SUCCESS;
}

}  // namespace knn
