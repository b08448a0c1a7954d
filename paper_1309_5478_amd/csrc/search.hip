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
// When the sample is the whole corpus (small corpora), step 1 already selects
// each row's kk smallest keys and steps 2-3 are skipped.
// Unfused path (KNN_FLAG_UNFUSED): blocks of the distance matrix are
// materialised and selected directly, then re-ranked the same way.
#include <cmath>
#include <string>
#include <vector>

#include "autotune.hpp"
#include "dist.hpp"
#include "handle.hpp"
#include "internal.hpp"
#include "knn.h"
#include "plan.hpp"

namespace knn {

knn_status_t ensure_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
knn_status_t ensure_unit_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg);
uint32_t *host_counter(knn_handle_t h);
unsigned long long *stats_ptr(knn_handle_t h);
void add_host_stats(knn_handle_t h, int64_t rows, int64_t fallback_rows);
void add_host_rerun(knn_handle_t h, int64_t rows);
void add_product_time(knn_handle_t h, double ms, double flops);
int handle_num_cu(knn_handle_t h);
const uint16_t *handle_net(knn_handle_t h);

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_sum_u32(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t stream);

knn_status_t run_search(knn_handle_t h, const float *Q, int64_t m, const float *C, int64_t n, int d, int k, bool graph,
                        float *out_dist, int32_t *out_idx, hipStream_t stream, const knn_options_t *opt) {
    const int num_cu = handle_num_cu(h);
    // cosine / Pearson: the same path on unit vectors (centred for Pearson),
    // returning half their squared distance, 1 - similarity
    float oscale = 1.0f;
    const int metric = opt ? opt->metric : KNN_METRIC_SQEUCLIDEAN;
    if (metric != KNN_METRIC_SQEUCLIDEAN) {
        void *u = nullptr;
        const size_t need = (size_t)(graph ? n : n + m) * (size_t)d * sizeof(float);
        knn_status_t us = ensure_unit_ws(h, need, stream, &u);
        if (us != KNN_SUCCESS) return us;
        float *U = static_cast<float *>(u);
        const bool centre = metric == KNN_METRIC_PEARSON;
        hipError_t ue = launch_unit_rows(C, n, d, centre, U, stream);
        if (ue == hipSuccess && !graph) ue = launch_unit_rows(Q, m, d, centre, U + (size_t)n * d, stream);
        if (ue != hipSuccess) return fail_msg(h, KNN_ERROR_DEVICE, std::string("unit rows: ") + hipGetErrorString(ue));
        C = U;
        Q = graph ? U : U + (size_t)n * d;
        oscale = 0.5f;
    }
    // pivot rule of every quick multi-select in the path (the learned rule needs
    // a loaded pivot network; without one it is the sample rule)
    const uint16_t *net = handle_net(h);
    int smode = opt ? opt->pivot : kPivotSample;
    if (smode == kPivotLearned && !net) smode = kPivotSample;
    Plan p = make_plan(m, n, d, k, graph, opt, m);
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

    KNN_TRY(launch_fill_u32(b.cmax2, 1, 0u, stream));
    KNN_TRY(launch_sqnorm(C, n, d, b.cnorm, b.cmax2, stream));
    KNN_TRY(launch_sqnorm(Q, m, d, b.qn2, nullptr, stream));
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
    int64_t fallback_total = 0, rerun_total = 0;
    ProductTimer timer;
    KNN_TRY(timer.init(opt && (opt->flags & KNN_FLAG_TIMING)));
    uint32_t *hcount = host_counter(h);
    // FP32 rows whose candidate margin is not certified are re-run exactly
    const bool refix = certify && p.prec == kPrecF32;

    // certificate and exact re-rank of one block's kk candidates (ascending
    // reduced keys `keys`, corpus indices `cidx`), then the exact re-run of the
    // uncertified rows, from the block's materialised reduced-key rows when
    // there are (Dblock, row stride ldd), else from rows materialised here
    auto finish = [&](const float *keys, const int32_t *cidx, int64_t i0, int64_t mb, const float *Dblock,
                      int64_t ldd) -> knn_status_t {
        const float *Qb = Q + i0 * d;
        if (certify) {
            if (refix) KNN_TRY(launch_fill_u32(b.nu, 1, 0u, stream));
            CertifyArgs ca{keys, mb, p.kk, k, b.qn2 + i0, b.cmax2, p.rel, p.gamma, stats_ptr(h) + kStatUncertified,
                           refix ? b.ulist : nullptr, b.nu, b.tfix, refix && p.force_rerun};
            KNN_TRY(launch_certify(ca, stream));
        }
        RerankArgs rr{Qb, mb, C, n, d, cidx, (uint32_t)p.kk, k, out_dist + i0 * k, out_idx + i0 * k,
                      graph ? i0 : -1, oscale};
        KNN_TRY(launch_rerank(rr, stream));
        if (!refix) return KNN_SUCCESS;
        KNN_TRY(hipMemcpyAsync(hcount, b.nu, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        KNN_TRY(hipStreamSynchronize(stream));
        const int64_t nu = *hcount;
        rerun_total += nu;
        FixupArgs fx{};
        fx.out_scale = oscale;
        fx.tfix = b.tfix;
        fx.Q = Qb;
        fx.C = C;
        fx.n = n;
        fx.d = d;
        fx.k = k;
        fx.self_offset = graph ? i0 : -1;
        fx.out_dist = out_dist + i0 * k;
        fx.out_idx = out_idx + i0 * k;
        if (Dblock) {
            fx.D = Dblock;
            fx.ldd = ldd;
            fx.by_row = true;
            fx.rows = b.ulist;
            fx.nrows = nu;
            KNN_TRY(launch_fixup(fx, stream));
            return KNN_SUCCESS;
        }
        for (int64_t f0 = 0; f0 < nu; f0 += p.Fb) {
            const int64_t fb = nu - f0 < p.Fb ? nu - f0 : p.Fb;
            KNN_TRY(launch_gather_rows(Qb, mb, d, b.ulist + f0, fb, b.Qf, nullptr, nullptr, stream));
            DistArgs da{};
            da.Q = b.Qf;
            da.m = fb;
            da.C = C;
            da.n = n;
            da.d = d;
            da.cnorm = b.cnorm;
            da.self_offset = graph ? i0 : -1;
            da.row_ids = b.ulist + f0;
            da.out = b.Df;
            da.ldo = n;
            KNN_TRY(launch_dist_gemm(da, kEpiDense, stream));
            fx.D = b.Df;
            fx.ldd = n;
            fx.by_row = false;
            fx.rows = b.ulist + f0;
            fx.nrows = fb;
            KNN_TRY(launch_fixup(fx, stream));
        }
        return KNN_SUCCESS;
    };

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
            knn_status_t fs = finish(b.sv, b.si, i0, mb, b.Dm, n);
            if (fs != KNN_SUCCESS) return fs;
            if (timer.on) {
                KNN_TRY(hipStreamSynchronize(stream));
                KNN_TRY(timer.collect(h));
            }
        }
        add_host_stats(h, m, 0);
        add_host_rerun(h, rerun_total);
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
    // tile shape of the fused product: measured once per shape class when
    // autotuning is on (the timing launches keep nothing: threshold -inf)
    int ftile = -1;
    if (autotune_enabled(opt)) {
        const std::string key = "fused|" + h->arch + "|cu" + std::to_string(num_cu) + "|p" + std::to_string(p.prec) +
                                "|d" + std::to_string(d) + "|m" + std::to_string(size_bucket(p.Mb)) + "|n" +
                                std::to_string(size_bucket(n));
        ftile = autotune_lookup(key);
        if (ftile < 0) {
            KNN_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(b.ninf), 1, 0xFF800000u, stream));
            DistArgs pa{};
            pa.Q = Q;
            pa.m = p.Mb < 8192 ? p.Mb : 8192;
            pa.C = C;
            pa.n = n;
            pa.d = d;
            pa.cnorm = b.cnorm;
            pa.self_offset = graph ? 0 : -1;
            pa.tau = b.ninf;
            pa.tau_stride = 0;
            pa.cnt = b.cnt;
            pa.cand = b.cand;
            pa.cap = p.cap;
            set_prec(pa, qrow(0), qsrow(0), Cq, csc);
            // the default first, kept unless another shape is more than 3 %
            // faster: these probes keep nothing (threshold -inf), and the
            // candidate writes they leave out favour the default's more
            // resident workgroups per CU (512-job batch: probes tied, real
            // calls 4 % faster on the default)
            std::vector<int> cands = {kTileSmall1, kTileSmall, kTileWide};
            if (p.prec != kPrecFP8) cands.push_back(kTileBig);
            auto run = [&](int t) -> hipError_t {
                pa.tile = t;
                return launch_dist_gemm(pa, kEpiFilter, stream);
            };
            KNN_TRY(autotune_pick(key, cands, run, stream, 2, &ftile, 0.03f));
        }
    }
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
        if (!p.gathered) KNN_TRY(timer.begin(stream, 2.0 * (double)mb * (double)n * d));
        KNN_TRY(launch_dist_gemm(sa, kEpiDense, stream));
        if (!p.gathered) KNN_TRY(timer.end(stream));
        KNN_TRY(select_dense(b.Ds, mb, p.S, p.S, p.r + 1, b.tv, b.ti, b.selws, num_cu, smode, net, stream));
        if (!p.gathered) {
            // the sample is the whole corpus: its selection already holds each
            // row's kk smallest keys, in order, so the filtered product, the
            // candidate lists and their selection would only repeat it
            knn_status_t fs = finish(b.tv, b.ti, i0, mb, b.Ds, p.S);
            if (fs != KNN_SUCCESS) return fs;
            if (timer.on) {
                KNN_TRY(hipStreamSynchronize(stream));
                KNN_TRY(timer.collect(h));
            }
            continue;
        }
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
        fa.tile = ftile;
        fa.stage = b.stage;
        fa.stage_bytes = (int64_t)b.stage_bytes;
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
        KNN_TRY(launch_select_keys(ka, b.selws, mb, num_cu, stream));
        knn_status_t fs = finish(b.sv, b.si, i0, mb, nullptr, 0);
        if (fs != KNN_SUCCESS) return fs;
    }
#undef KNN_TRY
    add_host_stats(h, m, fallback_total);
    add_host_rerun(h, rerun_total);
    return KNN_SUCCESS;
}

}  // namespace knn
