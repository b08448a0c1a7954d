// knn_batch_search: many independent k-NN jobs of uneven sizes in one call.
//
// Every job follows the steps of knn_search (threshold from a corpus sample,
// fused product with candidate filtering, exact fallback of unusable rows,
// candidate selection, exact re-rank), so its output is the same.  What changes
// is how the work reaches the device:
//  * the fused products of all jobs run as ONE launch of (job part, row tile,
//    column tile) items that the host orders for the hardware's round-robin
//    dispatch over the eight XCDs: per XCD a queue of parts, longest first, a
//    part's column range split into eight contiguous chunks, one per XCD, so
//    each corpus tile is read by one XCD, where the part's row tiles reuse it
//    from L2.  The items run one per workgroup, or (queue form) a resident
//    grid takes them from eight per-XCD atomic queues in the same order;
//  * every step of a call (norms, sample product, threshold selection, the
//    product, list flagging, candidate selection, certificate, re-rank) is
//    captured into one HIP graph on the first call and replayed by later calls
//    with the same job table; one synchronisation then brings the counts of
//    rows needing the exact fallback or re-run (rare) to the host;
//  * with autotuning on, the tile shape and form of the grouped launch are
//    the fastest of the candidates, timed on the batch itself with a threshold
//    of -inf (nothing is kept, so the timing run has no effect on the results).
// Jobs with more than kRowBlock queries are split into parts of at most that
// many rows; each part has its own candidate lists.  Jobs whose threshold
// sample is their whole corpus are finished in the first phase, as in
// knn_search.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "autotune.hpp"
#include "dist.hpp"
#include "handle.hpp"
#include "internal.hpp"
#include "knn.h"
#include "plan.hpp"

namespace knn {

knn_status_t fail_msg(knn_handle_t h, knn_status_t s, const std::string &msg);
unsigned long long *stats_ptr(knn_handle_t h);
void add_host_stats(knn_handle_t h, int64_t rows, int64_t fallback_rows);
void add_host_rerun(knn_handle_t h, int64_t rows);
int handle_num_cu(knn_handle_t h);
const uint16_t *handle_net(knn_handle_t h);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_sum_u32(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t stream);
knn_status_t ensure_unit_ws(knn_handle_t h, size_t bytes, hipStream_t stream, void **out);
knn_status_t run_search(knn_handle_t h, const float *Q, int64_t m, const float *C, int64_t n, int d, int k, bool graph,
                        float *out_dist, int32_t *out_idx, hipStream_t stream, const knn_options_t *opt);

struct BatchJob {
    const float *Q, *C;
    int64_t m, n;
    int d, k;
    bool graph;
    float *out_dist;
    int32_t *out_idx;
    Plan p;
    double cost;  // 2 m n d
    float oscale = 1.0f;  // returned distance = oscale * squared distance (cosine / Pearson: 1/2)
    // per-job buffers
    float *cnorm = nullptr, *qn2 = nullptr;
    unsigned int *cmax2 = nullptr;
    void *Cq = nullptr, *Qq = nullptr;
    float *cs = nullptr, *qs = nullptr;
    // the threshold sample of the corpus (the corpus itself when not gathered)
    const float *Cs = nullptr, *csn = nullptr, *css = nullptr;
    const void *Csq = nullptr;
    int first_part = 0, nparts = 0;
};

struct BatchPart {
    int job;
    int64_t i0, mb;
    bool direct;    // the threshold sample is the whole corpus: its selection is the candidate list
    bool grouped;   // FILTER product in the grouped launch (else its own: FP32 with d % 4 != 0)
    bool sgrouped;  // sample product in the grouped launch (same condition)
    float *Ds = nullptr;   // mb x S sample distances
    float *tv = nullptr;   // mb x (r + 1) selected sample keys (values, indices)
    int32_t *ti = nullptr;
    uint32_t *cnt = nullptr;
    uint64_t *cand = nullptr;
    int32_t *flags = nullptr;
    float *sv = nullptr;   // mb x kk selected candidates
    int32_t *si = nullptr;
    int32_t *ulist = nullptr;  // FP32: uncertified rows, re-run exactly
    float *tfix = nullptr;
};

// A multi-matrix selection launch: its segments and the segment of each row.
struct SegLaunch {
    int cap = 0;
    int64_t rows = 0;
    uint32_t cols = 0, k = 0;
    std::vector<SelectSeg> segs;
    std::vector<uint32_t> row_seg;
    SelectSeg *dsegs = nullptr;
    uint32_t *drow_seg = nullptr;
};

// Buffers shared by all jobs; every use of one is ordered on the stream.
struct BatchShared {
    float *Qf = nullptr, *Df = nullptr, *fv = nullptr, *qfs = nullptr;
    void *Qfq = nullptr;
    int32_t *fi = nullptr;
    void *selws = nullptr;
    float *ninf = nullptr;
    uint32_t *cnt_all = nullptr;  // the candidate counts of all parts, contiguous
    int64_t cnt_rows = 0;
    DistArgs *table = nullptr, *probe = nullptr, *stable = nullptr;
    GemmItem *items = nullptr, *sitems = nullptr;
    uint32_t *nflag = nullptr;
    uint32_t *nu = nullptr;  // uncertified-row counts, one per part
    uint32_t *queues = nullptr;  // the eight per-XCD item queues of the persistent product
};

// State of the last batch of a handle: its workspace, plan and graphs.
struct BatchState {
    std::vector<uint8_t> key;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t *nflag_host = nullptr;  // pinned: per part the flagged-row count, then the uncertified-row count
    size_t nflag_host_cap = 0;
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraphExec_t> graphs;  // in launch order, see the segments
    bool eager = true;                   // replay eagerly (no graphs)
    bool timed = false;
    std::vector<BatchJob> jobs;
    std::vector<BatchPart> parts;
    std::vector<int> order;  // jobs, longest first
    BatchShared sh;
    int tile = kTileWide;
    bool queue = false;  // the product as a resident grid over per-XCD item queues
    size_t nitems = 0, nsitems = 0;
    std::vector<SegLaunch> sample_sel;  // threshold selections, one launch per capacity class
    SegLaunch keys_sel;                 // candidate selections
    int smode = kPivotSample;
    const uint16_t *net = nullptr;
    int force = 0;

    void drop_graphs() {
        for (hipGraphExec_t g : graphs) hipGraphExecDestroy(g);
        graphs.clear();
    }
    ~BatchState() {
        drop_graphs();
        if (cap_stream) hipStreamDestroy(cap_stream);
        if (ws) hipFree(ws);
        if (nflag_host) hipHostFree(nflag_host);
    }
};

void batch_release(knn_handle_t h) {
    delete h->batch;
    h->batch = nullptr;
}

namespace {

// Items of the grouped launch for a tile shape, in dispatch order.  Eight
// queues, one per XCD, each holding the parts longest first; a part's column
// tiles are split into eight contiguous chunks (chunk q to queue q), each
// column tile followed by all of the part's row tiles (which then find it in
// their XCD's L2).  Workgroup b runs on XCD b % 8 and takes the next item of
// that queue; once a queue is empty its XCD takes items from the back of the
// fullest remaining queue (the shortest work there).
// Autotune candidates: a tile shape, plus this for the queue form.
constexpr int kQueueChoice = 16;

void build_items(const BatchState &b, int tile, std::vector<GemmItem> &items) {
    constexpr int kQueues = 8;
    int bm, bn;
    gemm_tile_dims(tile, &bm, &bn);
    std::vector<std::vector<GemmItem>> q(kQueues);
    for (int j : b.order) {
        const BatchJob &js = b.jobs[j];
        for (int pi = js.first_part; pi < js.first_part + js.nparts; ++pi) {
            const BatchPart &pt = b.parts[pi];
            if (!pt.grouped) continue;
            const uint32_t tm_n = (uint32_t)((pt.mb + bm - 1) / bm);
            const uint32_t tn_n = (uint32_t)((js.n + bn - 1) / bn);
            for (int qi = 0; qi < kQueues; ++qi) {
                const uint32_t c0 = (uint32_t)((uint64_t)tn_n * qi / kQueues);
                const uint32_t c1 = (uint32_t)((uint64_t)tn_n * (qi + 1) / kQueues);
                for (uint32_t tn = c0; tn < c1; ++tn)
                    for (uint32_t tm = 0; tm < tm_n; ++tm) q[qi].push_back(GemmItem{(uint32_t)pi, tm, tn});
            }
        }
    }
    size_t total = 0;
    for (const auto &x : q) total += x.size();
    items.clear();
    items.reserve(total);
    std::vector<size_t> head(kQueues, 0), tail(kQueues);
    for (int qi = 0; qi < kQueues; ++qi) tail[qi] = q[qi].size();
    for (size_t t = 0; t < total; ++t) {
        const int qi = (int)(t % kQueues);
        if (head[qi] < tail[qi]) {
            items.push_back(q[qi][head[qi]++]);
            continue;
        }
        int best = -1;
        for (int o = 0; o < kQueues; ++o)
            if (head[o] < tail[o] && (best < 0 || tail[o] - head[o] > tail[best] - head[best])) best = o;
        items.push_back(q[best][--tail[best]]);
    }
}

size_t max_items(const BatchState &b) {
    // the 128 x 128 tile gives the most items
    size_t n = 0;
    for (const BatchPart &pt : b.parts)
        if (pt.grouped) n += (size_t)((pt.mb + 127) / 128) * (size_t)((b.jobs[pt.job].n + 127) / 128);
    return n;
}

// Items of the grouped sample products (128 x 128 tiles), part after part.
void build_sample_items(const BatchState &b, std::vector<GemmItem> &items) {
    items.clear();
    for (size_t pi = 0; pi < b.parts.size(); ++pi) {
        const BatchPart &pt = b.parts[pi];
        if (!pt.sgrouped) continue;
        const uint32_t tm_n = (uint32_t)((pt.mb + 127) / 128), tn_n = (uint32_t)((b.jobs[pt.job].p.S + 127) / 128);
        for (uint32_t tm = 0; tm < tm_n; ++tm)
            for (uint32_t tn = 0; tn < tn_n; ++tn) items.push_back(GemmItem{(uint32_t)pi, tm, tn});
    }
}

// The threshold selections of all parts (k = r + 1 over their S sample
// distances), one launch per capacity class, and the candidate selections of
// the filtered parts (k = kk over their candidate lists), one launch.
void plan_selects(BatchState &b) {
    b.sample_sel.clear();
    // a sample row that fits the on-chip capacity is selected there directly
    // (no pivot sample, no streaming), so short rows go to the class that holds them
    auto sample_cap = [](const Plan &p) {
        int c = select_cap_for_k((uint32_t)(p.r + 1));
        if (p.S > c && p.S <= kSelectKeysCap) c = p.S <= 2048 ? 2048 : 4096;
        return c;
    };
    for (int cap : {1024, 2048, 4096}) {
        SegLaunch L;
        L.cap = cap;
        for (const BatchPart &pt : b.parts) {
            const Plan &p = b.jobs[pt.job].p;
            if (sample_cap(p) != cap) continue;
            SelectSeg sg{};
            sg.dist = pt.Ds;
            sg.ld = p.S;
            sg.row0 = L.rows;
            sg.cols = (uint32_t)p.S;
            sg.k = (uint32_t)(p.r + 1);
            sg.out_val = pt.tv;
            sg.out_idx = pt.ti;
            L.cols = std::max(L.cols, sg.cols);
            L.k = std::max(L.k, sg.k);
            for (int64_t i = 0; i < pt.mb; ++i) L.row_seg.push_back((uint32_t)L.segs.size());
            L.segs.push_back(sg);
            L.rows += pt.mb;
        }
        if (L.rows) b.sample_sel.push_back(std::move(L));
    }
    SegLaunch K;
    K.cap = kSelectKeysCap;
    for (const BatchPart &pt : b.parts) {
        if (pt.direct) continue;
        const Plan &p = b.jobs[pt.job].p;
        SelectSeg sg{};
        sg.keys = pt.cand;
        sg.key_cnt = pt.cnt;
        sg.ld = p.cap;
        sg.row0 = K.rows;
        sg.cols = (uint32_t)p.cap;
        sg.k = (uint32_t)p.kk;
        sg.out_val = pt.sv;
        sg.out_idx = pt.si;
        K.cols = std::max(K.cols, sg.cols);
        K.k = std::max(K.k, sg.k);
        for (int64_t i = 0; i < pt.mb; ++i) K.row_seg.push_back((uint32_t)K.segs.size());
        K.segs.push_back(sg);
        K.rows += pt.mb;
    }
    b.keys_sel = std::move(K);
}

// Lays out the batch workspace (sizing pass with base == nullptr).  Every
// part keeps its own sample distances, selections and candidate lists, so
// each phase can run as one launch over all parts.
size_t carve_batch(Carve &c, BatchState &b, int num_cu, bool probe) {
    BatchShared &s = b.sh;
    size_t qf = 0, df = 0, fv = 0, qfq = 0, fb = 0, selws = 0;
    for (BatchJob &js : b.jobs) {
        const Plan &p = js.p;
        js.cnorm = c.take<float>(js.n);
        js.qn2 = c.take<float>(js.m);
        js.cmax2 = c.take<unsigned int>(1);
        if (p.prec != kPrecF32) {
            js.Cq = c.take<char>((size_t)js.n * p.ldq);
            js.cs = c.take<float>(js.n);
            if (!js.graph) {
                js.Qq = c.take<char>((size_t)js.m * p.ldq);
                js.qs = c.take<float>(js.m);
            } else {
                js.Qq = js.Cq;
                js.qs = js.cs;
            }
        }
        js.Cs = js.C;
        js.csn = js.cnorm;
        js.Csq = js.Cq;
        js.css = js.cs;
        if (p.gathered && js.nparts) {
            js.Cs = c.take<float>((size_t)p.S * p.d);
            js.csn = c.take<float>(p.S);
            if (p.prec != kPrecF32) {
                js.Csq = c.take<char>((size_t)p.S * p.ldq);
                js.css = c.take<float>(p.S);
            }
        }
        qf = std::max(qf, (size_t)p.Fb * p.d);
        df = std::max(df, (size_t)p.Fb * js.n);
        fv = std::max(fv, (size_t)p.Fb * p.kk);
        qfq = std::max(qfq, (size_t)p.Fb * p.ldq);
        fb = std::max(fb, (size_t)p.Fb);
        const int cap2 = select_cap_for_k(p.kk);
        selws = std::max(selws, select_ws_bytes(cap2, (uint32_t)js.n, select_grid(cap2, p.Fb, num_cu)));
    }
    int64_t cnt_rows = 0;
    for (const BatchPart &pt : b.parts)
        if (!pt.direct) cnt_rows += pt.mb;
    s.cnt_all = c.take<uint32_t>((size_t)std::max<int64_t>(cnt_rows, 1));
    s.cnt_rows = cnt_rows;
    int64_t cnt_off = 0;
    for (BatchPart &pt : b.parts) {
        const Plan &p = b.jobs[pt.job].p;
        pt.Ds = c.take<float>((size_t)pt.mb * p.S);
        pt.tv = c.take<float>((size_t)pt.mb * (p.r + 1));
        pt.ti = c.take<int32_t>((size_t)pt.mb * (p.r + 1));
        if (pt.direct) continue;
        pt.cnt = s.cnt_all ? s.cnt_all + cnt_off : nullptr;
        cnt_off += pt.mb;
        pt.cand = c.take<uint64_t>((size_t)pt.mb * p.cap);
        pt.flags = c.take<int32_t>(pt.mb);
        pt.sv = c.take<float>((size_t)pt.mb * p.kk);
        pt.si = c.take<int32_t>((size_t)pt.mb * p.kk);
    }
    for (BatchPart &pt : b.parts) {
        if (b.jobs[pt.job].p.prec != kPrecF32) continue;
        pt.ulist = c.take<int32_t>((size_t)pt.mb);
        pt.tfix = c.take<float>((size_t)pt.mb);
    }
    plan_selects(b);
    for (SegLaunch &L : b.sample_sel) {
        selws = std::max(selws, select_ws_bytes(L.cap, L.cols, select_grid(L.cap, L.rows, num_cu)));
        L.dsegs = c.take<SelectSeg>(L.segs.size());
        L.drow_seg = c.take<uint32_t>((size_t)L.rows);
    }
    b.keys_sel.dsegs = c.take<SelectSeg>(std::max<size_t>(b.keys_sel.segs.size(), 1));
    b.keys_sel.drow_seg = c.take<uint32_t>((size_t)std::max<int64_t>(b.keys_sel.rows, 1));
    s.Qf = c.take<float>(qf);
    s.Df = c.take<float>(df);
    s.fv = c.take<float>(fv);
    s.fi = c.take<int32_t>(fv);
    s.Qfq = c.take<char>(qfq);
    s.qfs = c.take<float>(fb);
    s.selws = c.take<char>(selws < 256 ? 256 : selws);
    s.ninf = c.take<float>(1);
    s.table = c.take<DistArgs>(b.parts.size());
    s.stable = c.take<DistArgs>(b.parts.size());
    s.probe = probe ? c.take<DistArgs>(b.parts.size()) : nullptr;
    s.items = c.take<GemmItem>(std::max<size_t>(max_items(b), 1));
    std::vector<GemmItem> si;
    build_sample_items(b, si);
    s.sitems = c.take<GemmItem>(std::max<size_t>(si.size(), 1));
    b.nsitems = si.size();
    s.nflag = c.take<uint32_t>(b.parts.size());
    s.nu = c.take<uint32_t>(b.parts.size());
    s.queues = c.take<uint32_t>(8);
    return c.off;
}

DistArgs part_args(const BatchState &b, const BatchPart &pt) {
    const BatchJob &js = b.jobs[pt.job];
    const Plan &p = js.p;
    DistArgs a{};
    a.Q = js.Q + pt.i0 * js.d;
    a.m = pt.mb;
    a.C = js.C;
    a.n = js.n;
    a.d = js.d;
    a.cnorm = js.cnorm;
    a.self_offset = js.graph ? pt.i0 : -1;
    a.tau = pt.tv ? pt.tv + p.r : nullptr;  // the threshold is the last selected sample key
    a.tau_stride = p.r + 1;
    a.cnt = pt.cnt;
    a.cand = pt.cand;
    a.cap = p.cap;
    a.prec = p.prec;
    a.Qq = js.Qq ? static_cast<const char *>(js.Qq) + pt.i0 * p.ldq : nullptr;
    a.Cq = js.Cq;
    a.ldq = p.ldq;
    a.qscale = js.qs ? js.qs + pt.i0 : nullptr;
    a.cscale = js.cs;
    return a;
}

// The sample product of a part: its rows against the job's threshold sample.
DistArgs sample_args(const BatchState &b, const BatchPart &pt) {
    const BatchJob &js = b.jobs[pt.job];
    const Plan &p = js.p;
    DistArgs sa = part_args(b, pt);
    sa.C = js.Cs;
    sa.n = p.S;
    sa.cnorm = js.csn;
    sa.self_offset = (js.graph && !p.gathered) ? pt.i0 : -1;
    sa.out = pt.Ds;
    sa.ldo = p.S;
    sa.tau = nullptr;
    sa.cnt = nullptr;
    sa.cand = nullptr;
    sa.Cq = js.Csq;
    sa.cscale = js.css;
    return sa;
}

SelectArgs seg_select_args(const BatchState &b, const SegLaunch &L) {
    SelectArgs a{};
    a.rows = L.rows;
    a.cols = L.cols;
    a.k = L.k;
    a.mode = b.smode;
    a.net = b.smode == kPivotLearned ? b.net : nullptr;
    a.segs = L.dsegs;
    a.row_seg = L.drow_seg;
    return a;
}

// Certificate of a part's kk candidates (FP32: uncertified rows are listed for
// the exact re-run), then the exact re-rank.
hipError_t certify_rerank(const BatchState &b, knn_handle_t h, size_t pi, const float *keys, const int32_t *cidx,
                          hipStream_t s) {
    const BatchPart &pt = b.parts[pi];
    const BatchJob &js = b.jobs[pt.job];
    const Plan &p = js.p;
    hipError_t e = hipSuccess;
    if (p.kk < p.n_eff) {
        CertifyArgs ca{keys, pt.mb, p.kk, js.k, js.qn2 + pt.i0, js.cmax2, p.rel, p.gamma,
                       stats_ptr(h) + kStatUncertified, pt.ulist, b.sh.nu + pi, pt.tfix,
                       pt.ulist != nullptr && p.force_rerun};
        if ((e = launch_certify(ca, s)) != hipSuccess) return e;
    }
    RerankArgs rr{js.Q + pt.i0 * js.d, pt.mb, js.C, js.n, js.d, cidx, (uint32_t)p.kk, js.k,
                  js.out_dist + pt.i0 * js.k, js.out_idx + pt.i0 * js.k, js.graph ? pt.i0 : -1, js.oscale};
    return launch_rerank(rr, s);
}

// ---- the phases, enqueued on a stream (captured or eager) ------------------
hipError_t enqueue_prep(const BatchState &b, knn_handle_t h, int num_cu, hipStream_t s) {
    hipError_t e = hipSuccess;
    const BatchShared &sh = b.sh;
#define BTRY(call)                                 \
    do {                                           \
        if ((e = (call)) != hipSuccess) return e;  \
    } while (0)
    BTRY(launch_fill_u32(sh.nu, (int64_t)b.parts.size(), 0u, s));
    // per job: norms, quantised copies, the gathered threshold sample
    for (int j : b.order) {
        const BatchJob &js = b.jobs[j];
        const Plan &p = js.p;
        if (js.nparts == 0) continue;
        BTRY(launch_fill_u32(js.cmax2, 1, 0u, s));
        BTRY(launch_sqnorm(js.C, js.n, js.d, js.cnorm, js.cmax2, s));
        BTRY(launch_sqnorm(js.Q, js.m, js.d, js.qn2, nullptr, s));
        if (p.prec != kPrecF32) {
            BTRY(launch_quantize(js.C, js.n, js.d, p.prec, js.Cq, js.cs, s));
            if (!js.graph) BTRY(launch_quantize(js.Q, js.m, js.d, p.prec, js.Qq, js.qs, s));
        }
        if (p.gathered) {
            float *Cs = const_cast<float *>(js.Cs), *csn = const_cast<float *>(js.csn);
            BTRY(launch_gather_rows(js.C, js.n, js.d, nullptr, p.S, Cs, js.cnorm, csn, s));
            if (p.prec != kPrecF32)
                BTRY(launch_quantize(Cs, p.S, js.d, p.prec, const_cast<void *>(js.Csq), const_cast<float *>(js.css),
                                     s));
        }
    }
    // all sample products in one launch (FP32 parts with d % 4 != 0 on their own)
    BTRY(launch_dist_gemm_grouped(sh.stable, sh.sitems, (int64_t)b.nsitems, b.jobs[0].p.prec, kTileSmall, s,
                                  kEpiDense));
    for (const BatchPart &pt : b.parts)
        if (!pt.sgrouped) BTRY(launch_dist_gemm(sample_args(b, pt), kEpiDense, s));
    // all threshold selections, one launch per capacity class
    for (const SegLaunch &L : b.sample_sel) {
        SelectArgs sa = seg_select_args(b, L);
        BTRY(launch_select(sa, L.cap, select_grid(L.cap, L.rows, num_cu), sh.selws, s));
    }
    // parts whose sample is the whole corpus: certificate and re-rank now
    for (size_t pi = 0; pi < b.parts.size(); ++pi)
        if (b.parts[pi].direct) BTRY(certify_rerank(b, h, pi, b.parts[pi].tv, b.parts[pi].ti, s));
    if (sh.cnt_rows) BTRY(launch_fill_u32(sh.cnt_all, sh.cnt_rows, 0u, s));
    return e;
}

hipError_t enqueue_product(const BatchState &b, const DistArgs *table, int tile, bool queue, int num_cu,
                           hipStream_t s) {
    hipError_t e = hipSuccess;
    if (queue)
        BTRY(launch_dist_gemm_queue(table, b.sh.items, (int64_t)b.nitems, b.jobs[0].p.prec, tile, b.sh.queues, num_cu,
                                    s));
    else
        BTRY(launch_dist_gemm_grouped(table, b.sh.items, (int64_t)b.nitems, b.jobs[0].p.prec, tile, s));
    for (const BatchPart &pt : b.parts) {
        if (pt.grouped || pt.direct) continue;
        DistArgs fa = part_args(b, pt);
        if (table == b.sh.probe) {
            fa.tau = b.sh.ninf;
            fa.tau_stride = 0;
        }
        BTRY(launch_dist_gemm(fa, kEpiFilter, s));
    }
    return e;
}

hipError_t enqueue_flags(const BatchState &b, knn_handle_t h, hipStream_t s) {
    hipError_t e = hipSuccess;
    BTRY(launch_fill_u32(b.sh.nflag, (int64_t)b.parts.size(), 0u, s));
    if (b.sh.cnt_rows) BTRY(launch_sum_u32(b.sh.cnt_all, b.sh.cnt_rows, stats_ptr(h) + kStatCandidates, s));
    for (size_t pi = 0; pi < b.parts.size(); ++pi) {
        const BatchPart &pt = b.parts[pi];
        const Plan &p = b.jobs[pt.job].p;
        if (pt.direct) continue;
        BTRY(launch_flag_rows(pt.cnt, pt.mb, (uint32_t)p.kk, (uint32_t)p.cap, b.force, b.sh.nflag + pi, pt.flags, s));
    }
    return hipMemcpyAsync(b.nflag_host, b.sh.nflag, b.parts.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
}

hipError_t enqueue_final(const BatchState &b, knn_handle_t h, int num_cu, hipStream_t s) {
    hipError_t e = hipSuccess;
    // the kk smallest candidate keys of every filtered row, one launch
    if (b.keys_sel.rows) {
        SelectArgs ka = seg_select_args(b, b.keys_sel);
        BTRY(launch_select_keys(ka, b.sh.selws, ka.rows, num_cu, s));
    }
    for (size_t pi = 0; pi < b.parts.size(); ++pi)
        if (!b.parts[pi].direct) BTRY(certify_rerank(b, h, pi, b.parts[pi].sv, b.parts[pi].si, s));
    // the uncertified-row counts, for the exact re-run that follows
    return hipMemcpyAsync(b.nflag_host + b.parts.size(), b.sh.nu, b.parts.size() * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, s);
}

// After the flagged rows' candidate lists are re-done: the candidate selection,
// certificate and re-rank of one part again (its uncertified list restarts).
hipError_t refinal_part(const BatchState &b, knn_handle_t h, int num_cu, size_t pi, hipStream_t s) {
    hipError_t e = hipSuccess;
    const BatchPart &pt = b.parts[pi];
    const Plan &p = b.jobs[pt.job].p;
    BTRY(launch_fill_u32(b.sh.nu + pi, 1, 0u, s));
    SelectArgs ka{};
    ka.keys = pt.cand;
    ka.key_cnt = pt.cnt;
    ka.rows = pt.mb;
    ka.cols = (uint32_t)p.cap;
    ka.ld = p.cap;
    ka.k = (uint32_t)p.kk;
    ka.out_val = pt.sv;
    ka.out_idx = pt.si;
    ka.mode = b.smode;
    ka.net = b.smode == kPivotLearned ? b.net : nullptr;
    BTRY(launch_select_keys(ka, b.sh.selws, pt.mb, num_cu, s));
    BTRY(certify_rerank(b, h, pi, pt.sv, pt.si, s));
    return hipMemcpyAsync(b.nflag_host + b.parts.size() + pi, b.sh.nu + pi, sizeof(uint32_t), hipMemcpyDeviceToHost,
                          s);
}

// Exact re-do of the flagged rows of every part (after the flag counts reached
// the host), as in knn_search.
hipError_t run_fallback(const BatchState &b, int num_cu, hipStream_t s, int64_t *total) {
    hipError_t e = hipSuccess;
    const BatchShared &sh = b.sh;
    for (size_t pi = 0; pi < b.parts.size(); ++pi) {
        const int64_t nf = b.nflag_host[pi];
        if (nf == 0) continue;
        *total += nf;
        const BatchPart &pt = b.parts[pi];
        const BatchJob &js = b.jobs[pt.job];
        const Plan &p = js.p;
        const float *Qb = js.Q + pt.i0 * js.d;
        for (int64_t f0 = 0; f0 < nf; f0 += p.Fb) {
            const int64_t fb = nf - f0 < p.Fb ? nf - f0 : p.Fb;
            BTRY(launch_gather_rows(Qb, pt.mb, js.d, pt.flags + f0, fb, sh.Qf, nullptr, nullptr, s));
            if (p.prec != kPrecF32) BTRY(launch_quantize(sh.Qf, fb, js.d, p.prec, sh.Qfq, sh.qfs, s));
            DistArgs da{};
            da.Q = sh.Qf;
            da.m = fb;
            da.C = js.C;
            da.n = js.n;
            da.d = js.d;
            da.cnorm = js.cnorm;
            da.self_offset = js.graph ? pt.i0 : -1;
            da.row_ids = pt.flags + f0;
            da.out = sh.Df;
            da.ldo = js.n;
            da.prec = p.prec;
            da.Qq = sh.Qfq;
            da.Cq = js.Cq;
            da.ldq = p.ldq;
            da.qscale = sh.qfs;
            da.cscale = js.cs;
            BTRY(launch_dist_gemm(da, kEpiDense, s));
            BTRY(select_dense(sh.Df, fb, js.n, js.n, p.kk, sh.fv, sh.fi, sh.selws, num_cu, b.smode, b.net, s));
            BTRY(launch_scatter_fallback(pt.flags + f0, fb, sh.fv, sh.fi, p.kk, pt.cand, pt.cnt, p.cap, s));
        }
    }
    return e;
}
// Exact re-run of the uncertified FP32 rows of every part (after their counts
// reached the host): from the part's sample distances when the sample is the
// whole corpus, else from rows materialised here.
hipError_t run_rerun(const BatchState &b, hipStream_t s, int64_t *total) {
    hipError_t e = hipSuccess;
    const BatchShared &sh = b.sh;
    const uint32_t *counts = b.nflag_host + b.parts.size();
    for (size_t pi = 0; pi < b.parts.size(); ++pi) {
        const int64_t nu = counts[pi];
        if (nu == 0) continue;
        *total += nu;
        const BatchPart &pt = b.parts[pi];
        const BatchJob &js = b.jobs[pt.job];
        const Plan &p = js.p;
        const float *Qb = js.Q + pt.i0 * js.d;
        FixupArgs fx{};
        fx.out_scale = js.oscale;
        fx.tfix = pt.tfix;
        fx.Q = Qb;
        fx.C = js.C;
        fx.n = js.n;
        fx.d = js.d;
        fx.k = js.k;
        fx.self_offset = js.graph ? pt.i0 : -1;
        fx.out_dist = js.out_dist + pt.i0 * js.k;
        fx.out_idx = js.out_idx + pt.i0 * js.k;
        if (pt.direct) {
            fx.D = pt.Ds;
            fx.ldd = p.S;
            fx.by_row = true;
            fx.rows = pt.ulist;
            fx.nrows = nu;
            BTRY(launch_fixup(fx, s));
            continue;
        }
        for (int64_t f0 = 0; f0 < nu; f0 += p.Fb) {
            const int64_t fb = nu - f0 < p.Fb ? nu - f0 : p.Fb;
            BTRY(launch_gather_rows(Qb, pt.mb, js.d, pt.ulist + f0, fb, sh.Qf, nullptr, nullptr, s));
            DistArgs da{};
            da.Q = sh.Qf;
            da.m = fb;
            da.C = js.C;
            da.n = js.n;
            da.d = js.d;
            da.cnorm = js.cnorm;
            da.self_offset = js.graph ? pt.i0 : -1;
            da.row_ids = pt.ulist + f0;
            da.out = sh.Df;
            da.ldo = js.n;
            BTRY(launch_dist_gemm(da, kEpiDense, s));
            fx.D = sh.Df;
            fx.ldd = js.n;
            fx.by_row = false;
            fx.rows = pt.ulist + f0;
            fx.nrows = fb;
            BTRY(launch_fixup(fx, s));
        }
    }
    return e;
}
#undef BTRY

// Captures `fn` enqueued on the state's capture stream into an executable graph.
hipError_t capture(BatchState &b, const std::function<hipError_t(hipStream_t)> &fn, hipGraphExec_t *out) {
    *out = nullptr;
    hipError_t e = hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    hipError_t fe = fn(b.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b.cap_stream, &g);
    if (fe != hipSuccess) e = fe;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
    }
    return e;
}

std::vector<uint8_t> make_key(const knn_job_t *jobs, int32_t njobs, const knn_options_t &o, int smode,
                              const uint16_t *net, const void *ws) {
    std::vector<uint8_t> k(sizeof(knn_job_t) * (size_t)njobs + sizeof(o) + sizeof(smode) + 2 * sizeof(void *));
    uint8_t *p = k.data();
    std::memcpy(p, jobs, sizeof(knn_job_t) * (size_t)njobs);
    p += sizeof(knn_job_t) * (size_t)njobs;
    std::memcpy(p, &o, sizeof(o));
    p += sizeof(o);
    std::memcpy(p, &smode, sizeof(smode));
    p += sizeof(smode);
    std::memcpy(p, &net, sizeof(void *));
    p += sizeof(void *);
    std::memcpy(p, &ws, sizeof(void *));
    return k;
}

}  // namespace

knn_status_t run_batch(knn_handle_t h, const knn_job_t *jobs, int32_t njobs, hipStream_t stream,
                       const knn_options_t *opt_in) {
    knn_options_t o{};
    o.pivot = kPivotSample;
    if (opt_in) o = *opt_in;
    const int num_cu = handle_num_cu(h);
    const uint16_t *net = handle_net(h);
    int smode = o.pivot;
    if (smode == kPivotLearned && !net) smode = kPivotSample;

    hipError_t e;
#define KTRY(call)                                                                                       \
    do {                                                                                                 \
        if ((e = (call)) != hipSuccess)                                                                  \
            return fail_msg(h, KNN_ERROR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e));     \
    } while (0)

    if (o.flags & KNN_FLAG_UNFUSED) {  // one job after the other, as knn_search
        for (int32_t j = 0; j < njobs; ++j) {
            const knn_job_t &jb = jobs[j];
            if (jb.m == 0) continue;
            const bool graph = jb.queries == nullptr;  // m > 0 here
            knn_status_t st = run_search(h, graph ? jb.corpus : jb.queries, jb.m, jb.corpus, jb.n, jb.d, jb.k, graph,
                                         jb.out_dist, jb.out_idx, stream, &o);
            if (st != KNN_SUCCESS) return st;
        }
        return KNN_SUCCESS;
    }

    // cosine / Pearson: every job on unit vectors (centred for Pearson), made
    // on each call before the captured steps run
    std::vector<knn_job_t> unit_jobs;
    if (o.metric != KNN_METRIC_SQEUCLIDEAN) {
        size_t total = 0;
        for (int32_t j = 0; j < njobs; ++j)
            if (jobs[j].m > 0) total += (size_t)(jobs[j].n + (jobs[j].queries ? jobs[j].m : 0)) * (size_t)jobs[j].d;
        void *u = nullptr;
        knn_status_t us = ensure_unit_ws(h, total * sizeof(float) + 256, stream, &u);
        if (us != KNN_SUCCESS) return us;
        float *U = static_cast<float *>(u);
        const bool centre = o.metric == KNN_METRIC_PEARSON;
        unit_jobs.assign(jobs, jobs + njobs);
        size_t off = 0;
        for (int32_t j = 0; j < njobs; ++j) {
            knn_job_t &jb = unit_jobs[(size_t)j];
            if (jb.m == 0) continue;
            KTRY(launch_unit_rows(jb.corpus, jb.n, jb.d, centre, U + off, stream));
            jb.corpus = U + off;
            off += (size_t)jb.n * jb.d;
            if (jb.queries) {
                KTRY(launch_unit_rows(jb.queries, jb.m, jb.d, centre, U + off, stream));
                jb.queries = U + off;
                off += (size_t)jb.m * jb.d;
            }
        }
        jobs = unit_jobs.data();
    }

    if (!h->batch) h->batch = new BatchState();
    BatchState &b = *h->batch;
    std::vector<uint8_t> key = make_key(jobs, njobs, o, smode, net, b.ws);
    const bool timed = (o.flags & KNN_FLAG_TIMING) != 0;
    const bool want_graph = (o.flags & KNN_FLAG_NO_GRAPH) == 0;

    if (key != b.key || b.ws == nullptr) {
        // ---- plan the batch ----
        KTRY(hipDeviceSynchronize());  // earlier batches may still use the graphs and workspace
        b.drop_graphs();
        b.key.clear();
        b.jobs.clear();
        b.parts.clear();
        b.smode = smode;
        b.net = net;
        b.force = (o.flags & KNN_FLAG_FORCE_FALLBACK) ? 1 : 0;
        b.timed = timed;
        for (int32_t j = 0; j < njobs; ++j) {
            const knn_job_t &jb = jobs[j];
            BatchJob js{};
            js.graph = jb.queries == nullptr && jb.m > 0;
            js.Q = js.graph ? jb.corpus : jb.queries;
            js.C = jb.corpus;
            js.m = jb.m;
            js.n = jb.n;
            js.d = jb.d;
            js.k = jb.k;
            js.out_dist = jb.out_dist;
            js.out_idx = jb.out_idx;
            js.p = make_plan(jb.m > 0 ? jb.m : 1, jb.n, jb.d, jb.k, js.graph, &o, kRowBlock);
            js.cost = 2.0 * (double)jb.m * (double)jb.n * jb.d;
            js.oscale = o.metric != KNN_METRIC_SQEUCLIDEAN ? 0.5f : 1.0f;
            js.first_part = (int)b.parts.size();
            for (int64_t i0 = 0; i0 < jb.m; i0 += js.p.Mb) {
                BatchPart pt{};
                pt.job = j;
                pt.i0 = i0;
                pt.mb = jb.m - i0 < js.p.Mb ? jb.m - i0 : js.p.Mb;
                pt.direct = !js.p.gathered;
                pt.sgrouped = !(js.p.prec == kPrecF32 && js.d % 4 != 0);
                pt.grouped = !pt.direct && pt.sgrouped;
                b.parts.push_back(pt);
            }
            js.nparts = (int)b.parts.size() - js.first_part;
            b.jobs.push_back(js);
        }
        b.order.resize(b.jobs.size());
        for (size_t j = 0; j < b.jobs.size(); ++j) b.order[j] = (int)j;
        std::stable_sort(b.order.begin(), b.order.end(),
                         [&](int x, int y) { return b.jobs[x].cost > b.jobs[y].cost; });
        if (b.parts.empty()) return KNN_SUCCESS;

        const bool tune = autotune_enabled(&o);
        Carve sizing{nullptr};
        const size_t bytes = carve_batch(sizing, b, num_cu, tune);
        if (bytes > b.ws_bytes) {
            if (b.ws) {
                hipFree(b.ws);
                b.ws = nullptr;
                b.ws_bytes = 0;
            }
            if (hipMalloc(&b.ws, bytes) != hipSuccess) {
                b.ws = nullptr;
                (void)hipGetLastError();
                return fail_msg(h, KNN_ERROR_OUT_OF_MEMORY,
                                "knn_batch_search: workspace of " + std::to_string(bytes) + " bytes");
            }
            b.ws_bytes = bytes;
        }
        Carve real{static_cast<char *>(b.ws)};
        carve_batch(real, b, num_cu, tune);
        if (b.parts.size() > b.nflag_host_cap) {
            if (b.nflag_host) hipHostFree(b.nflag_host);
            b.nflag_host = nullptr;
            b.nflag_host_cap = 0;
            if (hipHostMalloc(&b.nflag_host, 2 * b.parts.size() * sizeof(uint32_t), hipHostMallocDefault) !=
                hipSuccess) {
                b.nflag_host = nullptr;
                (void)hipGetLastError();
                return fail_msg(h, KNN_ERROR_OUT_OF_MEMORY, "knn_batch_search: pinned host buffer");
            }
            b.nflag_host_cap = b.parts.size();
        }
        if (!b.cap_stream) KTRY(hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking));

        // ---- device tables ----
        std::vector<DistArgs> table(b.parts.size());
        for (size_t pi = 0; pi < b.parts.size(); ++pi) table[pi] = part_args(b, b.parts[pi]);
        KTRY(hipMemcpyAsync(b.sh.table, table.data(), table.size() * sizeof(DistArgs), hipMemcpyHostToDevice, stream));
        std::vector<DistArgs> stable(b.parts.size());
        for (size_t pi = 0; pi < b.parts.size(); ++pi) stable[pi] = sample_args(b, b.parts[pi]);
        KTRY(hipMemcpyAsync(b.sh.stable, stable.data(), stable.size() * sizeof(DistArgs), hipMemcpyHostToDevice,
                            stream));
        std::vector<GemmItem> sitems;
        build_sample_items(b, sitems);
        if (!sitems.empty())
            KTRY(hipMemcpyAsync(b.sh.sitems, sitems.data(), sitems.size() * sizeof(GemmItem), hipMemcpyHostToDevice,
                                stream));
        std::vector<SegLaunch *> launches;
        for (SegLaunch &L : b.sample_sel) launches.push_back(&L);
        launches.push_back(&b.keys_sel);
        for (SegLaunch *L : launches) {
            if (!L->rows) continue;
            KTRY(hipMemcpyAsync(L->dsegs, L->segs.data(), L->segs.size() * sizeof(SelectSeg), hipMemcpyHostToDevice,
                                stream));
            KTRY(hipMemcpyAsync(L->drow_seg, L->row_seg.data(), L->row_seg.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, stream));
        }
        KTRY(hipStreamSynchronize(stream));  // the host vectors above are released at scope end
        KTRY(launch_fill_u32(reinterpret_cast<uint32_t *>(b.sh.ninf), 1, 0xFF800000u, stream));
        const int prec = b.jobs[0].p.prec;
        b.tile = kTileSmall1;
        b.queue = false;
        // overrides of the default form (tests, measurements): KNN_GEMM_TILE
        // small / wide / big / small1, KNN_BATCH_QUEUE 1 / 0 (the queue form has
        // no single-stage tile: small1 runs as small there)
        if (const char *te = std::getenv("KNN_GEMM_TILE")) {
            if (!std::strcmp(te, "small1")) b.tile = kTileSmall1;
            else if (!std::strcmp(te, "small")) b.tile = kTileSmall;
            else if (!std::strcmp(te, "wide")) b.tile = kTileWide;
            else if (!std::strcmp(te, "big") && prec != kPrecFP8) b.tile = kTileBig;
        }
        if (const char *qe = std::getenv("KNN_BATCH_QUEUE")) b.queue = qe[0] == '1';
        std::vector<GemmItem> items;
        int uploaded = -1;
        auto upload = [&](int tile) -> hipError_t {
            if (tile == uploaded) return hipSuccess;
            build_items(b, tile, items);
            b.nitems = items.size();
            hipError_t ue = hipSuccess;
            if (!items.empty())
                ue = hipMemcpyAsync(b.sh.items, items.data(), items.size() * sizeof(GemmItem), hipMemcpyHostToDevice,
                                    stream);
            if (ue == hipSuccess) ue = hipStreamSynchronize(stream);  // host vectors change on the next upload
            if (ue == hipSuccess) uploaded = tile;
            return ue;
        };
        if (tune) {
            // key: device, precision, work-weighted dimension and corpus size, total work
            double w = 0, wd = 0, wn = 0;
            for (const BatchJob &js : b.jobs) {
                w += js.cost;
                wd += js.cost * js.d;
                wn += js.cost * (double)js.n;
            }
            w = w > 0 ? w : 1;
            const std::string tkey = "grouped|" + h->arch + "|cu" + std::to_string(num_cu) + "|p" +
                                     std::to_string(prec) + "|d" + std::to_string(size_bucket((int64_t)(wd / w))) +
                                     "|n" + std::to_string(size_bucket((int64_t)(wn / w))) + "|f" +
                                     std::to_string(size_bucket((int64_t)(w / 1e6)));
            int choice = autotune_lookup(tkey);
            if (choice < 0) {
                std::vector<DistArgs> probe = table;
                for (DistArgs &a : probe) {
                    a.tau = b.sh.ninf;
                    a.tau_stride = 0;
                }
                KTRY(hipMemcpyAsync(b.sh.probe, probe.data(), probe.size() * sizeof(DistArgs), hipMemcpyHostToDevice,
                                    stream));
                KTRY(hipStreamSynchronize(stream));
                // every tile shape, as one workgroup per item (c) and as a
                // resident grid over the per-XCD queues (c + kQueueChoice)
                // the default (single-stage 128 x 128, one workgroup per item)
                // first, kept unless another form is more than 3 % faster: the
                // probes keep nothing (threshold -inf), and the candidate writes
                // they leave out favour the default's more resident workgroups
                // per CU (512-job batch: probes tied, real calls 4 % faster)
                std::vector<int> cands = {kTileSmall1, kTileSmall, kTileWide};
                if (prec != kPrecFP8) cands.push_back(kTileBig);
                const size_t nshape = cands.size();
                for (size_t i = 1; i < nshape; ++i) cands.push_back(cands[i] + kQueueChoice);
                auto run = [&](int c) -> hipError_t {
                    const int tile = c % kQueueChoice;
                    hipError_t re = upload(tile);
                    if (re == hipSuccess) re = enqueue_product(b, b.sh.probe, tile, c >= kQueueChoice, num_cu, stream);
                    return re;
                };
                KTRY(autotune_pick(tkey, cands, run, stream, 2, &choice, 0.03f));
            }
            b.tile = choice % kQueueChoice;
            b.queue = choice >= kQueueChoice;
        }
        KTRY(upload(b.tile));

        // ---- graphs: prep (+ product + flags), then final ----
        b.eager = true;
        if (want_graph) {
            std::vector<hipGraphExec_t> gs;
            hipGraphExec_t g = nullptr;
            bool ok = true;
            // one graph for the whole call (two around the timed product); rows
            // flagged for the exact fallback come out of it with provisional
            // results, re-done eagerly afterwards
            if (timed) {
                ok = capture(b, [&](hipStream_t s) { return enqueue_prep(b, h, num_cu, s); }, &g) == hipSuccess;
                if (ok) gs.push_back(g);
                ok = ok && capture(b, [&](hipStream_t s) {
                               hipError_t ce = enqueue_flags(b, h, s);
                               if (ce == hipSuccess) ce = enqueue_final(b, h, num_cu, s);
                               return ce;
                           }, &g) == hipSuccess;
                if (ok) gs.push_back(g);
            } else {
                ok = capture(b, [&](hipStream_t s) {
                         hipError_t ce = enqueue_prep(b, h, num_cu, s);
                         if (ce == hipSuccess) ce = enqueue_product(b, b.sh.table, b.tile, b.queue, num_cu, s);
                         if (ce == hipSuccess) ce = enqueue_flags(b, h, s);
                         if (ce == hipSuccess) ce = enqueue_final(b, h, num_cu, s);
                         return ce;
                     }, &g) == hipSuccess;
                if (ok) gs.push_back(g);
            }
            if (ok) {
                b.graphs = gs;
                b.eager = false;
            } else {
                for (hipGraphExec_t x : gs) hipGraphExecDestroy(x);  // capture failed: eager steps
            }
        }
        b.key = make_key(jobs, njobs, o, smode, net, b.ws);
    }

    // ---- run ----
    int64_t rows = 0;
    for (const BatchJob &js : b.jobs) rows += js.m;
    ProductTimer timer;
    KTRY(timer.init(timed));
    double flops = 0;
    for (const BatchJob &js : b.jobs) flops += js.cost;
    if (b.eager) {
        KTRY(enqueue_prep(b, h, num_cu, stream));
        KTRY(timer.begin(stream, flops));
        KTRY(enqueue_product(b, b.sh.table, b.tile, b.queue, num_cu, stream));
        KTRY(timer.end(stream));
        KTRY(enqueue_flags(b, h, stream));
        KTRY(enqueue_final(b, h, num_cu, stream));
    } else if (timed) {
        KTRY(hipGraphLaunch(b.graphs[0], stream));
        KTRY(timer.begin(stream, flops));
        KTRY(enqueue_product(b, b.sh.table, b.tile, b.queue, num_cu, stream));
        KTRY(timer.end(stream));
        KTRY(hipGraphLaunch(b.graphs[1], stream));
    } else {
        KTRY(hipGraphLaunch(b.graphs[0], stream));
    }
    // the flag and uncertified-row counts reach the host here (one
    // synchronisation per call)
    KTRY(hipStreamSynchronize(stream));
    KTRY(timer.collect(h));
    int64_t fallback = 0;
    for (size_t pi = 0; pi < b.parts.size(); ++pi) fallback += b.nflag_host[pi];
    if (fallback > 0) {
        // rare: the flagged rows' candidate lists are re-done exactly, then the
        // selection, certificate and re-rank of the parts holding them run again
        int64_t done = 0;
        KTRY(run_fallback(b, num_cu, stream, &done));
        for (size_t pi = 0; pi < b.parts.size(); ++pi)
            if (b.nflag_host[pi] > 0) KTRY(refinal_part(b, h, num_cu, pi, stream));
        KTRY(hipStreamSynchronize(stream));
    }
    int64_t rerun = 0;
    if (b.jobs[0].p.prec == kPrecF32) KTRY(run_rerun(b, stream, &rerun));
#undef KTRY
    add_host_stats(h, rows, fallback);
    add_host_rerun(h, rerun);
    return KNN_SUCCESS;
}

}  // namespace knn
