#!/usr/bin/env python3
"""Benchmark of the fused distance-product + quick multi-select k-NN graph.

Workload (one step): knn_graph on N = 262144 points, d = 1024, FP32, drawn
from a 64-component Gaussian mixture (means N(0, 4I), unit covariance), k = 32,
own index excluded -- norms, sample threshold, fused MFMA product with
candidate filtering, exact fallback rows, candidate selection and FP32
re-rank.  Inputs are generated on the host, uploaded once and resident in HBM
before the timed region.  Also reported: quick multi-select throughput on a
materialised 8192 x 262144 block of the same graph's squared-distance matrix
(k = 32), per pivot rule, and the CPU oracle timed on a bounded row sample.

With --workload lowprec the step is one knn_graph on N = 2^20 points, d = 256,
k = 64 (Gaussian mixture) with the distance product in BF16, 4x oversampled
candidates and the exact FP32 re-rank; FP8 and FP32 products are timed once
beside it, with recall against the FP64 oracle on 32 sampled rows.

With --workload sweep: the paper's saturation shape, Q = 8 ... 256 rows of
n = 2^20 uniform values, k = 32 and 1024, rows split across workgroups or not,
with the nth_element CPU baseline beside it.

With --workload select: knn_select_k on 16384 x 65536 squared distances, k =
32, 256, 1024, every pivot rule, with the oracle and nth_element CPU baselines.

With --workload hostcorpus: knn_search_host_corpus with an 8 GiB corpus in
pinned host memory, its copies overlapping the search.

With --workload batch the step is instead one knn_batch_search over 512
uneven jobs (corpus sizes log-uniform in [1e3, 1e6], 1024 queries each, d in
{64, 128, 768}, k log-uniform in [1, 1024], uniform or Gaussian-mixture data
drawn on the device), replayed from its captured HIP graphs.

Prints one JSON line.  One GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # dense matrix peaks
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E peak
METRIC = "k-NNG rows/s & select GB/s (N=262144,d=1024,k=32), learned vs plain pivots"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(profile="knng_fused_262144x1024_k32_traffic.md", sources=("gemm.hip",), key=None):
    """HBM bytes per launch from a committed memory-counter summary, if the
    kernel sources it names are unchanged since the counters were taken.
    `key` picks a `traffic_bytes_per_launch[key]` line instead of the plain one."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(prof).read()
        tag = re.escape(f"[{key}]") if key else ""
        value = int(re.search(r"traffic_bytes_per_launch" + tag + r": (\d+)", text).group(1))
        for name in sources:
            src = os.path.join(ROOT, "paper_1309_5478_amd", "csrc", name)
            want = re.search(r"source_sha256\(" + re.escape(name) + r"\): ([0-9a-f]{64})", text)
            if want is None and name == sources[0]:
                want = re.search(r"source_sha256: ([0-9a-f]{64})", text)
            if want is None or hashlib.sha256(open(src, "rb").read()).hexdigest() != want.group(1):
                return None
    except (OSError, AttributeError):
        return None
    return value


def parity_block(Q, C, rows, gd, gi, od, oi, k, self_ids=None, band=1e-5, tol=1e-5):
    """GPU rows (gd, gi: the listed query rows, k columns) against the oracle's
    k + 1 nearest (od, oi; FP64 direct distances, stable order).  A row whose set
    differs only by points within the near-tie band of the oracle's k-th
    distance counts as a near tie; any other difference is a mismatch.  Every
    returned distance is compared with its FP64 direct value."""
    import numpy as np
    mismatch = near = bad_dist = 0
    max_rel = 0.0
    for t, r in enumerate(rows):
        g = gi[t].astype(np.int64)
        diff = Q[r].astype(np.float64)[None, :] - C[g].astype(np.float64)
        ref = np.einsum("ij,ij->i", diff, diff)
        nz = ref > 0
        rel = np.abs(gd[t].astype(np.float64) - ref)
        if nz.any():
            max_rel = max(max_rel, float(np.max(rel[nz] / ref[nz])))
        bad_dist += int(np.sum(rel[nz] > tol * ref[nz]))
        gs, os_ = set(g.tolist()), set(oi[t, :k].tolist())
        ok = len(gs) == k and (self_ids is None or int(self_ids[t]) not in gs)
        if ok and gs != os_:
            kth = od[t, k - 1]
            ok = all(abs(float(np.dot(Q[r].astype(np.float64) - C[j], Q[r].astype(np.float64) - C[j])) - kth)
                     <= band * max(kth, 1e-30) for j in gs ^ os_)
            near += int(ok)
        mismatch += int(not ok)
    return {"rows": int(len(rows)), "set_mismatch": int(mismatch), "near_ties": int(near),
            "dist_errors": int(bad_dist), "max_rel_dist_err": max_rel, "tolerance": tol}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--d", type=int, default=1024)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--pivot", default="sample", choices=["plain", "sample", "learned"])
    ap.add_argument("--select-rows", type=int, default=8192)
    ap.add_argument("--no-select", action="store_true", help="skip the select_k block")
    ap.add_argument("--no-pivot-compare", action="store_true", help="skip the per-pivot-rule steps")
    ap.add_argument("--cpu-rows", type=int, default=1536, help="query rows in the CPU oracle sample (0: skip)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-product row of the k-NNG workload")
    ap.add_argument("--workload", default="knng",
                    choices=["knng", "small", "batch", "select", "lowprec", "sweep", "hostcorpus"])
    ap.add_argument("--batch-jobs", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference dispatch for memory counters)")
    ap.add_argument("--select-case", default=None,
                    help="select workload: only this case, as k,pivot (e.g. 1024,sample), one timed call per step")
    ap.add_argument("--precisions", default="bf16,fp8,fp32",
                    help="lowprec workload: the timed precision first, then the others (comma-separated)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1309_5478_amd as knn
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)           # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batch":
        return bench_batch(args, knn, torch, np)
    if args.workload == "select":
        return bench_select(args, knn, torch, np)
    if args.workload == "lowprec":
        return bench_lowprec(args, knn, torch, np, synth)
    if args.workload == "sweep":
        return bench_sweep(args, knn, torch, np, synth)
    if args.workload == "hostcorpus":
        return bench_hostcorpus(args, knn, torch, np, synth)
    if args.workload == "small":
        return bench_small(args, knn, torch, np, synth)
    N, d, k = args.n, args.d, args.k
    t0 = time.perf_counter()
    P = synth.gmm_points(N, d, seed=synth.SEEDS["knng_fused"])
    log(f"generated {N}x{d} points in {time.perf_counter() - t0:.1f} s")
    dev = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    h = knn.Handle(0)
    flags = knn.FLAG_TIMING

    out = {}

    def step(pivot):
        out["d"], out["i"] = h.graph(dev, k, pivot=pivot, flags=flags)
        return h.stats()   # synchronises the stream

    for _ in range(args.warmup):
        step(args.pivot)
    torch.cuda.synchronize()
    prod_ms = prod_flops = 0.0
    prod_launches = fallback = cands = uncert = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step(args.pivot)
        prod_ms += st["product_ms"]
        prod_flops += st["product_flops"]
        prod_launches += st["product_launches"]
        fallback += st["fallback_rows"]
        cands += st["candidates_total"]
        uncert += st["rows_uncertified"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g_dist, g_idx = out["d"].cpu().numpy(), out["i"].cpu().numpy()   # the last timed step's output
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    rows_per_s = N / (ms_per_step / 1e3)
    achieved = prod_flops / (prod_ms / 1e3) / 1e12 if prod_ms > 0 else 0.0
    log(f"knn_graph: {ms_per_step:.1f} ms/step, {rows_per_s:.0f} rows/s; product {prod_ms / max(prod_launches, 1):.2f} ms"
        f" per launch, {achieved:.1f} TFLOP/s")

    pivots = {args.pivot: round(rows_per_s, 1)}
    if not args.no_pivot_compare:
        for pv in ("plain", "sample", "learned"):
            if pv in pivots:
                continue
            step(pv)
            torch.cuda.synchronize()
            a = time.perf_counter()
            step(pv)
            torch.cuda.synchronize()
            pivots[pv] = round(N / (time.perf_counter() - a), 1)
            log(f"knn_graph pivot={pv}: {pivots[pv]:.0f} rows/s")

    # the same k-NN graph with the product in BF16 (k' = 4k candidates, exact
    # FP32 re-rank), against the BF16 matrix-core peak
    bf16 = None
    if not args.no_bf16:
        for _ in range(2):
            out["bd"], out["bi"] = h.graph(dev, k, precision="bf16", flags=flags)
            bst = h.stats()
        a = time.perf_counter()
        bsteps = 2
        bms = bfl = 0.0
        for _ in range(bsteps):
            out["bd"], out["bi"] = h.graph(dev, k, precision="bf16", flags=flags)
            bst = h.stats()
            bms += bst["product_ms"]
            bfl += bst["product_flops"]
        bsec = (time.perf_counter() - a) / bsteps
        btf = bfl / (bms / 1e3) / 1e12 if bms > 0 else 0.0
        bf16 = {"ms_per_step": round(bsec * 1e3, 2), "rows_per_s": round(N / bsec, 1),
                "product_ms_per_launch": round(bms / max(bsteps * bst["product_launches"], 1), 3),
                "product_tflops": round(btf, 1), "frac_of_bf16_peak": round(btf / PEAK_MFMA_TFLOPS["bf16"], 4),
                "rows_uncertified": bst["rows_uncertified"], "fallback_rows": bst["fallback_rows"]}
        log(f"knn_graph bf16: {bf16['ms_per_step']} ms/step, {bf16['rows_per_s']:.0f} rows/s; product {btf:.1f} TFLOP/s")

    select = None
    if not args.no_select:
        R = min(args.select_rows, N)
        D = h.distances(dev[:R], dev)          # R x N squared distances, resident in HBM
        torch.cuda.synchronize()
        select = {"rows": R, "cols": N, "k": k, "GB/s": {}, "bytes_per_call": 4 * R * N + 8 * R * k}
        for pv in ("sample", "plain", "learned"):
            h.select_k(D, k, pivot=pv)
            torch.cuda.synchronize()
            reps = 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                h.select_k(D, k, pivot=pv)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            select["GB/s"][pv] = round(select["bytes_per_call"] / ms / 1e6, 1)
            log(f"select_k {R}x{N} k={k} pivot={pv}: {ms:.3f} ms, {select['GB/s'][pv]:.0f} GB/s")
        select["frac_of_hbm_peak"] = round(select["GB/s"]["sample"] / PEAK_HBM_GBS, 4)
        del D
        torch.cuda.empty_cache()

    cpu = parity = None
    if args.cpu_rows > 0:
        import oracle
        rows = np.sort(np.random.default_rng(0).choice(N, args.cpu_rows, replace=False))
        threads = oracle.default_threads()
        a = time.perf_counter()
        od, oi = oracle.knn(P[rows], P, k + 1, self_ids=rows, nthreads=threads)
        sec = time.perf_counter() - a
        cpu = {"value": round(args.cpu_rows / sec, 3), "unit": "rows/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_rows} query rows of the same k-NNG (FP64 direct distances to all {N} points"
                         f" + stable sort), {sec:.1f} s"}
        log(f"oracle: {cpu['value']} rows/s on {threads} threads")
        # the same rows of the last timed GPU step against the oracle
        parity = parity_block(P, P, rows, g_dist[rows], g_idx[rows], od, oi, k, self_ids=rows)
        parity["rows_uncertified"] = uncert // max(args.steps, 1)
        log(f"parity: {parity}")
        if bf16 is not None:
            bd, bi = out["bd"].cpu().numpy()[rows], out["bi"].cpu().numpy()[rows]
            hits = sum(len(set(x.tolist()) & set(y[:k].tolist())) for x, y in zip(bi, oi))
            bf16["recall"] = round(hits / (len(rows) * k), 6)
            bf16["parity"] = parity_block(P, P, rows, bd, bi, od, oi, k, self_ids=rows)
            log(f"bf16 recall {bf16['recall']}, parity {bf16['parity']}")
        # one core: a smaller sample of the same rows
        r1 = rows[:64]
        a = time.perf_counter()
        oracle.knn(P[r1], P, k + 1, self_ids=r1, nthreads=1)
        sec1 = time.perf_counter() - a
        cpu["one_core"] = {"value": round(len(r1) / sec1, 3), "unit": "rows/s", "cores": 1,
                           "sample": f"{len(r1)} of the same rows on one thread, {sec1:.1f} s"}
        log(f"oracle one core: {cpu['one_core']['value']} rows/s")

    line = {
        "metric": METRIC,
        "value": round(rows_per_s, 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fused k-NNG, N={N}, d={d}, k={k}, Gaussian mixture (64 comp.), FP32",
                   "N": N, "d": d, "k": k, "pivot": args.pivot, "oversample": 4},
        "pivots_rows_per_s": pivots,
        "bf16": bf16,
        "roofline": {"bound": "mfma", "kernel": "dist_gemm_kernel (fused filter epilogue)",
                     "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                     "traffic": measured_traffic() if (N, d, k) == (262144, 1024, 32) else None,
                     "launch_ms": round(prod_ms / max(prod_launches, 1), 3),
                     "flops_per_launch": prod_flops / max(prod_launches, 1)},
        "select": select,
        "fallback_rows_per_step": fallback / args.steps,
        "candidates_per_row": round(cands / args.steps / N, 1),
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if parity and (parity["set_mismatch"] or parity["dist_errors"]):
        log("PARITY FAILURE: GPU rows differ from the oracle beyond the near-tie band / distance tolerance")
        sys.exit(1)


def bench_small(args, knn, torch, np, synth):
    """The smallest graph configuration: N = 4096 uniform[0,1) points in d = 128,
    k = 16, the own point excluded.  Launch- and latency-bound (4.3e9 flops), so
    the roofline fraction only says how far from compute-bound it is.  One step
    is one knn_graph call, timed fused (threshold filter in the product) and
    unfused (the distance matrix materialised, then select_k: the paper's
    two-step pipeline); every row of both is checked against the oracle, which
    is timed on all rows on all host threads and on one."""
    import oracle
    N, d, k = 4096, 128, 16
    P = synth.uniform_points(N, d, seed=synth.SEEDS["knng_small"])
    dev = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    h = knn.Handle(0)
    rows = np.arange(N)
    threads = oracle.default_threads()
    a = time.perf_counter()
    od, oi = oracle.knn(P, P, k + 1, self_ids=rows, nthreads=threads)
    cpu_sec = time.perf_counter() - a
    a = time.perf_counter()
    oracle.knn(P, P, k + 1, self_ids=rows, nthreads=1)
    cpu1_sec = time.perf_counter() - a
    res = {}
    for tag, flags in (("fused", 0), ("unfused", knn.FLAG_UNFUSED)):
        for _ in range(max(args.warmup, 1)):
            h.graph(dev, k, flags=flags)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            gd, gi = h.graph(dev, k, flags=flags)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
        par = parity_block(P, P, rows, gd, gi, od, oi, k, self_ids=rows)
        res[tag] = {"ms_per_call": round(ms, 4), "rows_per_s": round(N / ms * 1e3, 1), "parity": par}
        log(f"knn_graph {tag} N={N} d={d} k={k}: {ms:.3f} ms per call; parity {par}")
    flops = 2.0 * N * N * d
    ms = res["fused"]["ms_per_call"]
    line = {
        "metric": "k-NNG rows/s (N=4096, d=128, k=16, uniform; launch-bound)",
        "value": res["fused"]["rows_per_s"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "k-NNG, N=4096, d=128, k=16, uniform[0,1), own point excluded; fused and unfused",
                   "N": N, "d": d, "k": k},
        "per_path": res,
        "roofline": {"bound": "mfma", "kernel": "whole knn_graph call (latency-bound: a few launches of a few us)",
                     "achieved": round(flops / ms / 1e9, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flops / ms / 1e9 / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None},
        "cpu_baseline": {"value": round(N / cpu_sec, 1), "unit": "rows/s", "cores": threads, "kind": "oracle",
                         "sample": f"all {N} rows (FP64 direct distances + stable sort), {cpu_sec:.2f} s",
                         "one_core": {"value": round(N / cpu1_sec, 1), "unit": "rows/s", "cores": 1,
                                      "sample": f"all {N} rows on one thread, {cpu1_sec:.2f} s"}},
    }
    print(json.dumps(line), flush=True)


def bench_select(args, knn, torch, np):
    import synth
    M, N, d = 16384, 65536, 256
    t0 = time.perf_counter()
    D = synth.sqdist_matrix_normal(M, N, d, seed=synth.SEEDS["select"])
    log(f"generated {M}x{N} squared-distance matrix in {time.perf_counter() - t0:.1f} s")
    dev = torch.from_numpy(D).cuda()
    torch.cuda.synchronize()
    h = knn.Handle(0)
    res, tot_bytes, tot_ms = {}, 0.0, 0.0
    cases = [(k, pv) for k in (32, 256, 1024) for pv in ("sample", "learned", "plain")]
    if args.select_case:
        ck, cp = args.select_case.split(",")
        cases = [(int(ck), cp)]
    for k, pivot in cases:
        nbytes = 4 * M * N + 8 * M * k
        for _ in range(args.warmup):
            h.select_k(dev, k, pivot=pivot)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            h.select_k(dev, k, pivot=pivot)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        st = h.stats()
        res[f"k={k},{pivot}"] = {"ms": round(ms, 4), "GB/s": round(nbytes / ms / 1e6, 1),
                                 "passes_per_row": round(st["passes_total"] / M, 3),
                                 "streams_per_row": round(st["stream_passes_total"] / M, 4)}
        if pivot == "sample":
            res[f"k={k},{pivot}"]["traffic"] = measured_traffic("select_16384x65536_traffic.md", ("select.hip",),
                                                                key=f"k={k}")
        log(f"select_k k={k} pivot={pivot}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
        if pivot == "sample" or args.select_case:
            tot_bytes += nbytes
            tot_ms += ms
    gbs = tot_bytes / tot_ms / 1e6
    # reference: a plain device-to-device copy (torch) of 2 GiB, bytes read +
    # written per second, beside the 8 TB/s spec (never substituted for it)
    del dev
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 * 5 / c0.elapsed_time(c1) / 1e6
    del src, dst
    log(f"reference device copy: {copy_gbs:.0f} GB/s (read + write)")
    # HBM bytes per launch of the selection kernel, the mean over the timed k
    # (from the committed counter summary; null if the kernel changed since)
    tr = [v.get("traffic") for key, v in res.items() if key.endswith(",sample")]
    traffic = round(sum(tr) / len(tr)) if tr and None not in tr else None
    cpu = None
    if args.cpu_rows > 0:
        import oracle
        rows = np.random.default_rng(0).choice(M, min(args.cpu_rows, 256), replace=False)
        threads = oracle.default_threads()
        sec = 0.0
        for k in (32, 256, 1024):
            a = time.perf_counter()
            oracle.select_k(D[rows], k, nthreads=threads)
            sec += time.perf_counter() - a
        cpu = {"value": round(3 * len(rows) * 4 * N / sec / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(rows)} rows of the matrix at each of k = 32, 256, 1024 (stable sort of each row), {sec:.1f} s"}
        log(f"oracle: {cpu['value']} GB/s on {threads} threads")
        # one core, and the standard library's nth_element + sort of the first k
        # (the kind of CPU selection the paper compares against), on the same rows
        a = time.perf_counter()
        oracle.select_k(D[rows[:64]], 1024, nthreads=1)
        s1 = time.perf_counter() - a
        cpu["one_core"] = {"value": round(64 * 4 * N / s1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                           "sample": f"64 of the rows at k = 1024 on one thread, {s1:.1f} s"}
        nth = {}
        for k in (32, 256, 1024):
            for nt, tag in ((threads, "all_cores"), (1, "one_core")):
                rr = rows if nt > 1 else rows[:64]
                a = time.perf_counter()
                oracle.nth_select_k(D[rr], k, nthreads=nt)
                sec_n = time.perf_counter() - a
                nth[f"k={k},{tag}"] = round(len(rr) * 4 * N / sec_n / 1e9, 3)
        cpu["nth_element_GBps"] = nth
        cpu["nth_element_cores"] = threads
        log(f"oracle one core: {cpu['one_core']['value']} GB/s; nth_element GB/s: {nth}")
    line = {
        "metric": "select_k GB/s (16384x65536 FP32 squared distances, k = 32 / 256 / 1024)",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tot_ms, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "select_k on 16384 x 65536 FP32 squared distances of N(0,1) points in d = 256,"
                               " k = 32, 256, 1024, sample pivots (one step = the three k)",
                   "rows": M, "cols": N},
        "per_k": res,
        "reference_copy_GBps": round(copy_gbs, 1),
        "roofline": {"bound": "hbm", "kernel": "select_rows_kernel", "achieved": round(gbs, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_sweep(args, knn, torch, np, synth):
    """The paper's saturation workload shape (Results, Figure 8): rows of
    n = 2^20 uniform[0,1) values, Q = 8 ... 256 rows, k = 32 and 1024, with
    rows split across workgroups (default) and without (one workgroup per row,
    as the paper's method); time per row and GB/s.  Then the shapes of its
    comparisons (Figures 6 and 7): a fixed n Q = 2^27 values, Q = 2^3 ... 2^14,
    k = 32 and 512, GB/s against log2(n / Q).  Beside it the CPU selection
    baseline (nth_element + sort of k) at Q = 256, one core and all cores."""
    n = 1 << 20
    Qmax = 256
    D = synth.uniform_points(Qmax, n, seed=synth.SEEDS["sweep"])
    dev = torch.from_numpy(D).cuda()
    torch.cuda.synchronize()
    h = knn.Handle(0)
    res = {}
    for k in (32, 1024):
        for Q in (8, 16, 32, 64, 128, 256):
            sub = dev[:Q]
            for tag, flags in (("split", 0), ("whole_rows", knn.FLAG_NO_SPLIT)):
                for _ in range(max(args.warmup, 1)):
                    h.select_k(sub, k, flags=flags)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    h.select_k(sub, k, flags=flags)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                parts = h.stats()["split_parts"]
                nbytes = 4 * Q * n + 8 * Q * k
                res[f"k={k},Q={Q},{tag}"] = {"ms": round(ms, 4), "us_per_row": round(1e3 * ms / Q, 2),
                                              "GB/s": round(nbytes / ms / 1e6, 1), "parts": parts}
                log(f"sweep k={k} Q={Q} {tag}: {ms:.3f} ms, {1e3 * ms / Q:.2f} us/row, {nbytes / ms / 1e6:.0f} GB/s,"
                    f" parts {parts}")
    # fixed total size n Q = 2^27 (the paper's comparison shapes, Results,
    # Figures 6-7): Q = 2^3 ... 2^14 rows, GB/s against log2(n / Q)
    del dev
    flat = torch.from_numpy(synth.uniform_points(1 << 13, 1 << 14, seed=synth.SEEDS["sweep"] + 100)).cuda().view(-1)
    torch.cuda.synchronize()
    fixed = {}
    for k in (32, 512):
        for lq in range(3, 15):
            Q, n2 = 1 << lq, 1 << (27 - lq)
            sub = flat.view(Q, n2)
            for _ in range(max(args.warmup, 1)):
                h.select_k(sub, k)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                h.select_k(sub, k)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            nbytes = 4 * Q * n2 + 8 * Q * k
            fixed[f"k={k},log2(n/Q)={27 - 2 * lq}"] = {"Q": Q, "n": n2, "ms": round(ms, 4),
                                                       "GB/s": round(nbytes / ms / 1e6, 1),
                                                       "parts": h.stats()["split_parts"]}
            log(f"n Q = 2^27, k={k}, Q={Q}, n={n2}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
    del flat
    cpu = None
    if args.cpu_rows > 0:
        import oracle
        threads = oracle.default_threads()
        nth = {}
        for k in (32, 1024):
            for nt, tag, Q in ((threads, "all_cores", 256), (1, "one_core", 32)):
                a = time.perf_counter()
                oracle.nth_select_k(D[:Q], k, nthreads=nt)
                sec = time.perf_counter() - a
                nth[f"k={k},{tag}"] = {"us_per_row": round(1e6 * sec / Q, 1), "rows": Q}
        cpu = {"value": nth["k=1024,one_core"]["us_per_row"], "unit": "us/row", "cores": 1, "kind": "nth_element",
               "sample": "std::nth_element + sort of the first k per row: 32 rows on one core, 256 rows on all"
                         f" {threads} cores, k = 32 and 1024", "per_case": nth}
        log(f"nth_element: {nth}")
    head = res["k=32,Q=8,split"]
    line = {
        "metric": "select_k rows of n = 2^20 at few rows (saturation sweep, Q = 8 ... 256)",
        "value": head["GB/s"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "select_k on Q x 2^20 uniform[0,1) FP32 rows, Q = 8 ... 256, k = 32 and 1024;"
                               " value: Q = 8, k = 32, rows split across workgroups", "n": n},
        "per_case": res,
        "fixed_total_2p27": fixed,
        "roofline": {"bound": "hbm", "kernel": "select_rows_kernel (parts) + key-list merges",
                     "achieved": head["GB/s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(head["GB/s"] / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_hostcorpus(args, knn, torch, np, synth):
    """A corpus in pinned host memory (2^23 points in d = 256, 8 GiB, Gaussian
    mixture) searched by 16384 resident queries, k = 32, in 1 GiB partitions
    whose copies overlap the search (knn_search_host_corpus).  Beside it: the
    copies alone and the search of one resident partition, to show the overlap."""
    n, d, m, k = 1 << 23, 256, 16384, 32
    t0 = time.perf_counter()
    C = synth.gmm_points(n, d, seed=synth.SEEDS["lowprec"] + 10)
    Q = synth.gmm_points(m, d, seed=synth.SEEDS["lowprec"] + 11)
    Cp = torch.empty((n, d), dtype=torch.float32, pin_memory=True)
    Cp.copy_(torch.from_numpy(C))
    qd = torch.from_numpy(Q).cuda()
    log(f"generated {n}x{d} host corpus ({n * d * 4 / 2**30:.0f} GiB, pinned) in {time.perf_counter() - t0:.1f} s")
    h = knn.Handle(0)
    part = (1 << 30) // (d * 4)
    for _ in range(max(args.warmup, 1)):
        h.search_host_corpus(qd, Cp, k, part_rows=part)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        gd, gi = h.search_host_corpus(qd, Cp, k, part_rows=part)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / args.steps
    # the copies alone, and the search of one resident partition
    dbuf = torch.empty((part, d), dtype=torch.float32, device="cuda")
    t = time.perf_counter()
    for p0 in range(0, n, part):
        dbuf[: min(part, n - p0)].copy_(Cp[p0:p0 + part], non_blocking=True)
    torch.cuda.synchronize()
    copy_sec = time.perf_counter() - t
    h.search(qd, dbuf, k)
    torch.cuda.synchronize()
    t = time.perf_counter()
    h.search(qd, dbuf, k)
    torch.cuda.synchronize()
    part_sec = time.perf_counter() - t
    parts = (n + part - 1) // part
    serial = copy_sec + parts * part_sec
    log(f"host corpus: {sec * 1e3:.1f} ms/step; copies alone {copy_sec * 1e3:.1f} ms "
        f"({n * d * 4 / copy_sec / 1e9:.1f} GB/s), {parts} partition searches {parts * part_sec * 1e3:.1f} ms")
    cpu = None
    if args.cpu_rows > 0:
        import oracle
        threads = oracle.default_threads()
        rows = np.arange(0, m, m // 16)
        a = time.perf_counter()
        od, oi = oracle.knn(Q[rows], C, k, nthreads=threads)
        csec = time.perf_counter() - a
        g = gi.cpu().numpy()[rows]
        match = int(sum(set(x.tolist()) == set(y.tolist()) for x, y in zip(g, oi)))
        cpu = {"value": round(len(rows) / csec, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(rows)} queries against the whole corpus (FP64 direct distances + stable sort),"
                         f" {csec:.1f} s; {match} of {len(rows)} neighbour sets equal to the GPU's"}
        log(f"oracle: {cpu['value']} queries/s; sets equal on {match}/{len(rows)} rows")
    flops = 2.0 * m * n * d
    line = {
        "metric": "k-NN queries/s with the corpus in host memory (2^23 x 256 corpus, 16384 queries, k = 32)",
        "value": round(m / sec, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 2),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "knn_search_host_corpus: 8 GiB pinned host corpus (Gaussian mixture, d = 256),"
                               " 16384 resident queries, k = 32, 1 GiB partitions", "n": n, "d": d, "m": m, "k": k},
        "copy_only_ms": round(copy_sec * 1e3, 1),
        "h2d_GBps": round(n * d * 4 / copy_sec / 1e9, 1),
        "partition_search_ms": round(part_sec * 1e3, 1),
        "serial_estimate_ms": round(serial * 1e3, 1),
        "overlap_saving": round(1.0 - sec / serial, 3),
        "roofline": {"bound": "mfma", "kernel": "dist_gemm_kernel (fused filter epilogue, per partition)",
                     "achieved": round(flops / sec / 1e12, 1), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flops / sec / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_lowprec(args, knn, torch, np, synth):
    N, d, k = 1 << 20, 256, 64
    t0 = time.perf_counter()
    P = synth.gmm_points(N, d, seed=synth.SEEDS["lowprec"])
    log(f"generated {N}x{d} points in {time.perf_counter() - t0:.1f} s")
    dev = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    h = knn.Handle(0)
    rows = np.random.default_rng(0).choice(N, 256, replace=False)
    import oracle
    threads = oracle.default_threads()
    a = time.perf_counter()
    od, oi = oracle.knn(P[rows], P, k, self_ids=rows, nthreads=threads)
    cpu_sec = time.perf_counter() - a

    def run(prec, steps, warmup):
        for _ in range(warmup):
            h.graph(dev, k, precision=prec, flags=knn.FLAG_TIMING)
            h.stats()
        torch.cuda.synchronize()
        tot = {"product_ms": 0.0, "product_flops": 0.0, "product_launches": 0, "fallback_rows": 0,
               "candidates_total": 0, "rows_uncertified": 0}
        t = time.perf_counter()
        for _ in range(steps):
            gd, gi = h.graph(dev, k, precision=prec, flags=knn.FLAG_TIMING)
            st = h.stats()   # synchronises the stream
            for key in tot:
                tot[key] += st[key]
        sec = (time.perf_counter() - t) / steps
        g = gi.cpu().numpy()[rows]
        gdist = gd.cpu().numpy()[rows].astype(np.float64)
        recall = sum(len(set(x.tolist()) & set(y.tolist())) for x, y in zip(g, oi)) / (len(rows) * k)
        relv = np.abs(gdist - od) / np.maximum(np.abs(od), 1e-30)
        rel = float(np.max(relv))
        tf = tot["product_flops"] / (tot["product_ms"] / 1e3) / 1e12 if tot["product_ms"] > 0 else 0.0
        r = {"ms_per_step": round(sec * 1e3, 2), "rows_per_s": round(N / sec, 1),
             "product_ms_per_launch": round(tot["product_ms"] / max(tot["product_launches"], 1), 3),
             "product_tflops": round(tf, 1), "frac_of_peak": round(tf / PEAK_MFMA_TFLOPS[prec], 4),
             "fallback_rows_per_step": tot["fallback_rows"] / steps,
             "candidates_per_row": round(tot["candidates_total"] / steps / N, 1),
             "certified_fraction": round(1.0 - tot["rows_uncertified"] / (steps * N), 4),
             "recall": recall, "max_rel_dist_err": rel, "mean_rel_dist_err": float(np.mean(relv)),
             "oracle_rows": int(len(rows))}
        log(f"knn_graph {prec}: {r['ms_per_step']} ms/step, {r['rows_per_s']:.0f} rows/s; product {tf:.1f} TFLOP/s"
            f" ({100 * r['frac_of_peak']:.1f} % of peak), recall {recall}, max rel. distance error {rel:.2e}")
        return r, tot

    precs = args.precisions.split(",")
    res, tot = run(precs[0], args.steps, args.warmup)
    others = {p: run(p, 1, 1)[0] for p in precs[1:]}
    achieved = res["product_tflops"]
    line = {
        "metric": "reduced-precision k-NNG rows/s (N=2^20, d=256, k=64, BF16 product + FP32 re-rank)",
        "value": res["rows_per_s"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"reduced-precision k-NNG, N={N}, d={d}, k={k}, Gaussian mixture (64 comp.),"
                               " BF16 product, k' = 4k candidates, exact FP32 re-rank",
                   "N": N, "d": d, "k": k, "oversample": 4},
        precs[0]: res,
        **others,
        "roofline": {"bound": "mfma", "kernel": "dist_gemm_sk_kernel + sk_append_kernel (resident corpus, fused filter"
                                                   " epilogue with the kept keys staged per wave, BF16)",
                     "achieved": achieved, "peak": PEAK_MFMA_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_MFMA_TFLOPS["bf16"], 4),
                     "traffic": measured_traffic("lowprec_2p20x256_k64_traffic.md", ("gemm_sk.hip", "plan.hpp"))
                     if precs[0] == "bf16" else None,
                     "launch_ms": res["product_ms_per_launch"],
                     "flops_per_launch": tot["product_flops"] / max(tot["product_launches"], 1)},
        "cpu_baseline": {"value": round(len(rows) / cpu_sec, 3), "unit": "rows/s", "cores": threads, "kind": "oracle",
                         "sample": f"{len(rows)} query rows (FP64 direct distances to all {N} points + stable sort),"
                                   f" {cpu_sec:.1f} s"},
    }
    print(json.dumps(line), flush=True)


def bench_batch(args, knn, torch, np):
    from synth.gpu import batch_jobs, job_points
    J = batch_jobs(args.batch_jobs)
    t0 = time.perf_counter()
    data = [job_points(j) for j in J]
    outs = [(torch.empty((j["m"], j["k"]), dtype=torch.float32, device="cuda"),
             torch.empty((j["m"], j["k"]), dtype=torch.int32, device="cuda")) for j in J]
    torch.cuda.synchronize()
    gb = sum(j["n"] * j["d"] * 4 for j in J) / 1e9
    log(f"generated {len(J)} jobs, {gb:.1f} GB of corpora, in {time.perf_counter() - t0:.1f} s")
    jobs = [(q, c, j["k"]) for (q, c), j in zip(data, J)]
    flops = sum(2.0 * j["m"] * j["n"] * j["d"] for j in J)
    queries = sum(j["m"] for j in J)
    h = knn.Handle(0)
    pivot = "learned"
    flags = knn.FLAG_AUTOTUNE

    def step(extra=0):
        h.batch_search(jobs, pivot=pivot, flags=flags | extra, out=outs)
        return h.stats()   # synchronises the stream

    a = time.perf_counter()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warm-up (plan, tile timing, graph capture): {time.perf_counter() - a:.1f} s")
    fallback = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        fallback += st["fallback_rows"]
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    # one more step with the product launch timed by HIP events (its own plan)
    step(knn.FLAG_TIMING)
    st = step(knn.FLAG_TIMING)
    prod_ms = st["product_ms"]
    achieved = st["product_flops"] / (prod_ms / 1e3) / 1e12 if prod_ms > 0 else 0.0
    log(f"knn_batch_search: {ms_per_step:.1f} ms/step, {queries / ms_per_step * 1e3:.0f} queries/s;"
        f" grouped product {prod_ms:.2f} ms, {achieved:.1f} TFLOP/s")

    # the same call with every step eager (no graph replays), and with the
    # plain pivot rule instead of the learned one (its own plan and graphs)
    compare = {}
    for tag, extra, pv in (("eager", knn.FLAG_NO_GRAPH, pivot), ("plain_pivots", 0, "plain"),
                           ("sample_pivots", 0, "sample")):
        h.batch_search(jobs, pivot=pv, flags=flags | extra, out=outs)
        h.stats()
        a = time.perf_counter()
        h.batch_search(jobs, pivot=pv, flags=flags | extra, out=outs)
        h.stats()
        compare[tag] = round((time.perf_counter() - a) * 1e3, 2)
        log(f"knn_batch_search {tag}: {compare[tag]} ms")
    compare["graph_learned"] = round(ms_per_step, 2)

    cpu = None
    if args.cpu_rows > 0:
        import oracle
        rng = np.random.default_rng(0)
        pick = rng.choice(len(J), 32, replace=False)
        threads = oracle.default_threads()
        sec, rows = 0.0, 0
        for t in pick:
            q, c = data[t]
            r = rng.choice(J[t]["m"], 64, replace=False)
            Qh, Ch = q[torch.from_numpy(r).cuda()].cpu().numpy(), c.cpu().numpy()
            a = time.perf_counter()
            oracle.knn(Qh, Ch, min(J[t]["k"], J[t]["n"]), nthreads=threads)
            sec += time.perf_counter() - a
            rows += 64
        cpu = {"value": round(rows / sec, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"64 query rows of each of 32 jobs drawn from the batch (FP64 direct distances to the"
                         f" job's whole corpus + stable sort), {sec:.1f} s"}
        log(f"oracle: {cpu['value']} queries/s on {threads} threads")

    line = {
        "metric": "batched k-NN queries/s (512 uneven jobs, one graph replay per call)",
        "value": round(queries / ms_per_step * 1e3, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(J)} k-NN jobs, 1024 queries each, N log-uniform in [1e3, 1e6],"
                               " d in {64, 128, 768}, k log-uniform in [1, 1024], uniform / Gaussian mixture, FP32",
                   "jobs": len(J), "corpus_GB": round(gb, 1), "pivot": pivot, "autotune": True},
        "jobs_per_s": round(len(J) / ms_per_step * 1e3, 2),
        "roofline": {"bound": "mfma", "kernel": "dist_gemm_grouped_kernel (fused filter epilogue)",
                     "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                     "launch_ms": round(prod_ms, 3), "flops_per_launch": flops},
        "fallback_rows_per_step": fallback / max(args.steps, 1),
        "ms_per_call": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
