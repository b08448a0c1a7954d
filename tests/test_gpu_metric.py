"""Cosine and Pearson distances (Methods, "Distance calculation"): knn_graph,
knn_search and knn_batch_search with metric "cosine" / "pearson" against the
FP64 oracle's 1 - similarity, under the bar of knn_check.metric_tol."""
import sys

import numpy as np
import pytest

import oracle  # noqa: F401
import synth
from knn_check import compare_metric

pytestmark = pytest.mark.gpu

METRICS = ("cosine", "pearson")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def knn():
    import paper_1309_5478_amd as m
    return m


@pytest.fixture(scope="module")
def h(torch, knn):
    return knn.Handle(0)


def graph(h, torch, P, k, **kw):
    gd, gi = h.graph(torch.from_numpy(P).cuda(), k, **kw)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gi.cpu().numpy()


def search(h, torch, Q, C, k, **kw):
    gd, gi = h.search(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k, **kw)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gi.cpu().numpy()


@pytest.mark.parametrize("flags", [0, 2, 1], ids=["fused", "unfused", "fallback"])
@pytest.mark.parametrize("metric", METRICS)
def test_graph_uniform_all_rows(h, torch, metric, flags):
    """4096 uniform[0,1) points in d = 128, k = 16, own index excluded: every
    row (uniform data have a large common mean, the hard case for Pearson's
    centring)."""
    P = synth.uniform_points(4096, 128, seed=synth.SEEDS["metric"])
    say(f"graph 4096x128 k=16 metric={metric} flags={flags}")
    gd, gi = graph(h, torch, P, 16, metric=metric, flags=flags)
    near = compare_metric(P, P, 16, gd, gi, np.arange(4096), metric, self_ids=np.arange(4096))
    say(f"  near-tie rows: {near}")
    assert near <= 40


@pytest.mark.parametrize("metric", METRICS)
@pytest.mark.parametrize("prec,min_recall", [("fp32", 1.0), ("bf16", 0.99)])
def test_search_mixture(h, torch, metric, prec, min_recall):
    """Mixture queries against a mixture corpus (d = 256, k = 32): FP32 sets
    match outside the near-tie band; BF16 products with the exact re-rank keep
    recall >= 0.99 and exact distances."""
    C = synth.gmm_points(30000, 256, seed=synth.SEEDS["metric"])
    Q = synth.gmm_points(700, 256, seed=synth.SEEDS["metric"] + 100)
    say(f"search 700 x 30000 x 256 k=32 metric={metric} prec={prec}")
    gd, gi = search(h, torch, Q, C, 32, metric=metric, precision=prec)
    rows = np.arange(0, 700, 5)
    if prec == "fp32":
        near = compare_metric(Q, C, 32, gd[rows], gi[rows], rows, metric)
        assert near <= 3
    else:
        od, oi = oracle.knn(Q[rows], C, 32, metric=metric)
        hits = sum(len(set(gi[r].tolist()) & set(oi[t].tolist())) for t, r in enumerate(rows))
        recall = hits / (len(rows) * 32)
        say(f"  recall@32 {recall:.4f}")
        assert recall >= min_recall


@pytest.mark.parametrize("metric", METRICS)
def test_vectors_without_direction(h, torch, metric):
    """Zero vectors (and, for Pearson, constant ones) and vectors with a
    non-finite element have NaN distances: as queries their neighbours are the
    lowest indices; as corpus points they come last."""
    rng = np.random.default_rng(9)
    P = rng.standard_normal((3000, 64)).astype(np.float32)
    P[5] = 0.0
    P[17] = 3.25                      # constant: no direction for Pearson only
    P[40, 7] = np.inf
    P[41, 3] = np.nan
    P[2999] = 0.0
    gd, gi = graph(h, torch, P, 20, metric=metric)
    rows = np.array([0, 1, 5, 17, 40, 41, 100, 2999])
    compare_metric(P, P, 20, gd[rows], gi[rows], rows, metric, self_ids=np.arange(3000))
    assert np.isnan(gd[5]).all() and list(gi[5]) == [j for j in range(21) if j != 5][:20]
    bad = {5, 40, 41, 2999} | ({17} if metric == "pearson" else set())
    assert not (set(gi[100].tolist()) & bad)


def test_cosine_is_scale_invariant_bitwise(h, torch):
    """Scaling a vector by a power of two leaves its unit vector, and so every
    cosine result, bit for bit unchanged."""
    P = synth.normal_points(5000, 96, seed=synth.SEEDS["metric"])
    S = P * np.float32(2.0) ** np.random.default_rng(1).integers(-20, 20, size=(5000, 1)).astype(np.float32)
    a = graph(h, torch, P, 10, metric="cosine")
    b = graph(h, torch, S, 10, metric="cosine")
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


@pytest.mark.parametrize("metric", METRICS)
def test_batch_equals_per_job_calls(h, torch, knn, metric):
    """knn_batch_search with a metric returns each job's knn_search / knn_graph
    output bit for bit, eager and replayed."""
    rng = np.random.default_rng(21)
    jobs, host = [], []
    for j, (m, n, d, k) in enumerate([(300, 5000, 64, 8), (0, 100, 16, 3), (900, 20000, 128, 100),
                                      (None, 3000, 32, 40), (50, 60, 8, 64)]):
        C = rng.standard_normal((n, d)).astype(np.float32) + np.float32(j)
        Q = None if m is None else rng.standard_normal((m, d)).astype(np.float32)
        jobs.append((None if Q is None else torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k))
        host.append((Q, C, k))
    for flags in (0, knn.FLAG_NO_GRAPH):
        for _ in range(2):
            res = h.batch_search(jobs, metric=metric, flags=flags)
            torch.cuda.synchronize()
            for (q, c, k), (bd, bi) in zip(jobs, res):
                if q is None:
                    rd, ri = h.graph(c, k, metric=metric)
                else:
                    if q.shape[0] == 0:
                        continue
                    kk = min(k, c.shape[0])
                    rd, ri = h.search(q, c, kk, metric=metric)
                    bd, bi = bd[:, :kk], bi[:, :kk]
                assert np.array_equal(bi.cpu().numpy(), ri.cpu().numpy())
                assert np.array_equal(bd.cpu().numpy().view(np.uint32), rd.cpu().numpy().view(np.uint32))


def test_metric_option_is_checked(h, torch, knn):
    P = torch.zeros((100, 8), device="cuda")
    with pytest.raises(knn.KnnError):
        h.graph(P, 5, metric=3)
