"""Parity at the full sizes the benchmark runs, against the FP64 oracle.

* Fused k-NN graph, N = 262144 points in d = 1024 (64-component Gaussian
  mixture), k = 32, FP32 products: 512 seeded query rows compared with the
  oracle (sets equal outside the 1e-5 near-tie band, distances within 1e-5
  relative), invariants on every row, and identical bits whatever the pivot
  rule.
* Reduced precision, N = 2^20 points in d = 256, k = 64: FP32 rows held to the
  same bar; BF16 and FP8 products (k' = 4k candidates, exact FP32 re-rank)
  report recall@k, distance error and the certified fraction on 256 rows, with
  recall floors and the distance bar asserted.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from knn_check import compare

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def h(torch):
    import paper_1309_5478_amd as knn
    return knn.Handle(0)


def every_row_invariants(gd, gi, n, self_exclude):
    """Indices in range and distinct, own index absent, rows ascending."""
    assert gi.min() >= 0 and gi.max() < n
    srt = np.sort(gi, axis=1)
    assert not (srt[:, 1:] == srt[:, :-1]).any(), "duplicate index in a row"
    if self_exclude:
        assert not (gi == np.arange(gi.shape[0])[:, None]).any(), "own index returned"
    assert (np.diff(gd, axis=1) >= 0).all(), "row not ascending"
    assert np.isfinite(gd).all()


_C3 = {}


def c3_points(torch):
    if "P" not in _C3:
        say("generating 262144 x 1024 mixture points")
        _C3["P"] = synth.gmm_points(262144, 1024, seed=synth.SEEDS["knng_fused"])
        _C3["dev"] = torch.from_numpy(_C3["P"]).cuda()
    return _C3["P"], _C3["dev"]


def test_headline_knng_sampled_rows(h, torch):
    """The headline k-NN graph: 512 sampled rows against the oracle, every row's
    invariants, and the certificate statistics."""
    P, dev = c3_points(torch)
    N, k = P.shape[0], 32
    say("knn_graph 262144 x 1024, k = 32, sample pivots")
    gd, gi = h.graph(dev, k)
    st = h.stats()
    gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
    say(f"  stats: {st}")
    every_row_invariants(gd, gi, N, True)
    _C3["out"] = (gd, gi)
    rows = np.sort(np.random.default_rng(2024).choice(N, 512, replace=False))
    near = compare(P, P, k, gd[rows], gi[rows], rows, self_ids=np.arange(N))
    say(f"  512 rows vs oracle: near-tie rows {near}")
    assert near <= 5
    assert st["rows_uncertified"] == 0


@pytest.mark.parametrize("pivot", ["plain", "learned"])
def test_headline_knng_pivot_rules_same_bits(h, torch, pivot):
    P, dev = c3_points(torch)
    if "out" not in _C3:
        gd, gi = h.graph(dev, 32)
        _C3["out"] = (gd.cpu().numpy(), gi.cpu().numpy())
    say(f"knn_graph 262144 x 1024, k = 32, pivot={pivot}")
    gd, gi = h.graph(dev, 32, pivot=pivot)
    gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
    assert np.array_equal(gi, _C3["out"][1])
    assert np.array_equal(gd.view(np.uint32), _C3["out"][0].view(np.uint32))


_C4 = {}


def c4_setup(torch):
    if "P" not in _C4:
        N, d = 1 << 20, 256
        say("generating 2^20 x 256 mixture points")
        P = synth.gmm_points(N, d, seed=synth.SEEDS["lowprec"])
        _C4["P"] = P
        _C4["dev"] = torch.from_numpy(P).cuda()
        rows = np.sort(np.random.default_rng(4).choice(N, 256, replace=False))
        _C4["rows"] = rows
        say("oracle on 256 rows")
        _C4["oracle"] = oracle.knn(P[rows], P, 65, self_ids=rows)
    return _C4


@pytest.mark.parametrize("prec,min_recall", [("fp32", 1.0), ("bf16", 0.995), ("fp8", 0.95)])
def test_reduced_precision_full_size(h, torch, prec, min_recall):
    """N = 2^20, d = 256, k = 64, k' = 256: recall@k and the error of every
    returned distance on 256 oracle rows; FP32 rows must match the oracle's
    sets outside the near-tie band."""
    c = c4_setup(torch)
    P, dev, rows = c["P"], c["dev"], c["rows"]
    N, k = P.shape[0], 64
    say(f"knn_graph 2^20 x 256, k = 64, {prec}")
    gd, gi = h.graph(dev, k, precision=prec)
    st = h.stats()
    gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
    every_row_invariants(gd, gi, N, True)
    od, oi = c["oracle"]
    hits = sum(len(set(gi[r].tolist()) & set(oi[t, :k].tolist())) for t, r in enumerate(rows))
    recall = hits / (len(rows) * k)
    rel = 0.0
    for r in rows:
        ref = ((P[r].astype(np.float64) - P[gi[r]].astype(np.float64)) ** 2).sum(axis=1)
        rel = max(rel, float(np.max(np.abs(gd[r] - ref) / ref)))
    say(f"  {prec}: recall@{k} {recall:.5f}, max rel distance error {rel:.2e}, certified rows "
        f"{N - st['rows_uncertified']}/{N}, fallback rows {st['fallback_rows']}")
    assert rel <= 1e-5
    assert recall >= min_recall
    if prec == "fp32":
        compare(P, P, k, gd[rows], gi[rows], rows, self_ids=np.arange(N))
