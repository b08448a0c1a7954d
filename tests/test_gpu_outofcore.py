"""knn_search_host_corpus: the corpus in (pinned) host memory, streamed to the
device in partitions whose k nearest are merged (Discussion: partitioning the
data past the device's memory).  FP32 results must equal knn_search on the
whole corpus bit for bit, and the oracle on sampled rows."""
import sys

import numpy as np
import pytest

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
def knn():
    import paper_1309_5478_amd as m
    return m


@pytest.fixture(scope="module")
def h(torch, knn):
    return knn.Handle(0)


def pinned(torch, X):
    t = torch.empty(X.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(X))
    return t


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


@pytest.mark.parametrize("n,m,d,k,part", [
    (40, 30, 8, 5, 3),              # partitions smaller than k
    (2000, 300, 16, 10, 7),         # hundreds of partitions, ragged last one
    (200003, 3000, 64, 32, 65536),  # ragged last partition
    (200003, 3000, 64, 300, 50000),
    (100000, 1000, 33, 1, 30000),   # d not a multiple of 4
])
def test_host_corpus_equals_device_search(h, torch, knn, n, m, d, k, part):
    C = synth.uniform_points(n, d, seed=31 + n)
    Q = synth.uniform_points(m, d, seed=32 + n)
    qd = torch.from_numpy(Q).cuda()
    say(f"host corpus n={n} m={m} d={d} k={k} part_rows={part}")
    gd, gi = h.search_host_corpus(qd, pinned(torch, C), k, part_rows=part)
    torch.cuda.synchronize()
    rd, ri = h.search(qd, torch.from_numpy(C).cuda(), k)
    torch.cuda.synchronize()
    gd, gi, rd, ri = gd.cpu().numpy(), gi.cpu().numpy(), rd.cpu().numpy(), ri.cpu().numpy()
    assert np.array_equal(gi, ri)
    assert np.array_equal(bits(gd), bits(rd))
    rows = np.arange(0, m, max(1, m // 40))
    compare(Q, C, k, gd[rows], gi[rows], rows)


def test_host_corpus_pageable_memory_and_default_partitions(h, torch, knn):
    """A pageable (not pinned) corpus: same result, copies simply do not overlap."""
    C = synth.gmm_points(50000, 128, seed=41)
    Q = synth.gmm_points(500, 128, seed=42)
    qd = torch.from_numpy(Q).cuda()
    gd, gi = h.search_host_corpus(qd, torch.from_numpy(C), 16)
    rd, ri = h.search(qd, torch.from_numpy(C).cuda(), 16)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), ri.cpu().numpy())
    assert np.array_equal(bits(gd.cpu().numpy()), bits(rd.cpu().numpy()))


@pytest.mark.parametrize("metric", ["cosine", "pearson"])
def test_host_corpus_metrics(h, torch, knn, metric):
    C = synth.normal_points(60000, 48, seed=43)
    Q = synth.normal_points(700, 48, seed=44)
    qd = torch.from_numpy(Q).cuda()
    gd, gi = h.search_host_corpus(qd, pinned(torch, C), 24, part_rows=17000, metric=metric)
    rd, ri = h.search(qd, torch.from_numpy(C).cuda(), 24, metric=metric)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), ri.cpu().numpy())
    assert np.array_equal(bits(gd.cpu().numpy()), bits(rd.cpu().numpy()))


def test_host_corpus_large_and_repeated(h, torch, knn):
    """1.5 M points in d = 128 (768 MB) in four partitions, twice in a row on the
    same handle (the second call reuses the buffers), and BF16 products."""
    C = synth.gmm_points(1500000, 128, seed=45)
    Q = synth.gmm_points(4096, 128, seed=46)
    qd = torch.from_numpy(Q).cuda()
    Cp = pinned(torch, C)
    a = h.search_host_corpus(qd, Cp, 32, part_rows=400000)
    b = h.search_host_corpus(qd, Cp, 32, part_rows=400000)
    rd, ri = h.search(qd, torch.from_numpy(C).cuda(), 32)
    torch.cuda.synchronize()
    for gd, gi in (a, b):
        assert np.array_equal(gi.cpu().numpy(), ri.cpu().numpy())
        assert np.array_equal(bits(gd.cpu().numpy()), bits(rd.cpu().numpy()))
    rows = np.arange(0, 4096, 128)
    compare(Q, C, 32, a[0].cpu().numpy()[rows], a[1].cpu().numpy()[rows], rows)
    bd, bi = h.search_host_corpus(qd, Cp, 32, part_rows=400000, precision="bf16")
    torch.cuda.synchronize()
    bi = bi.cpu().numpy()
    ri = ri.cpu().numpy()
    recall = np.mean([len(set(bi[r]) & set(ri[r])) / 32 for r in range(0, 4096, 8)])
    say(f"bf16 host-corpus recall vs FP32: {recall:.4f}")
    assert recall >= 0.99


def test_host_corpus_argument_errors(h, torch, knn):
    qd = torch.zeros((4, 8), device="cuda")
    C = torch.zeros((100, 8))
    with pytest.raises(knn.KnnError):
        h.search_host_corpus(qd, C, 101)
    with pytest.raises(knn.KnnError):
        h.search_host_corpus(qd, C, 5, part_rows=-1)
