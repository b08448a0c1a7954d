"""Exactness of the FP32 path where the candidate margin is not certified.

A row's kk candidates provably hold its exact k nearest when the gap between
the kk-th and the k-th reduced key exceeds twice the key error bound.  Rows
where it does not (k = kk = 1024, oversample 1, or every row under
KNN_FLAG_FORCE_RERUN) are re-run exactly: every point whose reduced key is
within the bound of the k-th candidate is re-ranked by its exact distance.  The
outputs are compared with the FP64 oracle row by row, and forced re-runs must
reproduce the certified path's bits."""
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
def knn():
    import paper_1309_5478_amd as k
    return k


@pytest.fixture(scope="module")
def h(torch, knn):
    return knn.Handle(0)


def bits(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n,k,over", [(40000, 1024, 4), (40000, 512, 1), (12000, 1024, 4), (2000, 700, 1)])
@pytest.mark.parametrize("flags", [0, 2], ids=["fused", "unfused"])
def test_uncertified_rows_rerun_exactly(h, torch, n, k, over, flags):
    """kk == k leaves no margin: every row is uncertified and re-run; the
    outputs match the oracle on every row (with n = 2000 the threshold sample is
    the whole corpus, so the re-run reads the sample distances)."""
    m, d = 200, 48
    Q = synth.gmm_points(m, d, seed=70 + n)
    C = synth.gmm_points(n, d, seed=71 + n)
    say(f"search n={n} m={m} k={k} oversample={over} flags={flags}")
    gd, gi = h.search(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k, oversample=over, flags=flags)
    st = h.stats()
    say(f"  uncertified {st['rows_uncertified']}, re-run {st['rows_rerun']}")
    assert st["rows_uncertified"] == m and st["rows_rerun"] == m
    near = compare(Q, C, k, gd.cpu().numpy(), gi.cpu().numpy(), np.arange(m))
    assert near <= 4


@pytest.mark.parametrize("n", [1500, 9000, 60000])
@pytest.mark.parametrize("flags", [0, 2], ids=["fused", "unfused"])
def test_forced_rerun_reproduces_certified_bits(h, knn, torch, n, flags):
    """Certified rows and their forced exact re-run give the same bits: both
    are the k smallest exact FP32 distances in (distance, index) order."""
    P = synth.uniform_points(n, 64, seed=90 + n)
    dev = torch.from_numpy(P).cuda()
    base = h.graph(dev, 24, flags=flags)
    st0 = h.stats()
    forced = h.graph(dev, 24, flags=flags | knn.FLAG_FORCE_RERUN)
    st = h.stats()
    say(f"graph n={n} flags={flags}: uncertified {st0['rows_uncertified']}, forced re-run {st['rows_rerun']}")
    assert st["rows_rerun"] == n
    assert np.array_equal(base[1].cpu().numpy(), forced[1].cpu().numpy())
    assert np.array_equal(bits(base[0]), bits(forced[0]))


def test_batch_rerun_matches_per_job_calls(h, knn, torch):
    """Batched jobs with k near 1024 (uncertified) and a forced re-run give the
    same bits as their own knn_search calls."""
    jobs, host = [], []
    for t, (n, d, k) in enumerate([(30000, 64, 1024), (5000, 32, 900), (20000, 96, 40), (1024, 16, 1000)]):
        C = synth.gmm_points(n, d, seed=300 + t)
        Q = synth.gmm_points(128, d, seed=400 + t)
        jobs.append((torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k))
        host.append((Q, C, k))
    for flags in (0, knn.FLAG_FORCE_RERUN):
        got = h.batch_search(jobs, flags=flags)
        torch.cuda.synchronize()
        st = h.stats()
        say(f"batch flags={flags}: uncertified {st['rows_uncertified']}, re-run {st['rows_rerun']}")
        for (q, c, k), (gd, gi) in zip(jobs, got):
            wd, wi = h.search(q, c, min(k, c.shape[0]), flags=flags)
            assert np.array_equal(gi.cpu().numpy(), wi.cpu().numpy())
            assert np.array_equal(bits(gd), bits(wd))
    for (Q, C, k), (gd, gi) in zip(host, got):
        compare(Q, C, k, gd.cpu().numpy()[:32], gi.cpu().numpy()[:32], np.arange(32))


def test_graph_with_nan_point(h, torch):
    """A point with a NaN coordinate: its distances are all NaN, which the total
    order puts above every number, so its neighbours are the lowest other
    indices and it is every other point's farthest neighbour; its own index is
    never returned."""
    P = synth.uniform_points(5000, 32, seed=55)
    P[7, 3] = np.nan
    k = 10
    gd, gi = h.graph(torch.from_numpy(P).cuda(), k)
    gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
    od, oi = oracle.knn(P, P, k, self_ids=np.arange(5000))
    assert np.array_equal(gi[7], oi[7]) and 7 not in gi[7].tolist()
    assert np.isnan(gd[7]).all()
    others = np.array([r for r in range(5000) if r != 7])
    assert not (gi[others] == 7).any()
    near = compare(P, P, k, gd[others[:300]], gi[others[:300]], others[:300], self_ids=np.arange(5000))
    assert near <= 2
