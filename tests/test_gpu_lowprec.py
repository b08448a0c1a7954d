"""Reduced-precision distance products (BF16, FP8 e4m3 with per-point scales)
with FP32 exact re-rank: exactness where the inputs are exactly representable,
and recall / distance error against the FP64 oracle where they are not."""
import sys

import numpy as np
import pytest

import oracle
import synth

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


MODES = [dict(), dict(flags=2), dict(flags=1)]
MODE_IDS = ["fused", "unfused", "fallback"]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_integer_lattice_exact(h, torch, prec, mode):
    """Coordinates in {0..7}: exact in BF16 and (scaled by 64) in e4m3, products
    and sums exact in FP32 at d = 24, so sets, order and distances equal the
    oracle's, massive ties included."""
    rng = np.random.default_rng(8)
    P = rng.integers(0, 8, size=(2500, 24)).astype(np.float32)
    P[7] = P[1]
    say(f"lattice prec={prec} mode={mode}")
    gd, gi = h.graph(torch.from_numpy(P).cuda(), 24, precision=prec, **mode)
    od, oi = oracle.knn(P, P, 24, self_ids=np.arange(2500))
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy().astype(np.float64), od)


@pytest.mark.parametrize("prec,min_recall", [("fp32", 1.0), ("bf16", 0.99), ("fp8", 0.9)])
def test_gmm_recall_and_distance_error(h, torch, prec, min_recall):
    """65536 mixture points in d = 256, k = 64, k' = 256: recall@k against the
    FP64 oracle on sampled rows, and the error of every returned distance."""
    N, d, k = 65536, 256, 64
    P = synth.gmm_points(N, d, seed=synth.SEEDS["lowprec"] + 100)
    gd, gi = h.graph(torch.from_numpy(P).cuda(), k, precision=prec)
    st = h.stats()
    gd, gi = gd.cpu().numpy(), gi.cpu().numpy()
    rows = np.random.default_rng(1).choice(N, 96, replace=False)
    od, oi = oracle.knn(P[rows], P, k, self_ids=rows)
    hits = sum(len(set(gi[r].tolist()) & set(oi[t].tolist())) for t, r in enumerate(rows))
    recall = hits / (len(rows) * k)
    rel = 0.0
    for t, r in enumerate(rows):
        ref = ((P[r].astype(np.float64) - P[gi[r]].astype(np.float64)) ** 2).sum(axis=1)
        rel = max(rel, float(np.max(np.abs(gd[r] - ref) / ref)))
    say(f"{prec}: recall@{k} {recall:.5f}, max rel distance error {rel:.2e}, "
        f"uncertified rows {st['rows_uncertified']}/{N}, fallback rows {st['fallback_rows']}")
    assert recall >= min_recall
    assert rel <= 1e-5
