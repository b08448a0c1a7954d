"""The resident-corpus product for short BF16 / FP8 rows (gemm_sk.hip) against
the tiled product (KNN_GEMM_SK=0): both form the reduced keys with the same MFMA
sequence, so every search and graph result must be the same bits; the FP32
re-rank then makes both exact where their candidates hold the true neighbours."""
import os
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
def h(torch):
    import paper_1309_5478_amd as knn
    return knn.Handle(0)


def run(h, torch, Q, C, k, prec, sk, graph=False):
    os.environ["KNN_GEMM_SK"] = "1" if sk else "0"
    try:
        if graph:
            d, i = h.graph(torch.from_numpy(C).cuda(), k, precision=prec)
        else:
            d, i = h.search(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k, precision=prec)
        torch.cuda.synchronize()
    finally:
        del os.environ["KNN_GEMM_SK"]
    return d.cpu().numpy(), i.cpu().numpy()


@pytest.mark.parametrize("prec,d", [("bf16", 256), ("bf16", 100), ("bf16", 128), ("fp8", 128), ("fp8", 77),
                                    ("fp8", 256), ("fp8", 200)])
@pytest.mark.parametrize("graph", [False, True])
def test_sk_equals_tiled(h, torch, prec, d, graph):
    """Ragged sizes (rows not a multiple of 64, columns not of 256), mixture data,
    k from 1 to 300."""
    m, n = 3001, 40000 + 37
    C = synth.gmm_points(n, d, seed=71 + d)
    Q = C if graph else synth.gmm_points(m, d, seed=72 + d)
    for k in (1, 16, 300):
        say(f"sk vs tiled: {prec} d={d} graph={graph} k={k}")
        a = run(h, torch, Q, C, k, prec, True, graph)
        b = run(h, torch, Q, C, k, prec, False, graph)
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


def test_sk_lattice_exact(h, torch):
    """Integer lattice points: every product is exact in BF16, so the resident
    product must give the oracle's sets and distances exactly (massive ties)."""
    rng = np.random.default_rng(5)
    P = rng.integers(0, 8, size=(6000, 192)).astype(np.float32)
    P[100:110] = P[5]                      # duplicates at distance 0
    gd, gi = run(h, torch, None, P, 20, "bf16", True, graph=True)
    rows = np.arange(0, 6000, 97)
    compare(P, P, 20, gd[rows], gi[rows], rows, self_ids=np.arange(6000))


@pytest.mark.parametrize("prec,d", [("bf16", 256), ("fp8", 200)])
@pytest.mark.parametrize("stage", ["0", "64"])
def test_sk_staging_forms(h, torch, prec, d, stage):
    """The kept keys staged per wave (the default), appended to the rows in the
    product itself (KNN_SK_STAGE=0), and staged with room for only 64 keys per
    wave, so that most go to the rows directly once a wave's part is full: the
    same candidate sets, so the same bits."""
    n = 20000 + 17
    C = synth.gmm_points(n, d, seed=90 + d)
    Q = synth.gmm_points(2000 + 3, d, seed=91 + d)
    for graph in (False, True):
        for k in (16, 300):
            say(f"sk staging {stage}: {prec} d={d} graph={graph} k={k}")
            a = run(h, torch, Q, C, k, prec, True, graph)
            var = "KNN_SK_STAGE" if stage == "0" else "KNN_SK_STAGE_KEYS"
            os.environ[var] = stage
            try:
                b = run(h, torch, Q, C, k, prec, True, graph)
            finally:
                del os.environ[var]
            assert np.array_equal(a[1], b[1])
            assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
