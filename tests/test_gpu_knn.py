"""Parity of knn_search / knn_graph / knn_distances (HIP, MFMA) with the FP64
CPU oracle.

Bar: neighbour sets equal per row, except where the oracle's FP64 gap between
the k-th and the (k+1)-th distance is within the 1e-5 relative band (counted
and reported, not failed); returned squared distances within 1e-5 relative of
FP64 (1e-6 of ||q||^2 + ||c||^2 for exact zeros); rows in ascending
(distance, index) order."""
import sys

import numpy as np
import pytest

import oracle
import synth
from knn_check import REL, compare, d64  # noqa: F401

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


def run_graph(h, torch, P, k, **kw):
    dev = torch.from_numpy(P).cuda()
    gd, gi = h.graph(dev, k, **kw)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gi.cpu().numpy()


def run_search(h, torch, Q, C, k, **kw):
    gd, gi = h.search(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda(), k, **kw)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gi.cpu().numpy()


MODES = [dict(), dict(flags=2), dict(flags=1)]          # fused, unfused, forced exact fallback
MODE_IDS = ["fused", "unfused", "fallback"]


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_graph_uniform_4096_all_rows(h, torch, mode):
    """N = M = 4096 uniform[0,1) points, d = 128, k = 16, own index excluded:
    every row against the oracle."""
    P = synth.uniform_points(4096, 128, seed=synth.SEEDS["knng_small"])
    say(f"graph 4096x128 k=16 mode={mode}")
    gd, gi = run_graph(h, torch, P, 16, **mode)
    near = compare(P, P, 16, gd, gi, np.arange(4096), self_ids=np.arange(4096))
    say(f"  near-tie rows: {near}  stats: {h.stats()}")
    assert near <= 8


@pytest.mark.parametrize("n,m,d,k", [(2, 1, 1, 1), (3, 5, 3, 2), (65, 7, 5, 9), (129, 130, 17, 64),
                                     (1000, 33, 130, 100), (2049, 64, 64, 1), (5000, 300, 33, 250),
                                     (3001, 257, 256, 1024)])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_search_ragged_shapes(h, torch, n, m, d, k, mode):
    k = min(k, n)
    Q = synth.normal_points(m, d, seed=11 + n)
    C = synth.normal_points(n, d, seed=12 + n)
    say(f"search n={n} m={m} d={d} k={k} mode={mode}")
    gd, gi = run_search(h, torch, Q, C, k, **mode)
    near = compare(Q, C, k, gd, gi, np.arange(m))
    assert near <= max(2, m // 50)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_integer_lattice_bit_exact(h, torch, mode):
    """Integer coordinates in [0, 8): every product and partial sum is exact in
    FP32, so distances, sets and the tie order (lower index first, with massive
    ties) must equal the oracle exactly."""
    rng = np.random.default_rng(7)
    P = rng.integers(0, 8, size=(3000, 24)).astype(np.float32)
    P[100] = P[5]          # exact duplicates: distance 0, kept as neighbours
    P[2999] = P[5]
    k = 40
    gd, gi = run_graph(h, torch, P, k, **mode)
    od, oi = oracle.knn(P, P, k, self_ids=np.arange(3000))
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd.astype(np.float64), od)
    assert gi[5, 0] == 100 and gi[5, 1] == 2999 and gd[5, 0] == 0.0


def test_duplicates_and_self_exclusion(h, torch):
    P = synth.uniform_points(700, 9, seed=3)
    P[10:20] = P[10]                   # ten identical points
    gd, gi = run_graph(h, torch, P, 12)
    for r in range(10, 20):
        assert r not in gi[r]
        assert set(range(10, 20)) - {r} <= set(gi[r].tolist())
        assert (gd[r, :9] == 0.0).all()


def test_knn_distances_norm_correction(h, torch):
    """The matrix-core norm expansion ||q||^2 + ||c||^2 - 2 q.c against FP64
    direct distances on sampled pairs, within the FP32 expansion's error bound
    2 * gamma_d * sum|q_t c_t| + (norm errors), gamma_d = d u / (1 - d u)."""
    Q = synth.gmm_points(512, 256, seed=21)
    C = synth.gmm_points(3000, 256, seed=22)
    D = h.distances(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda()).cpu().numpy()
    rng = np.random.default_rng(0)
    u = 2.0 ** -24
    dd = Q.shape[1]
    gamma = dd * u / (1 - dd * u)
    for _ in range(2000):
        i, j = int(rng.integers(512)), int(rng.integers(3000))
        ref = d64(Q[i], C[j])
        bound = 2 * gamma * float(np.abs(Q[i].astype(np.float64) * C[j]).sum()) \
            + 2 * gamma * (float(np.dot(Q[i].astype(np.float64), Q[i])) + float(np.dot(C[j].astype(np.float64), C[j])))
        assert abs(float(D[i, j]) - ref) <= bound, (i, j, float(D[i, j]), ref, bound)


def test_distances_feed_select_k_like_the_two_step_pipeline(h, torch):
    Q = synth.uniform_points(200, 40, seed=31)
    C = synth.uniform_points(5000, 40, seed=32)
    D = h.distances(torch.from_numpy(Q).cuda(), torch.from_numpy(C).cuda())
    v, i = h.select_k(D, 20)
    Dh = D.cpu().numpy()
    ov, oi = oracle.select_k(Dh, 20)
    assert np.array_equal(i.cpu().numpy(), oi)


def test_search_errors(h, torch):
    import paper_1309_5478_amd as knn
    Q = torch.zeros((4, 8), device="cuda")
    C = torch.zeros((10, 8), device="cuda")
    for bad, st in [(dict(k=0), 1), (dict(k=11), 1), (dict(k=1025), 1)]:
        with pytest.raises(knn.KnnError) as ei:
            h.search(Q, C, **bad)
        assert ei.value.status == st
    with pytest.raises(knn.KnnError) as ei:
        h.graph(C, 10)
    assert ei.value.status == 1


@pytest.mark.parametrize("seed", [1, 2])
def test_repeat_determinism(h, torch, seed):
    P = synth.gmm_points(6000, 64, seed=seed)
    a = run_graph(h, torch, P, 32)
    b = run_graph(h, torch, P, 32)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_tile_shapes_give_identical_bits(h, torch, prec):
    """The product's tile shape (and operand stage count) changes no output bit:
    every element's dot product accumulates in the same order."""
    import os
    P = synth.gmm_points(4096, 160, seed=synth.SEEDS["knng_small"] + 50)
    dev = torch.from_numpy(P).cuda()
    outs = {}
    old = os.environ.get("KNN_GEMM_TILE")
    try:
        for tile in ("small", "small1", "wide", "big"):
            if tile == "big" and prec == "fp8":
                continue
            os.environ["KNN_GEMM_TILE"] = tile
            d, i = h.graph(dev, 20, precision=prec)
            dm = h.distances(dev[:512], dev)
            torch.cuda.synchronize()
            outs[tile] = (d.cpu().numpy().view(np.uint32), i.cpu().numpy(), dm.cpu().numpy().view(np.uint32))
    finally:
        if old is None:
            os.environ.pop("KNN_GEMM_TILE", None)
        else:
            os.environ["KNN_GEMM_TILE"] = old
    ref = outs["small"]
    for tile, o in outs.items():
        for a, b in zip(o, ref):
            assert np.array_equal(a, b), (prec, tile)


def test_autotuned_tile_gives_identical_bits(h, torch, tmp_path):
    """KNN_FLAG_AUTOTUNE times the tile shapes on the call's operands (with a
    threshold that keeps nothing), records the choice in the cache file and
    returns the same bits as the default shape."""
    import os
    import paper_1309_5478_amd as knn
    P = synth.gmm_points(6000, 96, seed=synth.SEEDS["knng_small"] + 60)
    dev = torch.from_numpy(P).cuda()
    base = h.graph(dev, 12)
    path = str(tmp_path / "tune.json")
    os.environ["KNN_AUTOTUNE_CACHE"] = path
    try:
        tuned = h.graph(dev, 12, flags=knn.FLAG_AUTOTUNE)
        again = h.graph(dev, 12, flags=knn.FLAG_AUTOTUNE)   # cached choice
        torch.cuda.synchronize()
        assert "fused|" in open(path).read()
    finally:
        del os.environ["KNN_AUTOTUNE_CACHE"]
    for got in (tuned, again):
        assert np.array_equal(got[1].cpu().numpy(), base[1].cpu().numpy())
        assert np.array_equal(got[0].cpu().numpy().view(np.uint32), base[0].cpu().numpy().view(np.uint32))
