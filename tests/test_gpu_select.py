"""Parity of the HIP selection path (knn_select_k, knn_partition) with the CPU
oracle: bit-exact indices and value bits."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

PIVOTS = ("plain", "sample", "learned")


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


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def check_select(h, torch, D, k, pivot, rows=None, ld_pad=0, offset=0, tag="", flags=0):
    """Runs knn_select_k on D (optionally with padded rows / a misaligned base)
    and compares with the oracle on every (or the listed) row."""
    say(f"select_k {tag} shape={D.shape} k={k} pivot={pivot} ld_pad={ld_pad} offset={offset}")
    R, C = D.shape
    host = np.zeros(offset + R * (C + ld_pad), np.float32)
    view = host[offset:offset + R * (C + ld_pad)].reshape(R, C + ld_pad)
    view[:, :C] = D
    dev = torch.from_numpy(host).cuda()
    dmat = dev[offset:offset + R * (C + ld_pad)].view(R, C + ld_pad)[:, :C]
    vals, idx = h.select_k(dmat, k, pivot=pivot, flags=flags)
    torch.cuda.synchronize()
    gv, gi = vals.cpu().numpy(), idx.cpu().numpy()
    ov, oi = oracle.select_k(D, k, rows=rows)
    if rows is not None:
        gv, gi = gv[rows], gi[rows]
    bad = np.nonzero((gi != oi).any(axis=1) | (bits(gv) != bits(ov)).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5]}"
    st = h.stats()
    assert st["rows"] == R
    return st


@pytest.mark.parametrize("cols", [1, 5, 63, 64, 65, 1000, 1024, 1025, 2049, 4097, 10007, 65543])
@pytest.mark.parametrize("pivot", PIVOTS)
def test_select_random_sizes(h, torch, cols, pivot):
    rng = np.random.default_rng(cols)
    D = rng.standard_normal((37, cols)).astype(np.float32)
    for k in sorted({1, 7, 32, 64, 65, 256, 1000, 1024, cols} & set(range(1, min(cols, 1024) + 1))):
        check_select(h, torch, D, k, pivot, tag="random")


@pytest.mark.parametrize("cols", [1025, 2047, 2048, 2049, 2300, 4100])
def test_select_around_two_buffers(h, torch, cols):
    """Rows whose survivors straddle one LDS buffer (1024 keys), both buffers
    (2048) and the workspace beyond, at k where the finish sorts the streamed
    run in place (k >= 512), sorts it after it moved (k < 512) or runs the
    partition passes; sample and network pivots, plus adversarial rows."""
    rng = np.random.default_rng(cols + 17)
    D = np.concatenate([rng.standard_normal((24, cols)).astype(np.float32),
                        np.stack(list(synth.adversarial_rows(cols, seed=cols).values()))])
    for k in sorted({300, 511, 512, 700, 1000, 1024} & set(range(1, min(cols, 1024) + 1))):
        for pivot in ("sample", "learned"):
            check_select(h, torch, D, k, pivot, tag="two-buffer")


@pytest.mark.parametrize("cols", [3000, 70001])
@pytest.mark.parametrize("pivot", PIVOTS)
def test_select_adversarial_rows(h, torch, cols, pivot):
    adv = synth.adversarial_rows(cols, seed=12)
    names = sorted(adv)
    D = np.stack([adv[n] for n in names])
    for k in (1, 32, 333, 1024):
        check_select(h, torch, D, k, pivot, tag="adversarial:" + ",".join(names))


@pytest.mark.parametrize("cols", [65536, 70003])
def test_select_band_restreams(h, torch, cols):
    """Rows whose strided pivot sample (16 blocks of 64 entries at evenly spaced
    starts) holds their smallest values: the first pivot keeps fewer than k keys,
    so the row is streamed again for the next band of values, several times
    (Methods: when fewer than k keys lie below the pivot they are all kept and
    the search goes on above them).  Aligned rows take the tiled stream, the
    misaligned base the generic one.  Rows whole (not split), so that each one's
    sample is the one built here."""
    import paper_1309_5478_amd as knn
    rng = np.random.default_rng(21)
    D = rng.uniform(1.0, 2.0, size=(8, cols)).astype(np.float32)
    starts = [(b * (cols - 64)) // 15 for b in range(16)]
    for r in range(8):
        for s0 in starts:
            D[r, s0:s0 + 64] = rng.uniform(0.0, 1e-3, 64)
    D[1] = np.round(D[1] * 4) / 4          # ties at every band edge
    D[2, starts[3]:starts[3] + 64] = -0.0
    D[3, starts[5]:starts[5] + 64] = 0.0
    for k in (32, 256, 1024):
        st = check_select(h, torch, D, k, "sample", tag="band", flags=knn.FLAG_NO_SPLIT)
        assert st["stream_passes_total"] > D.shape[0], "no row was streamed twice"
        check_select(h, torch, D, k, "sample", offset=1, tag="band misaligned", flags=knn.FLAG_NO_SPLIT)
        check_select(h, torch, D, k, "sample", tag="band, split rows")


@pytest.mark.parametrize("pivot", PIVOTS)
def test_select_heavy_ties_and_layout(h, torch, pivot):
    rng = np.random.default_rng(5)
    D = rng.integers(0, 3, size=(20, 9000)).astype(np.float32)   # thousands of equal values
    D[3] = 1.0
    D[4, ::2] = -0.0
    for k in (1, 100, 1024):
        check_select(h, torch, D, k, pivot, tag="ties")
        check_select(h, torch, D, k, pivot, ld_pad=3, tag="ld+3")
        check_select(h, torch, D, k, pivot, ld_pad=0, offset=1, tag="misaligned")


def test_select_pivot_independence_and_repeat(h, torch):
    D = synth.sqdist_matrix_normal(300, 20000, 64, seed=2)
    dev = torch.from_numpy(D).cuda()
    outs = []
    for pivot in PIVOTS * 2:
        v, i = h.select_k(dev, 256, pivot=pivot)
        outs.append((bits(v.cpu().numpy()).copy(), i.cpu().numpy().copy()))
    for v, i in outs[1:]:
        assert np.array_equal(v, outs[0][0]) and np.array_equal(i, outs[0][1])


def test_select_empty_rows_is_noop(h, torch):
    D = torch.zeros((0, 100), device="cuda")
    v, i = h.select_k(D, 5)
    assert v.shape == (0, 5)


def test_select_argument_errors_leave_outputs(h, torch):
    import paper_1309_5478_amd as knn
    lib = h.lib
    D = torch.ones((4, 16), device="cuda")
    out_v = torch.full((4, 8), 7.0, device="cuda")
    out_i = torch.full((4, 8), 7, dtype=torch.int32, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    cases = [
        (dict(rows=-1), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(cols=0), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(ld=15), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(k=0), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(k=17), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(dist=None), knn._abi.KNN_ERROR_INVALID_VALUE),
        (dict(cols=2000, ld=2000, k=1025), knn._abi.KNN_ERROR_UNSUPPORTED),
        (dict(cols=1 << 31, ld=1 << 31), knn._abi.KNN_ERROR_UNSUPPORTED),
    ]
    for over, want in cases:
        a = dict(dist=p(D), rows=4, cols=16, ld=16, k=8)
        a.update(over)
        st = lib.knn_select_k(h.h, a["dist"], a["rows"], a["cols"], a["ld"], a["k"], p(out_v), p(out_i), None, None)
        assert st == want, (over, st, lib.knn_last_error(h.h))
    torch.cuda.synchronize()
    assert bool((out_v == 7.0).all()) and bool((out_i == 7).all())


@pytest.mark.parametrize("cols", [1, 4, 63, 64, 65, 200, 4099])
def test_partition_matches_oracle(h, torch, cols):
    rng = np.random.default_rng(cols)
    R = 9
    X = rng.integers(0, 7, size=(R, cols)).astype(np.float32)
    X[0, ::3] = np.nan
    X[1, ::2] = -0.0
    pj = rng.integers(0, cols, size=R).astype(np.int32)
    pv = X[np.arange(R), pj].copy()
    pv[2] = np.nan                    # pivot in the NaN class
    pv[3] = 3.5                       # a value between the classes
    say(f"partition cols={cols}")
    ov, oi, L = h.partition(torch.from_numpy(X).cuda(), torch.from_numpy(pv), torch.from_numpy(pj))
    ov, oi, L = ov.cpu().numpy(), oi.cpu().numpy(), L.cpu().numpy()
    for r in range(R):
        ev, ei, eL = oracle.partition(X[r], np.arange(cols, dtype=np.int32), float(pv[r]), int(pj[r]))
        assert L[r] == eL
        assert np.array_equal(oi[r], ei)
        assert np.array_equal(bits(ov[r]), bits(ev))


def test_partition_golden_example(h, torch):
    from golden_io import partition_cases
    for vals, piv, lanes, L in partition_cases():
        x = torch.tensor([vals], dtype=torch.float32, device="cuda")
        ov, oi, got_L = h.partition(x, torch.tensor([piv]), torch.tensor([1 << 30], dtype=torch.int32))
        assert int(got_L[0]) == L
        assert oi[0].cpu().tolist() == lanes


@pytest.mark.parametrize("k", [32, 256, 1024])
def test_select_full_size_all_rows(h, torch, k):
    """16384 x 65536 squared distances of N(0,1) points in d=256: every row
    bit-exact against the oracle, with each pivot rule."""
    M, N, d = 16384, 65536, 256
    D = _full_matrix(M, N, d)
    dev = _full_matrix_dev(torch, D)
    ov, oi = _full_oracle(D)        # first 1024 of each row's stable sort
    say(f"select_k full size k={k}")
    for pivot in PIVOTS:
        v, i = h.select_k(dev, k, pivot=pivot)
        torch.cuda.synchronize()
        gv, gi = v.cpu().numpy(), i.cpu().numpy()
        st = h.stats()
        say(f"  pivot={pivot} stats={st}")
        bad = np.nonzero((gi != oi[:, :k]).any(axis=1) | (bits(gv) != bits(ov[:, :k])).any(axis=1))[0]
        assert bad.size == 0, f"pivot={pivot}: {bad.size} of {M} rows differ, first {bad[:5]}"
        # the k-th value bounds the selection: nothing unselected lies below it
        kth = gv[:, k - 1:k]
        assert ((D < kth).sum(axis=1) <= k - 1).all()
        assert ((D <= kth).sum(axis=1) >= k).all()


_CACHE = {}


def _full_matrix(M, N, d):
    if "D" not in _CACHE:
        say("generating the 16384 x 65536 select matrix")
        _CACHE["D"] = synth.sqdist_matrix_normal(M, N, d, seed=synth.SEEDS["select"])
    return _CACHE["D"]


def _full_oracle(D):
    if "oracle" not in _CACHE:
        say("oracle: every row of the 16384 x 65536 matrix")
        _CACHE["oracle"] = oracle.select_k(D, 1024)
    return _CACHE["oracle"]


def _full_matrix_dev(torch, D):
    if "dev" not in _CACHE:
        _CACHE["dev"] = torch.from_numpy(D).cuda()
    return _CACHE["dev"]
