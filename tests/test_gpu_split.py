"""Few long rows: knn_select_k splits each row across workgroups and merges the
parts' key lists (Results, Figure 8 and Discussion: the GPU is saturated only
with enough rows in flight).  The output must equal the oracle's bit for bit,
split or not, with values only or with indices."""
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
def knn():
    import paper_1309_5478_amd as m
    return m


@pytest.fixture(scope="module")
def h(torch, knn):
    return knn.Handle(0)


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def run(h, torch, knn, D, k, flags=0, pivot="sample", indices=True, dev=None):
    dev = torch.from_numpy(D).cuda() if dev is None else dev
    v, i = h.select_k(dev, k, pivot=pivot, flags=flags, indices=indices)
    torch.cuda.synchronize()
    st = h.stats()
    return v.cpu().numpy(), (i.cpu().numpy() if i is not None else None), st


def assert_oracle(D, k, gv, gi, rows=None):
    ov, oi = oracle.select_k(D, k, rows=rows)
    if rows is not None:
        gv = gv[rows]
        gi = gi[rows] if gi is not None else None
    bad = (bits(gv) != bits(ov)).any(axis=1)
    if gi is not None:
        bad |= (gi != oi).any(axis=1)
    bad = np.nonzero(bad)[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5]}"


@pytest.mark.parametrize("rows,cols", [(1, 8192), (3, 65536 + 13), (8, 200003), (5, 1 << 20)])
@pytest.mark.parametrize("pivot", ["sample", "plain", "learned"])
def test_split_matches_oracle(h, torch, knn, rows, cols, pivot):
    rng = np.random.default_rng(rows * 7 + cols)
    D = rng.random((rows, cols), dtype=np.float32)
    dev = torch.from_numpy(D).cuda()
    for k in (1, 32, 100, 256, 1000, 1024):
        say(f"split rows={rows} cols={cols} k={k} pivot={pivot}")
        gv, gi, st = run(h, torch, knn, D, k, pivot=pivot, dev=dev)
        if cols >= 2 * max(65536, 32 * k):
            assert st["split_parts"] > 1, st
        assert st["rows"] == rows
        assert_oracle(D, k, gv, gi)
        nv, ni, nst = run(h, torch, knn, D, k, flags=knn.FLAG_NO_SPLIT, pivot=pivot, dev=dev)
        assert nst["split_parts"] == 1
        assert np.array_equal(bits(nv), bits(gv)) and np.array_equal(ni, gi)
        # forced: parts down to max(4096, 32 k) columns
        fv, fi, fst = run(h, torch, knn, D, k, flags=knn.FLAG_FORCE_SPLIT, pivot=pivot, dev=dev)
        if cols >= 2 * max(4096, 32 * k):
            assert fst["split_parts"] > 1, fst
        assert np.array_equal(bits(fv), bits(gv)) and np.array_equal(fi, gi)


def test_split_special_values_keep_their_bits(h, torch, knn):
    """Zeros of both signs, NaNs with payloads, infinities and long runs of
    equal values, across part boundaries: the merged result copies each
    selected value verbatim and resolves ties to the lower column."""
    cols = 65536 + 5
    D = np.random.default_rng(3).integers(0, 4, size=(6, cols)).astype(np.float32)
    D[0, ::3] = -0.0
    D[0, 1::3] = 0.0
    nan_payload = np.array([0x7fc00123, 0xffc00456, 0x7f800001], np.uint32).view(np.float32)
    D[1, :] = np.inf
    D[1, 5000::7] = nan_payload[np.arange(len(D[1, 5000::7])) % 3]
    D[1, 40000] = -np.inf
    D[2, :] = np.nan
    D[3, :] = 2.0
    D[4, 16383:16390] = -1.0                 # a run across the first part boundary
    D[5, ::2] = np.float32(-0.0)
    for k in (1, 7, 64, 500, 1024):
        gv, gi, st = run(h, torch, knn, D, k, flags=knn.FLAG_FORCE_SPLIT)
        assert st["split_parts"] > 1
        assert_oracle(D, k, gv, gi)


def test_force_split_many_rows_and_layouts(h, torch, knn):
    """FORCE_SPLIT with more rows than the device holds at once, a padded row
    stride and a base that is not 16-byte aligned."""
    D = synth.sqdist_matrix_normal(700, 16384 + 9, 32, seed=11)
    for k in (16, 256):
        gv, gi, st = run(h, torch, knn, D, k, flags=knn.FLAG_FORCE_SPLIT)
        assert st["split_parts"] == (4 if k == 16 else 2)
        assert_oracle(D, k, gv, gi)
    R, C = D.shape
    for pad, off in ((3, 0), (0, 1)):
        host = np.zeros(off + R * (C + pad), np.float32)
        host[off:].reshape(R, C + pad)[:, :C] = D
        dev = torch.from_numpy(host).cuda()[off:].view(R, C + pad)[:, :C]
        v, i = h.select_k(dev, 100, flags=knn.FLAG_FORCE_SPLIT)
        assert h.stats()["split_parts"] == 4
        assert_oracle(D, 100, v.cpu().numpy(), i.cpu().numpy())


@pytest.mark.parametrize("split", [0, "force", "none"])
def test_values_only(h, torch, knn, split):
    """out_idx = NULL: the same values, bit for bit, without indices."""
    flags = {0: 0, "force": knn.FLAG_FORCE_SPLIT, "none": knn.FLAG_NO_SPLIT}[split]
    D = synth.sqdist_matrix_normal(40, 40000, 16, seed=12)
    D[3, ::5] = -0.0
    for k in (1, 33, 1024):
        gv, gi, _ = run(h, torch, knn, D, k, flags=flags, indices=False)
        assert gi is None
        assert_oracle(D, k, gv, None)


def test_saturation_shape_q8_bit_exact(h, torch, knn):
    """The paper's saturation workload shape, n = 2^20 columns of uniform
    values, at Q = 8 rows (split), largest k: bit-exact on every row."""
    D = synth.uniform_points(8, 1 << 20, seed=synth.SEEDS["sweep"])
    for k in (32, 1024):
        gv, gi, st = run(h, torch, knn, D, k)
        say(f"Q=8 n=2^20 k={k}: split_parts={st['split_parts']}")
        assert st["split_parts"] > 1
        assert_oracle(D, k, gv, gi)


def test_split_flag_errors(h, torch, knn):
    D = torch.zeros((2, 10000), device="cuda")
    with pytest.raises(knn.KnnError):
        h.select_k(D, 5, flags=knn.FLAG_NO_SPLIT | knn.FLAG_FORCE_SPLIT)
