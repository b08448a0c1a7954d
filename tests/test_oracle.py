"""Pins for the CPU oracle: brute force, hand-worked examples, closed forms,
library special cases and invariants.  CPU only."""
import math
import struct

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth
from brute import knn_pairwise, select_by_subsets
from golden_io import lattice_cases, partition_cases, select_cases


def bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


# ---------------------------------------------------------------- selection
@pytest.mark.parametrize("vals,k,idx,vbits", list(select_cases()))
def test_select_hand_examples(vals, k, idx, vbits):
    v, i = oracle.select_k(np.array([vals], np.float32), k)
    assert i[0].tolist() == idx
    got = bits(v[0]).tolist()
    # NaN payloads are compared as "is NaN"; every other value bit for bit
    for g, e in zip(got, vbits):
        ef = struct.unpack("<f", struct.pack("<I", e))[0]
        if math.isnan(ef):
            assert math.isnan(struct.unpack("<f", struct.pack("<I", g))[0])
        else:
            assert g == e


_POOL = np.array([0.0, -0.0, 1.0, 1.0, 2.5, -3.0, np.inf, -np.inf, np.nan, 7.0], np.float32)


@pytest.mark.parametrize("seed", range(40))
def test_select_matches_subset_enumeration(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 10))
    row = rng.choice(_POOL, size=n).astype(np.float32)
    for k in range(1, n + 1):
        v, i = oracle.select_k(row[None, :], k)
        expect = select_by_subsets([float(x) for x in row], k)
        assert i[0].tolist() == expect, (row, k)
        # verbatim values: bits equal to the input's at the chosen indices
        assert bits(v[0]).tolist() == bits(row[expect]).tolist()


@pytest.mark.parametrize("seed", range(6))
def test_select_matches_numpy_stable_argsort(seed):
    # numpy's stable sort orders -0/+0 as equal and puts NaN last, i.e. the
    # same total order; a full stable argsort's prefix is the k-smallest list.
    rng = np.random.default_rng(100 + seed)
    cols = int(rng.integers(50, 3000))
    D = rng.integers(0, 40, size=(7, cols)).astype(np.float32)   # many ties
    D[0, ::7] = np.nan
    D[1, ::5] = -0.0
    D[2, ::3] = -np.inf
    for k in (1, 2, 17, cols):
        v, i = oracle.select_k(D, k)
        ref = np.argsort(D, axis=1, kind="stable")[:, :k]
        assert np.array_equal(i, ref)


def test_select_k1_is_first_argmin():
    rng = np.random.default_rng(7)
    D = rng.integers(0, 5, size=(50, 200)).astype(np.float32)
    _, i = oracle.select_k(D, 1)
    assert np.array_equal(i[:, 0], np.argmin(D, axis=1))     # argmin returns the first occurrence


def test_select_row_subset_and_invariants():
    D = synth.sqdist_matrix_normal(64, 3000, 32, seed=9)
    rows = np.array([5, 0, 63, 17])
    v_all, i_all = oracle.select_k(D, 40)
    v_sub, i_sub = oracle.select_k(D, 40, rows=rows)
    assert np.array_equal(i_sub, i_all[rows])
    for r in range(D.shape[0]):
        sel = set(i_all[r].tolist())
        assert len(sel) == 40 and all(0 <= c < D.shape[1] for c in sel)
        assert np.all(np.diff(v_all[r]) >= 0)                    # ascending
        kth = v_all[r, -1]
        rest = np.delete(D[r], i_all[r])
        assert np.all(rest >= kth)                                # k-th bounds every selected entry
        # entries equal to the k-th value left out all have higher indices
        tied_out = np.nonzero(D[r] == kth)[0]
        tied_out = [c for c in tied_out if c not in sel]
        assert all(c > max(j for j in sel if D[r, j] == kth) for c in tied_out)


@pytest.mark.parametrize("vals,piv,lanes,L", list(partition_cases()))
def test_partition_example(vals, piv, lanes, L):
    v = np.array(vals, np.float32)
    # the pivot key (value, index) with index past every element: a pure value pivot
    out_v, out_i, got_L = oracle.partition(v, np.arange(len(v), dtype=np.int32), piv, 1 << 30)
    assert got_L == L
    assert out_i.tolist() == lanes
    assert np.array_equal(out_v, v[lanes])


def test_partition_is_a_permutation_split_at_pivot():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 10, 300).astype(np.float32)
    idx = np.arange(300, dtype=np.int32)
    out_v, out_i, L = oracle.partition(v, idx, 5.0, 150)
    assert sorted(out_i.tolist()) == list(range(300))
    below = [(x < 5.0) or (x == 5.0 and j < 150) for x, j in zip(v, idx)]
    assert L == sum(below)
    assert all(below[j] for j in out_i[:L]) and not any(below[j] for j in out_i[L:])
    assert out_i[:L].tolist() == sorted(out_i[:L].tolist())            # left in input order
    assert out_i[L:].tolist() == sorted(out_i[L:].tolist())[::-1]      # right reversed


# ------------------------------------------------------------------- k-NN
@pytest.mark.parametrize("k,node,idx,dist", list(lattice_cases()))
def test_knng_lattice_closed_form(k, node, idx, dist):
    P = np.arange(5, dtype=np.float32)[:, None]
    d, i = oracle.knn(P, P, k, self_ids=np.arange(5))
    assert i[node].tolist() == idx
    assert d[node].tolist() == dist


def test_knng_long_lattice_order():
    # on x_i = i the order is i-1, i+1, i-2, i+2, ... (ties to the lower index)
    n, k = 40, 6
    P = np.arange(n, dtype=np.float32)[:, None]
    d, i = oracle.knn(P, P, k, self_ids=np.arange(n))
    for node in range(n):
        expect = []
        for step in range(1, n):
            for c in (node - step, node + step):
                if 0 <= c < n:
                    expect.append(c)
        assert i[node].tolist() == expect[:k]
        assert d[node].tolist() == [float((c - node) ** 2) for c in expect[:k]]


@pytest.mark.parametrize("seed", range(5))
def test_knn_matches_pairwise_brute(seed):
    rng = np.random.default_rng(seed)
    m, n, dim = int(rng.integers(1, 7)), int(rng.integers(2, 12)), int(rng.integers(1, 5))
    Q = rng.integers(-3, 4, size=(m, dim)).astype(np.float32) * np.float32(0.5)  # ties
    C = rng.integers(-3, 4, size=(n, dim)).astype(np.float32) * np.float32(0.5)
    for k in range(1, n + 1):
        d, i = oracle.knn(Q, C, k)
        bd, bi = knn_pairwise(Q.tolist(), C.tolist(), k)
        assert i.tolist() == bi
        assert d.tolist() == bd


def test_knng_matches_pairwise_brute_with_duplicates():
    P = np.array([[0, 0], [1, 0], [0, 0], [3, 1], [1, 0], [0, 2]], np.float32)
    ids = np.arange(len(P))
    for k in range(1, len(P)):
        d, i = oracle.knn(P, P, k, self_ids=ids)
        bd, bi = knn_pairwise(P.tolist(), P.tolist(), k, self_ids=ids.tolist())
        assert i.tolist() == bi and d.tolist() == bd
    d, i = oracle.knn(P, P, 1, self_ids=ids)
    assert i[0, 0] == 2 and d[0, 0] == 0.0          # the duplicate stays, at distance 0
    assert i[2, 0] == 0 and i[1, 0] == 4


def test_knn_distances_match_scipy_and_rectangular_shapes():
    # distinct m, n and d catch a transposed operand; scipy's cdist is an
    # independent FP64 evaluation of the same distances
    Q = synth.uniform_points(37, 19, seed=4)
    C = synth.uniform_points(113, 19, seed=5)
    k = 113
    d, i = oracle.knn(Q, C, k)
    ref = cdist(Q.astype(np.float64), C.astype(np.float64), "sqeuclidean")
    for r in range(Q.shape[0]):
        np.testing.assert_allclose(d[r], ref[r, i[r]], rtol=1e-13, atol=0)
        assert np.array_equal(i[r], np.argsort(ref[r], kind="stable"))


def test_knng_invariants_uniform():
    P = synth.uniform_points(300, 8, seed=1)
    k = 10
    d, i = oracle.knn(P, P, k, self_ids=np.arange(300))
    full = cdist(P.astype(np.float64), P.astype(np.float64), "sqeuclidean")
    for r in range(300):
        assert r not in i[r]                                       # self excluded
        assert len(set(i[r].tolist())) == k
        assert np.all(np.diff(d[r]) >= 0)
        others = np.delete(full[r], list(i[r]) + [r])
        assert np.all(others >= d[r, -1] * (1 - 1e-12))            # k-th bounds all selected
    # symmetry of the direct form: d(i, j) == d(j, i) exactly
    d2, i2 = oracle.knn(P, P, 299, self_ids=np.arange(300))
    D = np.full((300, 300), np.nan)
    for r in range(300):
        D[r, i2[r]] = d2[r]
    off = ~np.eye(300, dtype=bool)
    assert np.array_equal(D[off], D.T[off])


def test_knn_zero_self_distance_without_exclusion():
    P = synth.uniform_points(50, 5, seed=2)
    d, i = oracle.knn(P, P, 1)
    assert np.array_equal(i[:, 0], np.arange(50)) and np.all(d[:, 0] == 0.0)


def test_knn_padding_when_k_exceeds_corpus():
    P = np.array([[0.0], [1.0], [5.0]], np.float32)
    d, i = oracle.knn(P, P, 4, self_ids=np.arange(3))
    assert i[0].tolist() == [1, 2, -1, -1] and np.isinf(d[0, 2:]).all()


def test_generators_are_counter_based():
    a = synth.gmm_points(500, 12, seed=3)
    b = synth.gmm_points(500, 12, seed=3, rows=[4, 499, 0])
    assert np.array_equal(a[[4, 499, 0]], b)
    D = synth.sqdist_matrix_normal(20, 100, 16, seed=2)
    Dr = synth.sqdist_matrix_normal(20, 100, 16, seed=2, rows=[3, 19])
    assert np.array_equal(D[[3, 19]], Dr)
    u = synth.uniform_points(100, 4, seed=1)
    assert u.dtype == np.float32 and 0.0 <= u.min() and u.max() < 1.0
    z = synth.normal_points(20000, 4, seed=1)
    assert abs(float(z.mean())) < 0.02 and abs(float(z.std()) - 1.0) < 0.02
    assert np.all((u * (1 << 24)) == np.floor(u * (1 << 24)))


@pytest.mark.parametrize("k", [1, 5, 64, 300])
def test_nth_baseline_matches_oracle(k):
    """The nth_element CPU baseline selects the same entries, in the same
    order, as the oracle's stable sort: ties, signed zeros and NaNs included."""
    rng = np.random.default_rng(k)
    D = rng.integers(0, 40, size=(30, 700)).astype(np.float32)
    D[1, ::3] = -0.0
    D[2, ::5] = np.nan
    D[3] = rng.standard_normal(700).astype(np.float32)
    ov, oi = oracle.select_k(D, k)
    nv, ni = oracle.nth_select_k(D, k, nthreads=3)
    assert np.array_equal(ni, oi)
    assert np.array_equal(nv.view(np.uint32), ov.view(np.uint32))


@pytest.mark.parametrize("metric,scipy_name", [("cosine", "cosine"), ("pearson", "correlation")])
def test_oracle_cosine_pearson_match_scipy(metric, scipy_name):
    rng = np.random.default_rng(11)
    Q = rng.standard_normal((12, 33)).astype(np.float32)
    C = rng.standard_normal((200, 33)).astype(np.float32)
    d, i = oracle.knn(Q, C, 200, metric=metric)
    ref = cdist(Q.astype(np.float64), C.astype(np.float64), scipy_name)
    for r in range(12):
        assert np.allclose(d[r], ref[r, i[r]], rtol=1e-12, atol=1e-15)
        want = np.argsort(ref[r], kind="stable")
        assert np.array_equal(i[r], want) or np.allclose(ref[r, i[r]], ref[r, want], rtol=1e-12)


def test_oracle_cosine_hand_cases():
    """x = (1, 0): y = (0, 1) is at distance 1, (1, 1) at 1 - 1/sqrt 2,
    (-1, 0) at 2, (3, 0) at 0 (scale-free); a zero vector is at NaN, last."""
    Q = np.array([[1, 0]], np.float32)
    C = np.array([[0, 1], [1, 1], [-1, 0], [3, 0], [0, 0]], np.float32)
    d, i = oracle.knn(Q, C, 5, metric="cosine")
    assert i[0].tolist() == [3, 1, 0, 2, 4]
    assert d[0, 0] == 0.0 and abs(d[0, 1] - (1 - 2 ** -0.5)) < 1e-15 and d[0, 2] == 1.0 and d[0, 3] == 2.0
    assert np.isnan(d[0, 4])


def test_oracle_pearson_invariances():
    """Pearson distance ignores adding a constant to a vector and scaling it by
    a positive factor; cosine distance ignores only the scaling."""
    rng = np.random.default_rng(12)
    Q = rng.integers(-20, 21, (4, 20)).astype(np.float32)
    C = rng.integers(-20, 21, (60, 20)).astype(np.float32)
    C2 = (C * np.float32(4.0) + np.float32(8.0)).astype(np.float32)   # exact in FP32 (small integers)
    d1, i1 = oracle.knn(Q, C, 10, metric="pearson")
    d2, i2 = oracle.knn(Q, C2, 10, metric="pearson")
    assert np.array_equal(i1, i2) and np.allclose(d1, d2, rtol=1e-10, atol=1e-12)
    e1, j1 = oracle.knn(Q, C, 10, metric="cosine")
    e2, j2 = oracle.knn(Q, (C * np.float32(4.0)).astype(np.float32), 10, metric="cosine")
    assert np.array_equal(j1, j2) and np.allclose(e1, e2, rtol=1e-12, atol=1e-15)
