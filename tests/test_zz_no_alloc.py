"""knn_select_k_noalloc (the allocation-free variant of knn_select_k, with its
workspace in a static device array) against knn_select_k, bit for bit,
through the C ABI: two calls in a row, the second with a smaller input, so
the second runs on the array the first one left behind."""
import ctypes
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


def p(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def noalloc(h, torch, knn, dev, k, pivot="sample", indices=True):
    rows, cols = dev.shape
    v = torch.full((rows, k), 7.0, dtype=torch.float32, device=dev.device)
    i = torch.full((rows, k), -7, dtype=torch.int32, device=dev.device) if indices else None
    o = knn.Handle._opts(pivot)
    st = h.lib.knn_select_k_noalloc(h.h, p(dev), rows, cols, max(dev.stride(0), cols), k, p(v), p(i),
                                    h._stream(), ctypes.byref(o))
    assert st == 0, h.lib.knn_last_error(h.h).decode()
    torch.cuda.synchronize()
    return v.cpu().numpy(), (i.cpu().numpy() if i is not None else None)


CASES = [
    # (rows, cols, k): long rows first (fewer workgroups than usual), then a
    # smaller input on the array the first call left behind
    [(600, 20000, 256), (50, 3000, 100)],
    [(4, 300000, 1024), (3, 70001, 32)],
    [(2000, 1500, 64), (7, 1024, 1024)],
]


@pytest.mark.parametrize("pair", range(len(CASES)))
@pytest.mark.parametrize("pivot", ["sample", "plain", "learned"])
def test_noalloc_matches_select_k_twice(h, torch, knn, pair, pivot):
    for n, (rows, cols, k) in enumerate(CASES[pair]):
        say(f"select_k_noalloc call {n + 1}: {rows} x {cols}, k={k}, pivot={pivot}")
        D = synth.sqdist_matrix_normal(rows, cols, 24, seed=100 + 10 * pair + n)
        D[0, ::11] = -0.0
        dev = torch.from_numpy(D).cuda()
        v, i = noalloc(h, torch, knn, dev, k, pivot)
        rv, ri = h.select_k(dev, k, pivot=pivot, flags=knn.FLAG_NO_SPLIT)
        assert np.array_equal(bits(v), bits(rv.cpu().numpy()))
        assert np.array_equal(i, ri.cpu().numpy())
        rows_chk = np.arange(0, rows, max(1, rows // 16))
        ov, oi = oracle.select_k(D, k, rows=rows_chk)
        assert np.array_equal(bits(v[rows_chk]), bits(ov)) and np.array_equal(i[rows_chk], oi)


def test_noalloc_values_only_and_padded_rows(h, torch, knn):
    D = synth.sqdist_matrix_normal(300, 9000, 16, seed=7)
    host = np.zeros((300, 9003), np.float32)
    host[:, :9000] = D
    dev = torch.from_numpy(host).cuda()[:, :9000]
    v, _ = noalloc(h, torch, knn, dev, 500, indices=False)
    ov, _ = oracle.select_k(D, 500)
    assert np.array_equal(bits(v), bits(ov))


def test_noalloc_rejects_rows_beyond_the_array(h, torch, knn):
    x = torch.zeros((1, 16), device="cuda")
    out = torch.zeros((1, 8), device="cuda")
    o = knn.Handle._opts()
    cols = 4195313
    st = h.lib.knn_select_k_noalloc(h.h, p(x), 1, cols, cols, 8, p(out), p(None), h._stream(), ctypes.byref(o))
    assert st == knn._abi.KNN_ERROR_UNSUPPORTED
    assert b"scratch" in h.lib.knn_last_error(h.h)
