"""The reduced-precision operands (knn_quantize) element by element against the
reference conversions written from the BF16 and OCP e4m3 definitions."""
import sys

import numpy as np
import pytest

from oracle import quant

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


def points(d):
    rng = np.random.default_rng(d)
    rows = [rng.standard_normal(d) * 10.0 ** rng.uniform(-6, 6) for _ in range(300)]
    rows.append(np.zeros(d))
    special = rng.standard_normal(d)
    special[::7] = np.inf
    special[3 % d] = -np.inf                        # (d = 1: the only element)
    rows.append(special)
    nanrow = rng.standard_normal(d)
    nanrow[1::5] = np.nan
    rows.append(nanrow)
    rows.append(np.full(d, 1e-40))                  # FP32 subnormals: e limited to 100
    rows.append(np.full(d, 3.0e38) * np.sign(rng.standard_normal(d)))   # e limited to -100
    ties = np.arange(d) % 9 * 0.0625 + 1.0          # e4m3 and BF16 ties after scaling
    rows.append(ties)
    rows.append(rng.integers(-448, 449, d).astype(np.float64))
    X = np.array(rows, dtype=np.float32)
    bits = rng.integers(0, 1 << 32, (64, d), dtype=np.uint64).astype(np.uint32).view(np.float32)
    return np.concatenate([X, bits])                 # arbitrary bit patterns, NaNs and infinities included


@pytest.mark.parametrize("d", [1, 24, 128, 300])
def test_bf16_codes(h, torch, d):
    X = points(d)
    codes, _ = h.quantize(torch.from_numpy(X).cuda(), "bf16")
    got = codes.cpu().numpy().view(np.uint16)
    want = quant.to_bf16(X)
    nan = np.isnan(X)
    assert np.array_equal(got[:, :d][~nan], want[~nan])
    # NaN: a quiet NaN with the input's sign (payload bits are not specified)
    g = got[:, :d][nan].astype(np.int64)
    assert ((g & 0x7F80) == 0x7F80).all() and ((g & 0x40) != 0).all()
    assert np.array_equal(g >> 15, (X.view(np.uint32)[nan] >> 31).astype(np.int64))
    assert (got[:, d:] == 0).all()


@pytest.mark.parametrize("d", [1, 24, 128, 300])
def test_fp8_codes_and_scales(h, torch, d):
    X = points(d)
    codes, scale = h.quantize(torch.from_numpy(X).cuda(), "fp8")
    got, gs = codes.cpu().numpy(), scale.cpu().numpy()
    want, ws = quant.quantize_fp8(X)
    bad = np.nonzero((got[:, :d] != want).any(axis=1) | (gs.view(np.uint32) != ws.view(np.uint32)))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:3]}: {X[bad[0]][:4]}"
    assert (got[:, d:] == 0).all()
