"""Pins of the reference BF16 / e4m3 conversions (oracle/quant.py) against
hand-worked codes from the formats' definitions, torch's CPU casts where they
agree in range, and invariants (monotonicity, nearest value, per-point scale)."""
import numpy as np
import pytest

from oracle import quant


def test_e4m3_decode_hand_values():
    assert quant.e4m3_value(0x7E) == 448.0          # S.1111.110: largest finite
    assert np.isnan(quant.e4m3_value(0x7F))         # S.1111.111: NaN
    assert quant.e4m3_value(0x38) == 1.0            # exponent 7 = bias
    assert quant.e4m3_value(0x08) == 2.0 ** -6      # smallest normal
    assert quant.e4m3_value(0x01) == 2.0 ** -9      # smallest subnormal
    assert quant.e4m3_value(0x07) == 7 * 2.0 ** -9  # largest subnormal
    assert quant.e4m3_value(0xB8) == -1.0
    assert quant.e4m3_value(0x80) == 0.0 and np.signbit(quant.e4m3_value(0x80))


@pytest.mark.parametrize("x,code", [
    (1.0, 0x38), (1.0625, 0x38),          # tie between 1 (even) and 1.125 (odd)
    (1.1875, 0x3A),                       # tie between 1.125 (odd) and 1.25 (even)
    (1.07, 0x39), (448.0, 0x7E), (447.0, 0x7E), (420.0, 0x7D),
    (460.0, 0x7E), (1e6, 0x7E), (np.inf, 0x7E), (-500.0, 0xFE), (-np.inf, 0xFE),
    (3 * 2.0 ** -10, 0x02),               # subnormal tie: 2^-9 (odd) vs 2^-8 (even)
    (2.0 ** -10, 0x00),                   # tie between 0 (even) and 2^-9
    (1.01 * 2.0 ** -10, 0x01), (2.0 ** -6, 0x08), (-0.0, 0x80), (0.0, 0x00),
])
def test_e4m3_hand_cases(x, code):
    assert int(quant.to_e4m3(np.array([x], np.float32))[0]) == code


def test_e4m3_nan():
    assert int(quant.to_e4m3(np.array([np.nan], np.float32))[0]) & 0x7F == 0x7F


@pytest.mark.parametrize("x,code", [
    (1.0, 0x3F80), (1 + 2.0 ** -8, 0x3F80), (1 + 3 * 2.0 ** -8, 0x3F82), (-2.0, 0xC000),
    (3.4028235e38, 0x7F80),               # above the largest BF16 by more than half an ulp
    (3.3895314e38, 0x7F7F),               # the largest BF16 itself
    (-0.0, 0x8000), (np.inf, 0x7F80), (-np.inf, 0xFF80),
    (2.0 ** -133, 0x0001),                # smallest BF16 subnormal
    (2.0 ** -134, 0x0000),                # tie between 0 (even) and 2^-133
    (3 * 2.0 ** -134, 0x0002),            # tie between 2^-133 (odd) and 2^-132 (even)
])
def test_bf16_hand_cases(x, code):
    assert int(quant.to_bf16(np.array([x], np.float32))[0]) == code


def test_bf16_nan_stays_nan():
    x = np.array([0x7F800001, 0xFFC00000, 0x7FFFFFFF], np.uint32).view(np.float32)
    out = quant.to_bf16(x).astype(np.int64)
    assert ((out & 0x7F80) == 0x7F80).all() and ((out & 0x7F) != 0).all()
    assert list(out >> 15) == [0, 1, 0]


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n).astype(np.float32) * np.exp2(rng.integers(-30, 30, n)).astype(np.float32)
    bits = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32).view(np.float32)
    return np.concatenate([x, bits[np.isfinite(bits)]])


def test_bf16_matches_torch_on_finite_values():
    torch = pytest.importorskip("torch")
    x = _sample(200000, 1)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(quant.to_bf16(x), want)


def test_e4m3_matches_torch_in_range():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-460, 460, 100000), rng.standard_normal(100000) * 2.0 ** -7,
                        np.arange(-448, 448.25, 0.25)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(quant.to_e4m3(x), want)


@pytest.mark.parametrize("conv,value,top", [(quant.to_e4m3, quant.e4m3_value, 0x7E),
                                           (quant.to_bf16, quant.bf16_value, 0x7F7F)])
def test_nearest_and_monotone(conv, value, top):
    """The chosen code is never farther from x than any other code, and the
    conversion is monotone on a sorted sweep."""
    rng = np.random.default_rng(3)
    x = np.sort(rng.uniform(-1.5 * 448 if top == 0x7E else -1e3, 448 if top == 0x7E else 1e3, 20000))
    x = x.astype(np.float32)
    codes = conv(x).astype(np.int64)
    vals = np.array([value(int(c)) for c in codes])
    assert (np.diff(vals) >= 0).all()
    allv = np.array([value(c) for c in range(top + 1)])
    for xi, v in zip(x[::97].astype(np.float64), vals[::97]):
        if abs(xi) <= allv[-1]:
            assert abs(v - xi) <= np.min(np.abs(allv - abs(xi))) + 0.0


def test_fp8_scale_exponent():
    assert quant.fp8_scale_exponent(np.array([1.0, -0.5])) == 8          # 256 <= 448 < 512
    assert quant.fp8_scale_exponent(np.array([448.0])) == 0
    assert quant.fp8_scale_exponent(np.array([-449.0])) == -1
    assert quant.fp8_scale_exponent(np.zeros(5)) == 0
    assert quant.fp8_scale_exponent(np.array([np.nan, 2.0])) == 7         # NaN ignored
    assert quant.fp8_scale_exponent(np.array([1e-38])) == 100             # limited
    rng = np.random.default_rng(4)
    for _ in range(200):
        row = rng.standard_normal(16) * 10.0 ** rng.uniform(-5, 5)
        e = quant.fp8_scale_exponent(row)
        amax = np.abs(row).max()
        assert np.ldexp(amax, e) <= 448 < np.ldexp(amax, e + 1)


def test_quantize_fp8_rows_round_trip():
    rng = np.random.default_rng(5)
    X = (rng.standard_normal((50, 40)) * 3).astype(np.float32)
    codes, scales = quant.quantize_fp8(X)
    back = np.array([[quant.e4m3_value(int(c)) for c in row] for row in codes]) * scales[:, None]
    # relative error of a normal e4m3 value is at most 2^-4
    big = np.abs(X) * (1.0 / scales[:, None]) >= 2.0 ** -6
    assert np.all(np.abs(back - X)[big] <= 2.0 ** -4 * np.abs(X)[big])
