"""Pins for the FP64 pivot-network oracle: central finite differences, a
hand-worked one-unit case, the BF16 rounding rule and the feature definition."""
import numpy as np
import pytest

from oracle import mlp


def rand_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.NPARAM)


@pytest.mark.parametrize("q", [0.5, 0.9])
def test_gradient_matches_central_differences(q):
    rng = np.random.default_rng(1)
    theta = rand_theta(2)
    X = rng.normal(0, 1, (17, mlp.NIN))
    y = rng.normal(0, 1, 17)
    loss, g = mlp.loss_and_grad(theta, X, y, q)
    eps = 1e-6
    idx = rng.choice(mlp.NPARAM, 300, replace=False).tolist() + [mlp.NPARAM - 1, 0, 512, 4736]
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        fd = (mlp.pinball(y, mlp.forward(tp, X)[0], q) - mlp.pinball(y, mlp.forward(tm, X)[0], q)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_hand_worked_single_path():
    # Only hidden unit 0 of each layer is wired: h1_0 = relu(2 x0 - 1),
    # h2_0 = relu(3 h1_0 + 0.5), y_hat = 0.25 h2_0 + 1.
    theta = np.zeros(mlp.NPARAM)
    W1, b1, W2, b2, w3, b3 = (0, 512, 576, 4672, 4736, 4800)
    theta[W1 + 0] = 2.0; theta[b1 + 0] = -1.0
    theta[W2 + 0] = 3.0; theta[b2 + 0] = 0.5
    theta[w3 + 0] = 0.25; theta[b3] = 1.0
    X = np.zeros((2, 8)); X[0, 0] = 1.0; X[1, 0] = 0.25   # ReLU active / inactive in layer 1
    yhat, _ = mlp.forward(theta, X)
    assert yhat.tolist() == [1.0 + 0.25 * (3 * 1.0 + 0.5), 1.0 + 0.25 * 0.5]
    # pinball at q = 0.9 with both targets above the prediction: dL/dy_hat = -0.9 / 2 each
    loss, g = mlp.loss_and_grad(theta, X, np.array([10.0, 10.0]), 0.9)
    assert loss == pytest.approx(0.9 * ((10 - 1.875) + (10 - 1.125)) / 2)
    assert g[b3] == pytest.approx(-0.9)
    assert g[w3 + 0] == pytest.approx(-0.45 * (3.5 + 0.5))
    assert g[b2 + 0] == pytest.approx(-0.45 * 0.25 * 2)
    assert g[W2 + 0] == pytest.approx(-0.45 * 0.25 * 1.0)        # only sample 0 has h1_0 > 0
    assert g[W1 + 0] == pytest.approx(-0.45 * 0.25 * 3 * 1.0)
    assert g[b1 + 0] == pytest.approx(-0.45 * 0.25 * 3)
    assert g[W1 + 1] == 0.0                                        # x1 = 0


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8, 1.0 + 2 ** -9, -3.140625, 0.0], np.float32)
    got = mlp.bf16_round(vals)
    # 1+2^-8 is a tie between 1 and 1+2^-7: to even (1); 1+3*2^-8 ties up to 1+2^-6
    assert got.tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -3.140625, 0.0]


def test_features_definition():
    N, k = 65536, 32
    v = np.arange(256, dtype=np.float64) * 2.0 + 100.0    # a sorted, evenly spaced sample
    x, m, s = mlp.features(v, N, k)
    assert m == 354.0 and s == pytest.approx(256.0 / 1.349)   # v_191 - v_63 = 2 * 128
    r = 0   # ceil(256 * 32 / 65536) - 1 = 0
    assert x[0] == 1.0 and x[1] == pytest.approx(0.5)
    assert x[2] == pytest.approx((100 - 354) / s) and x[3] == x[2]
    assert x[4] == pytest.approx((102 - 354) / s)
    assert x[5] == pytest.approx((150 - 354) / s)
    assert x[6] == pytest.approx((v.mean() - 354) / s)
    assert mlp.features(v, 1024, 512)[0][3] == pytest.approx((v[127] - m) / s)   # r = 127
    assert mlp.sample_positions(65536) == [0, 21824, 43648, 65472]
