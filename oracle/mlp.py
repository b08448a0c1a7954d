"""FP64 oracle of the pivot network and its features.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Independent of the HIP
path: it re-implements, in plain numpy and float64, what the pivot network
computes.

The pivot network predicts, from statistics of a small strided sample of a
row, the standardised value of the row's k-th smallest entry:
    y = (v_k - m) / s,
where m is the sample's lower median and s a robust scale (interquartile range
/ 1.349).  The first partition pivot of the quick multi-select is then
m + s * y_hat.

Sample: 4 blocks of 64 contiguous entries, block b starting at
floor(b * (N - 64) / 3), sorted ascending (256 values v_0 <= ... <= v_255).
Features (8):
    x0 = log2(N) / 16
    x1 = log2(k) / 10
    x2 = (v_0 - m) / s                       sample minimum
    x3 = (v_r - m) / s,  r = clamp(ceil(256 k / N) - 1, 0, 255)
    x4 = (v_{min(r+1,255)} - m) / s
    x5 = (v_25 - m) / s                      about the 10th percentile
    x6 = (mean - m) / s
    x7 = log(s / (|m| + s))
with m = v_127, s = max((v_191 - v_63) / 1.349, 1e-30 * (|m| + 1)).

Network: x -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64) ->
y_hat = w3 . h2 + b3, with weights rounded to BF16 (round to nearest even).
Flat parameter layout (4801 floats): W1 (64 x 8, row-major), b1 (64),
W2 (64 x 64), b2 (64), w3 (64), b3 (1).
Loss: mean pinball (quantile) loss at quantile q,
    rho_q(u) = q u (u >= 0), (q - 1) u (u < 0),  u = y - y_hat,
whose derivative in y_hat is -q for u > 0, 1 - q for u < 0 and 0 at u = 0.
"""
from __future__ import annotations

import numpy as np

H = 64
NIN = 8
NPARAM = H * NIN + H + H * H + H + H + 1
SAMPLE = 256
BLOCKS = 4


def split(theta):
    theta = np.asarray(theta, np.float64)
    o = 0
    W1 = theta[o:o + H * NIN].reshape(H, NIN); o += H * NIN
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def bf16_round(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X):
    """Returns y_hat and the intermediate values (for backward)."""
    W1, b1, W2, b2, w3, b3 = split(theta)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def pinball(y, yhat, q):
    u = np.asarray(y, np.float64) - yhat
    return float(np.mean(np.where(u >= 0, q * u, (q - 1) * u)))


def loss_and_grad(theta, X, y, q):
    """Mean pinball loss and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = split(theta)
    yhat, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    u = np.asarray(y, np.float64) - yhat
    loss = float(np.mean(np.where(u >= 0, q * u, (q - 1) * u)))
    dy = np.where(u > 0, -q, np.where(u < 0, 1.0 - q, 0.0)) / B
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    d2 = np.outer(dy, w3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, g


def sample_positions(N):
    """Start of each of the 4 sample blocks of 64 entries in a row of N >= 64."""
    return [(b * (N - 64)) // (BLOCKS - 1) for b in range(BLOCKS)]


def row_sample(row):
    N = row.shape[0]
    return np.sort(np.concatenate([row[s:s + 64] for s in sample_positions(N)]).astype(np.float32))


def features(sample_sorted, N, k):
    """The 8 features of a row from its ascending 256-entry sample (FP64)."""
    v = np.asarray(sample_sorted, np.float64)
    m = v[127]
    s = max((v[191] - v[63]) / 1.349, 1e-30 * (abs(m) + 1.0))
    r = int(min(max(-(-SAMPLE * k // N) - 1, 0), SAMPLE - 1))
    r1 = min(r + 1, SAMPLE - 1)
    x = np.array([
        np.log2(N) / 16.0,
        np.log2(k) / 10.0,
        (v[0] - m) / s,
        (v[r] - m) / s,
        (v[r1] - m) / s,
        (v[25] - m) / s,
        (v.mean() - m) / s,
        np.log(s / (abs(m) + s)),
    ])
    return x, m, s
