"""Training of the pivot network on rows the method itself generates.

Rows: squared-distance rows produced by the library (``knn_distances``) for
synthetic point sets of three kinds (uniform[0,1), N(0,1), 64-component Gaussian
mixture) over a grid of corpus sizes and dimensions, drawn with seeds >= 1000
so that they never coincide with evaluation inputs.  Targets: the exact k-th
smallest value of each row from ``knn_select_k``, standardised with the row
sample's median and scale, for k from 1 to 1024.  Every optimisation step runs
the library's forward, backward and Adam kernels (``knn_pivot_train_step``).

    python -m paper_1309_5478_amd.pivot_train --out paper_1309_5478_amd/pivot_weights.bin
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pivot_weights.bin")
QUANTILE = 0.99

KINDS = ("uniform", "normal", "gmm")


def _points(kind, n, d, seed):
    import synth
    if kind == "uniform":
        return synth.uniform_points(n, d, seed)
    if kind == "normal":
        return synth.normal_points(n, d, seed)
    return synth.gmm_points(n, d, seed)


def make_rows(h, configs, rows_per_set=128, ks=(1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024), log=None):
    """Features and standardised targets for every (point set, k) of `configs`,
    a list of (kind, n, d, seed).  Returns device tensors (B x 8, B)."""
    import torch
    feats, targets = [], []
    for kind, n, d, seed in configs:
        P = torch.from_numpy(_points(kind, n, d, seed)).cuda()
        Q = P[:rows_per_set].contiguous()
        D = h.distances(Q, P)
        for k in ks:
            if k > n // 4:
                continue
            f, ms = h.pivot_features(D, k)
            v, _ = h.select_k(D, k)
            y = (v[:, k - 1] - ms[:, 0]) / ms[:, 1]
            ok = torch.isfinite(y) & torch.isfinite(f).all(dim=1)
            feats.append(f[ok])
            targets.append(y[ok])
        if log:
            log(f"  rows from {kind} n={n} d={d}")
        del D, P, Q
    return torch.cat(feats).contiguous(), torch.cat(targets).contiguous()


def default_configs(seed_base=1000, big=True):
    cfgs = []
    s = seed_base
    for kind in KINDS:
        for n in (4096, 16384, 65536, 262144 if big else 131072):
            for d in (16, 64, 256, 1024):
                cfgs.append((kind, n, d, s))
                s += 1
    return cfgs


def he_init(seed: int = 1000, b3: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H, NIN = 64, 8
    W1 = rng.normal(0, np.sqrt(2.0 / NIN), (H, NIN))
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0, np.sqrt(1.0 / H), H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [b3]]).astype(np.float32)


def train(h=None, out_path=DEFAULT_WEIGHTS, steps=3000, batch=4096, lr=2e-3, quantile=QUANTILE, seed=1000,
          configs=None, log=print):
    import torch

    import paper_1309_5478_amd as knn
    h = h or knn.Handle(0)
    t0 = time.time()
    configs = configs if configs is not None else default_configs(seed)
    X, Y = make_rows(h, configs, log=log)
    log(f"{X.shape[0]} training rows in {time.time() - t0:.1f} s")
    h.pivot_set_weights(he_init(seed, b3=float(Y.median())))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    B = X.shape[0]
    loss = None
    for it in range(steps):
        idx = torch.randint(0, B, (min(batch, B),), device="cuda", generator=g)
        step_lr = lr * (0.1 ** (it / max(steps, 1)))          # exponential decay to lr / 10
        loss = h.pivot_train_step(X[idx].contiguous(), Y[idx].contiguous(), quantile, step_lr)
        if it % 500 == 0 or it == steps - 1:
            log(f"step {it}: pinball loss {float(loss):.4f}")
    if out_path:
        h.pivot_save(out_path)
        log(f"saved {out_path}")
    return h, float(loss)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--quantile", type=float, default=QUANTILE)
    ap.add_argument("--seed", type=int, default=1000)
    args = ap.parse_args(argv)
    train(out_path=args.out, steps=args.steps, quantile=args.quantile, seed=args.seed,
          log=lambda *a: print(*a, file=sys.stderr, flush=True))


if __name__ == "__main__":
    main()
