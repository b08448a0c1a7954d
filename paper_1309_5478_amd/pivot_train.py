"""Training of the pivot network on rows the method itself generates.

Rows: squared-distance rows produced by the library (``knn_distances``) for
synthetic point sets of three kinds (uniform[0,1), N(0,1), 64-component Gaussian
mixture) over a grid of corpus sizes and dimensions, drawn with seeds >= 1000
so that they never coincide with evaluation inputs.  For each row and each k
from 1 to 1024 the library stores one example (``knn_pivot_add_examples``: the
row's features and its exact k-th smallest value standardised, computed on the
device), then trains the network from a seed (``knn_pivot_train``: He
initialisation, batch draws, forward, backward and Adam, all on the device).
This module only generates the point sets and calls the library.

    python -m paper_1309_5478_amd.pivot_train --out paper_1309_5478_amd/pivot_weights.bin
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pivot_weights.bin")
QUANTILE = 0.99     # the training quantile of knn_pivot_train
KS = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)

KINDS = ("uniform", "normal", "gmm")


def _points(kind, n, d, seed):
    import synth
    if kind == "uniform":
        return synth.uniform_points(n, d, seed)
    if kind == "normal":
        return synth.normal_points(n, d, seed)
    return synth.gmm_points(n, d, seed)


def add_rows(h, configs, rows_per_set=128, ks=KS, log=None):
    """Stores training examples for every (point set, k) of `configs`, a list
    of (kind, n, d, seed): the distance rows of the set's first rows_per_set
    points against the whole set.  Returns the example count."""
    import torch
    for kind, n, d, seed in configs:
        P = torch.from_numpy(_points(kind, n, d, seed)).cuda()
        D = h.distances(P[:rows_per_set].contiguous(), P)
        for k in ks:
            if k <= n // 4:
                h.pivot_add_examples(D, k)
        if log:
            log(f"  rows from {kind} n={n} d={d}")
        del D, P
    return h.pivot_example_count()


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
    """Random parameters for tests of the kernels (host draw; training itself
    initialises on the device)."""
    rng = np.random.default_rng(seed)
    H, NIN = 64, 8
    W1 = rng.normal(0, np.sqrt(2.0 / NIN), (H, NIN))
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0, np.sqrt(1.0 / H), H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [b3]]).astype(np.float32)


def train(h=None, out_path=DEFAULT_WEIGHTS, steps=3000, seed=1000, configs=None, log=print):
    import paper_1309_5478_amd as knn
    h = h or knn.Handle(0, pivot_weights=None)
    t0 = time.time()
    configs = configs if configs is not None else default_configs(seed)
    h.pivot_clear_examples()
    n = add_rows(h, configs, log=log)
    log(f"{n} training examples in {time.time() - t0:.1f} s")
    t1 = time.time()
    h.pivot_train(out_path, seed=seed, steps=steps)
    log(f"{steps} training steps in {time.time() - t1:.1f} s" + (f"; saved {out_path}" if out_path else ""))
    return h


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=1000)
    args = ap.parse_args(argv)
    train(out_path=args.out, steps=args.steps, seed=args.seed, log=lambda *a: print(*a, file=sys.stderr, flush=True))


if __name__ == "__main__":
    main()
