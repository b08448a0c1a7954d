"""Seeded synthetic inputs drawn on the device, for workloads too large to draw
on the host (the batched workload's corpora total tens of GB).

Same distributions as gen.py -- uniform[0,1), and the 64-component Gaussian
mixture with means N(0, 4I) and unit isotropic covariance -- but a different
stream of numbers: torch's seeded device generator (Philox), one generator per
job.  The oracle receives these arrays by copying them to the host; nothing
here evaluates any part of the k-NN method.
"""
from __future__ import annotations

import math

import numpy as np

from .gen import SEEDS

BATCH_DIMS = (64, 128, 768)


def batch_jobs(njobs: int = 512, m: int = 1024, seed: int = SEEDS["batch"], n_lo: float = 1e3, n_hi: float = 1e6,
               k_lo: int = 1, k_hi: int = 1024, dims=BATCH_DIMS):
    """The job table of the batched workload: per job a corpus size
    log-uniform in [n_lo, n_hi], a dimension drawn from `dims`, k log-uniform in
    [k_lo, k_hi] (rounded), m queries, and uniform or Gaussian-mixture data with
    equal probability.  Returns a list of dicts (n, m, d, k, kind, seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(njobs):
        n = int(round(10.0 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        d = int(dims[int(rng.integers(0, len(dims)))])
        k = int(round(math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))))
        k = min(max(k, k_lo), k_hi)
        kind = "uniform" if rng.random() < 0.5 else "gmm"
        out.append(dict(n=n, m=m, d=d, k=k, kind=kind, seed=seed * 1_000_000 + j))
    return out


def device_points(kind: str, count: int, d: int, seed: int, device="cuda"):
    """count x d float32 points on `device`: uniform[0,1) or the Gaussian mixture."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if kind == "uniform":
        return torch.rand((count, d), generator=g, device=device, dtype=torch.float32)
    means = 2.0 * torch.randn((64, d), generator=g, device=device, dtype=torch.float32)
    comp = torch.randint(0, 64, (count,), generator=g, device=device)
    x = torch.randn((count, d), generator=g, device=device, dtype=torch.float32)
    x += means[comp]
    return x


def job_points(job, device="cuda"):
    """(queries m x d, corpus n x d) of one job, both drawn from the job's
    distribution in one call (one mixture for both); contiguous views of one
    allocation."""
    x = device_points(job["kind"], job["n"] + job["m"], job["d"], job["seed"], device)
    return x[job["n"]:], x[:job["n"]]
