"""Counter-based seeded generators.

Every value is a pure function of (seed, stream, element index), so any row
subset of a large input can be regenerated on its own (the oracle checks sampled
rows of inputs too big to hold twice).

* hash: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014) applied twice: key = mix(seed*golden ^ stream*c2),
  h = mix(key + index).
* uniform[0,1): the top 24 bits of h times 2^-24 (exact in FP32).
* N(0,1): Box-Muller in FP64 from two independent hash streams, rounded once
  to FP32.
* Gaussian mixture: 64 equally weighted components, means 2*z (i.e. N(0,4I)),
  unit isotropic covariance; component of point i = hash(i) mod 64.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
C2 = 0xD1B54A32D192ED03

# Seeds per workload (evaluation seeds; the pivot-network training draws from
# seeds >= 1000 so that training rows never coincide with evaluation rows).
SEEDS = {"knng_small": 1, "select": 2, "knng_fused": 3, "lowprec": 4, "batch": 5,
         "sweep": 6, "metric": 7, "train_base": 1000}

# Stream ids (arbitrary distinct constants).
S_UNIFORM = 11
S_NORMAL = 21
S_GMM_MEANS = 31
S_GMM_COMP = 41
S_GMM_NOISE = 51
S_QUERY = 61
S_CORPUS = 71


def _mix_py(x: int) -> int:
    x = (x + GOLDEN) & MASK
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK
    return x ^ (x >> 31)


def _key(seed: int, stream: int) -> int:
    return _mix_py(((seed * GOLDEN) ^ (stream * C2)) & MASK)


def _mix_np(x: np.ndarray) -> np.ndarray:
    x = x + np.uint64(GOLDEN)
    x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def hash_u64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """h(seed, stream, i) for i in [start, start+count), as uint64."""
    idx = np.arange(count, dtype=np.uint64) + np.uint64(start)
    with np.errstate(over="ignore"):
        return _mix_np(idx + np.uint64(_key(seed, stream)))


def _uniform_chunk(seed, stream, start, count):
    h = hash_u64(seed, stream, start, count)
    return ((h >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32)


def _normal64_chunk(seed, stream, start, count):
    h1 = hash_u64(seed, 2 * stream, start, count)
    h2 = hash_u64(seed, 2 * stream + 1, start, count)
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)  # (0, 1]
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)          # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


_CHUNK = 1 << 22


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _fill(out_flat: np.ndarray, start: int, fn):
    """out_flat[i] = fn(start + i .. ) in chunks, threaded (numpy drops the GIL)."""
    n = out_flat.shape[0]
    spans = [(o, min(_CHUNK, n - o)) for o in range(0, n, _CHUNK)]

    def work(span):
        o, c = span
        out_flat[o:o + c] = fn(start + o, c)

    if len(spans) <= 1:
        for s in spans:
            work(s)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, spans))
    return out_flat


def uniform01(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, np.float32)
    return _fill(out, start, lambda s, c: _uniform_chunk(seed, stream, s, c))


def normal(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, np.float32)
    return _fill(out, start, lambda s, c: _normal64_chunk(seed, stream, s, c).astype(np.float32))


def _rows(n, d, rows):
    if rows is None:
        return np.arange(n, dtype=np.int64)
    return np.asarray(rows, dtype=np.int64)


def uniform_points(n: int, d: int, seed: int, stream: int = S_UNIFORM, rows=None) -> np.ndarray:
    """n x d row-major FP32 points, i.i.d. uniform[0,1).  `rows` regenerates a subset."""
    if rows is None:
        return uniform01(seed, stream, 0, n * d).reshape(n, d)
    r = _rows(n, d, rows)
    return np.stack([uniform01(seed, stream, int(i) * d, d) for i in r]) if len(r) else np.zeros((0, d), np.float32)


def normal_points(n: int, d: int, seed: int, stream: int = S_NORMAL, rows=None) -> np.ndarray:
    """n x d row-major FP32 points, i.i.d. N(0,1)."""
    if rows is None:
        return normal(seed, stream, 0, n * d).reshape(n, d)
    r = _rows(n, d, rows)
    return np.stack([normal(seed, stream, int(i) * d, d) for i in r]) if len(r) else np.zeros((0, d), np.float32)


def gmm_components(n: int, seed: int, ncomp: int = 64, rows=None) -> np.ndarray:
    r = _rows(n, 0, rows)
    h = np.empty(len(r), np.uint64)
    if rows is None:
        h[:] = hash_u64(seed, S_GMM_COMP, 0, n)
    else:
        for j, i in enumerate(r):
            h[j] = hash_u64(seed, S_GMM_COMP, int(i), 1)[0]
    return (h % np.uint64(ncomp)).astype(np.int64)


def gmm_means(d: int, seed: int, ncomp: int = 64) -> np.ndarray:
    return 2.0 * _normal64_chunk(seed, S_GMM_MEANS, 0, ncomp * d).reshape(ncomp, d)


def gmm_points(n: int, d: int, seed: int, ncomp: int = 64, rows=None) -> np.ndarray:
    """n x d FP32 points from an equal-weight mixture of `ncomp` Gaussians with
    means drawn from N(0, 4I) and unit isotropic covariance (rounded once to FP32)."""
    mu = gmm_means(d, seed, ncomp)
    comp = gmm_components(n, seed, ncomp, rows)
    r = _rows(n, d, rows)
    out = np.empty((len(r), d), np.float32)
    if rows is None:
        rb = max(1, _CHUNK // max(d, 1))
        spans = [(o, min(rb, n - o)) for o in range(0, n, rb)]

        def work(span):
            o, c = span
            z = _normal64_chunk(seed, S_GMM_NOISE, o * d, c * d).reshape(c, d)
            z += mu[comp[o:o + c]]
            out[o:o + c] = z

        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, spans))
    else:
        for j, i in enumerate(r):
            z = _normal64_chunk(seed, S_GMM_NOISE, int(i) * d, d)
            out[j] = (mu[comp[j]] + z).astype(np.float32)
    return out


def sqdist_matrix_normal(m: int, n: int, d: int, seed: int, rows=None) -> np.ndarray:
    """An m x n FP32 matrix whose entries are squared Euclidean distances between
    m query points and n corpus points, both i.i.d. N(0,1) in d dimensions.

    This is input synthesis for the selection-only workload (selection over a
    given matrix); it is evaluated here in FP64 with a library matrix product and
    rounded once to FP32, and is never used as the reference for any distance
    check.  `rows` restricts the output to a subset of query rows.
    """
    r = _rows(m, d, rows)
    Q = normal_points(m, d, seed, S_QUERY, rows=None if rows is None else r).astype(np.float64)
    C = normal_points(n, d, seed, S_CORPUS).astype(np.float64)
    cn = np.einsum("ij,ij->i", C, C)
    out = np.empty((len(r), n), np.float32)
    step = 512
    for o in range(0, len(r), step):
        q = Q[o:o + step]
        qn = np.einsum("ij,ij->i", q, q)
        out[o:o + step] = (qn[:, None] + cn[None, :] - 2.0 * (q @ C.T)).astype(np.float32)
    return out


def adversarial_rows(cols: int, seed: int) -> dict:
    """Named FP32 rows that stress selection: ties, signed zeros, infinities, NaNs,
    sorted and reversed orders, a single distinct outlier."""
    u = uniform01(seed, 97, 0, cols)
    rows = {
        "constant": np.full(cols, 3.25, np.float32),
        "sorted": np.sort(u),
        "reversed": np.sort(u)[::-1].copy(),
        "few_distinct": np.floor(u * 4).astype(np.float32),
        "signed_zeros": np.where(u < 0.5, np.float32(-0.0), np.float32(0.0)).astype(np.float32),
        "with_inf_nan": np.where(u < 0.1, np.float32(np.nan),
                                 np.where(u < 0.2, np.float32(np.inf),
                                          np.where(u < 0.3, np.float32(-np.inf), u))).astype(np.float32),
        "all_nan": np.full(cols, np.nan, np.float32),
        "one_low": np.concatenate([np.full(cols - 1, 7.0, np.float32), np.array([-1.0], np.float32)]),
        "sawtooth": (np.arange(cols) % 97).astype(np.float32),
        "negatives": (-u).astype(np.float32),
    }
    return rows
