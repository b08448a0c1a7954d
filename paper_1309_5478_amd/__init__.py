"""MI355X-native brute-force k-NN / k-NN graph by GPU quick multi-select.

A thin binding over libknn.so (include/knn.h): every step of the computation
runs in the library's HIP kernels; this module only checks tensors, allocates
outputs with torch on the same device and passes device pointers and the
current HIP stream.  Method: Komarov, Dashti & D'Souza, arXiv:1309.5478.
"""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import (PIVOT_LEARNED, PIVOT_PLAIN, PIVOT_SAMPLE, PREC_BF16, PREC_FP32,  # noqa: F401
                   PREC_FP8_E4M3, FLAG_FORCE_FALLBACK, FLAG_UNFUSED, FLAG_TIMING, FLAG_NO_GRAPH, FLAG_AUTOTUNE, FLAG_FORCE_RERUN, FLAG_NO_SPLIT,
                   FLAG_FORCE_SPLIT, Job, Options,
                   Stats)

_PIVOTS = {"plain": PIVOT_PLAIN, "sample": PIVOT_SAMPLE, "learned": PIVOT_LEARNED}
_PRECS = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp8": PREC_FP8_E4M3}
_METRICS = {"sqeuclidean": _abi.METRIC_SQEUCLIDEAN, "cosine": _abi.METRIC_COSINE, "pearson": _abi.METRIC_PEARSON}


class KnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _torch():
    import torch
    return torch


class Handle:
    """Owns a libknn handle (device workspace, statistics) on one device."""

    def __init__(self, device: int = 0, pivot_weights: str | None = "default"):
        """pivot_weights: a weights file for the learned pivot, "default" for the
        packaged one (if present), or None for none."""
        self.lib = _abi.load()
        h = ctypes.c_void_p()
        st = self.lib.knn_create(ctypes.byref(h), device)
        if st != 0:
            raise KnnError(st, self.lib.knn_last_error(None).decode())
        self.h = h
        self.device = device
        if pivot_weights == "default":
            import os
            pivot_weights = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pivot_weights.bin")
            if not os.path.exists(pivot_weights):
                pivot_weights = None
        if pivot_weights:
            self.pivot_load(pivot_weights)

    def close(self):
        if getattr(self, "h", None):
            self.lib.knn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise KnnError(st, self.lib.knn_last_error(self.h).decode())

    def _stream(self):
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    @staticmethod
    def _opts(pivot="sample", precision="fp32", oversample=4, flags=0, metric="sqeuclidean"):
        o = Options()
        o.metric = _METRICS[metric] if isinstance(metric, str) else int(metric)
        o.pivot = _PIVOTS[pivot] if isinstance(pivot, str) else int(pivot)
        o.precision = _PRECS[precision] if isinstance(precision, str) else int(precision)
        o.oversample = int(oversample)
        o.flags = int(flags)
        return o

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.knn_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def select_k(self, dist, k: int, pivot="sample", flags=0, indices=True):
        """k smallest entries per row of a 2-D FP32 CUDA tensor (row stride may
        exceed the width).  Returns (values [rows, k] f32, indices [rows, k] i32),
        or (values, None) with indices=False (values only)."""
        torch = _torch()
        if dist.dim() != 2 or dist.dtype != torch.float32 or not dist.is_cuda or dist.stride(1) != 1:
            raise ValueError("dist must be a 2-D float32 device tensor with unit column stride")
        rows, cols = dist.shape
        vals = torch.empty((rows, k), dtype=torch.float32, device=dist.device)
        idx = torch.empty((rows, k), dtype=torch.int32, device=dist.device) if indices else None
        o = self._opts(pivot, flags=flags)
        self._check(self.lib.knn_select_k(self.h, ctypes.c_void_p(dist.data_ptr()), rows, cols,
                                          max(dist.stride(0), cols), k, ctypes.c_void_p(vals.data_ptr()),
                                          ctypes.c_void_p(idx.data_ptr() if idx is not None else 0),
                                          self._stream(), ctypes.byref(o)))
        return vals, idx

    def partition(self, x, piv_val, piv_idx):
        """One partition pass per row (one wave per row).  Returns (values, indices, L)."""
        torch = _torch()
        if x.dim() != 2 or x.dtype != torch.float32 or not x.is_cuda or x.stride(1) != 1:
            raise ValueError("x must be a 2-D float32 device tensor with unit column stride")
        rows, cols = x.shape
        pv = piv_val.to(device=x.device, dtype=torch.float32).contiguous()
        pi = piv_idx.to(device=x.device, dtype=torch.int32).contiguous()
        ov = torch.empty((rows, cols), dtype=torch.float32, device=x.device)
        oi = torch.empty((rows, cols), dtype=torch.int32, device=x.device)
        L = torch.empty((rows,), dtype=torch.int32, device=x.device)
        self._check(self.lib.knn_partition(self.h, ctypes.c_void_p(x.data_ptr()), rows, cols,
                                           max(x.stride(0), cols), ctypes.c_void_p(pv.data_ptr()),
                                           ctypes.c_void_p(pi.data_ptr()), ctypes.c_void_p(ov.data_ptr()),
                                           ctypes.c_void_p(oi.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                                           self._stream()))
        return ov, oi, L

    def search(self, queries, corpus, k: int, pivot="sample", precision="fp32", oversample=4, flags=0,
               metric="sqeuclidean"):
        """k nearest corpus rows per query row (squared Euclidean, or with
        metric "cosine" / "pearson" the distance 1 - similarity).
        Returns (dist [m, k] f32, idx [m, k] i32)."""
        torch = _torch()
        for t in (queries, corpus):
            if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("queries and corpus must be contiguous 2-D float32 device tensors")
        m, d = queries.shape
        n, d2 = corpus.shape
        if d != d2:
            raise ValueError("queries and corpus differ in dimension")
        dist = torch.empty((m, k), dtype=torch.float32, device=queries.device)
        idx = torch.empty((m, k), dtype=torch.int32, device=queries.device)
        o = self._opts(pivot, precision, oversample, flags, metric)
        self._check(self.lib.knn_search(self.h, ctypes.c_void_p(queries.data_ptr()), m,
                                        ctypes.c_void_p(corpus.data_ptr()), n, d, k,
                                        ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                        self._stream(), ctypes.byref(o)))
        return dist, idx

    def search_host_corpus(self, queries, corpus_host, k: int, part_rows=0, pivot="sample", precision="fp32",
                           oversample=4, flags=0, metric="sqeuclidean"):
        """search() with the corpus in host memory (a contiguous float32 CPU
        tensor, pinned for copies that overlap the search), streamed to the
        device in partitions of part_rows points (0: about 1 GiB)."""
        torch = _torch()
        if queries.dim() != 2 or queries.dtype != torch.float32 or not queries.is_cuda or not queries.is_contiguous():
            raise ValueError("queries must be a contiguous 2-D float32 device tensor")
        if (corpus_host.dim() != 2 or corpus_host.dtype != torch.float32 or corpus_host.is_cuda
                or not corpus_host.is_contiguous()):
            raise ValueError("corpus_host must be a contiguous 2-D float32 host tensor")
        m, d = queries.shape
        n, d2 = corpus_host.shape
        if d != d2:
            raise ValueError("queries and corpus differ in dimension")
        dist = torch.empty((m, k), dtype=torch.float32, device=queries.device)
        idx = torch.empty((m, k), dtype=torch.int32, device=queries.device)
        o = self._opts(pivot, precision, oversample, flags, metric)
        self._check(self.lib.knn_search_host_corpus(self.h, ctypes.c_void_p(queries.data_ptr()), m,
                                                    ctypes.c_void_p(corpus_host.data_ptr()), n, d, k, int(part_rows),
                                                    ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                                    self._stream(), ctypes.byref(o)))
        return dist, idx

    def batch_search(self, jobs, pivot="sample", precision="fp32", oversample=4, flags=0, out=None,
                     metric="sqeuclidean"):
        """Many independent k-NN problems in one call.  `jobs` is a list of
        (queries, corpus, k) tuples of contiguous float32 device tensors, with
        queries None for the k-NN graph of the corpus.  Returns a list of
        (dist [m, k], idx [m, k]); `out` may pass that list preallocated (same
        tensors on every call let the library replay its captured graphs)."""
        torch = _torch()
        arr = (Job * max(len(jobs), 1))()
        res = []
        for j, (q, c, kj) in enumerate(jobs):
            for t in (c,) if q is None else (q, c):
                if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                    raise ValueError("job tensors must be contiguous 2-D float32 device tensors")
            n, d = c.shape
            m = n if q is None else q.shape[0]
            if q is not None and q.shape[1] != d:
                raise ValueError(f"job {j}: queries and corpus differ in dimension")
            if out is not None:
                dist, idx = out[j]
            else:
                dist = torch.empty((m, kj), dtype=torch.float32, device=c.device)
                idx = torch.empty((m, kj), dtype=torch.int32, device=c.device)
            arr[j] = Job(0 if q is None else q.data_ptr(), m, c.data_ptr(), n, d, kj, dist.data_ptr(),
                         idx.data_ptr())
            res.append((dist, idx))
        o = self._opts(pivot, precision, oversample, flags, metric)
        self._check(self.lib.knn_batch_search(self.h, arr, len(jobs), self._stream(), ctypes.byref(o)))
        return res

    def distances(self, queries, corpus):
        """Squared Euclidean distance matrix [m, n] f32 by the norm expansion."""
        torch = _torch()
        for t in (queries, corpus):
            if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("queries and corpus must be contiguous 2-D float32 device tensors")
        m, d = queries.shape
        n = corpus.shape[0]
        out = torch.empty((m, n), dtype=torch.float32, device=queries.device)
        self._check(self.lib.knn_distances(self.h, ctypes.c_void_p(queries.data_ptr()), m,
                                           ctypes.c_void_p(corpus.data_ptr()), n, d,
                                           ctypes.c_void_p(out.data_ptr()), n, self._stream()))
        return out

    def quantize(self, x, precision):
        """Reduced-precision operand codes of the rows of a contiguous FP32
        device tensor: (codes [n, ldo] uint8 (FP8) or int16 (BF16 bits), ldo = d
        rounded up to 128, scales [n] f32 or None)."""
        torch = _torch()
        if x.dim() != 2 or x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous 2-D float32 device tensor")
        n, d = x.shape
        prec = _PRECS[precision] if isinstance(precision, str) else int(precision)
        ldo = (d + 127) // 128 * 128
        codes = torch.empty((n, ldo), dtype=torch.int16 if prec == PREC_BF16 else torch.uint8, device=x.device)
        scale = torch.empty((n,), dtype=torch.float32, device=x.device) if prec == PREC_FP8_E4M3 else None
        self._check(self.lib.knn_quantize(self.h, ctypes.c_void_p(x.data_ptr()), n, d, prec,
                                          ctypes.c_void_p(codes.data_ptr()),
                                          ctypes.c_void_p(scale.data_ptr() if scale is not None else 0),
                                          self._stream()))
        return codes, scale

    # ---- pivot network -------------------------------------------------------
    def pivot_set_weights(self, params):
        import numpy as np
        w = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.knn_pivot_set_weights(self.h, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def pivot_get_weights(self):
        import numpy as np
        w = np.empty(_abi.PIVOT_NPARAM, np.float32)
        self._check(self.lib.knn_pivot_get_weights(self.h, w.ctypes.data_as(ctypes.c_void_p), w.size))
        return w

    def pivot_save(self, path: str):
        self._check(self.lib.knn_pivot_save(self.h, str(path).encode()))

    def pivot_load(self, path: str):
        self._check(self.lib.knn_pivot_load(self.h, str(path).encode()))

    def pivot_features(self, dist, k: int):
        """Features [rows, 8] and (m, s) [rows, 2] of each row of a device matrix."""
        torch = _torch()
        rows, cols = dist.shape
        f = torch.empty((rows, 8), dtype=torch.float32, device=dist.device)
        ms = torch.empty((rows, 2), dtype=torch.float32, device=dist.device)
        self._check(self.lib.knn_pivot_features(self.h, ctypes.c_void_p(dist.data_ptr()), rows, cols,
                                                max(dist.stride(0), cols), k, ctypes.c_void_p(f.data_ptr()),
                                                ctypes.c_void_p(ms.data_ptr()), self._stream()))
        return f, ms

    def pivot_predict(self, feats):
        torch = _torch()
        feats = feats.contiguous()
        out = torch.empty((feats.shape[0],), dtype=torch.float32, device=feats.device)
        self._check(self.lib.knn_pivot_predict(self.h, ctypes.c_void_p(feats.data_ptr()), feats.shape[0],
                                               ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def pivot_grad(self, feats, targets, quantile: float):
        torch = _torch()
        feats, targets = feats.contiguous(), targets.contiguous()
        g = torch.empty((_abi.PIVOT_NPARAM,), dtype=torch.float32, device=feats.device)
        loss = torch.empty((1,), dtype=torch.float32, device=feats.device)
        self._check(self.lib.knn_pivot_grad(self.h, ctypes.c_void_p(feats.data_ptr()),
                                            ctypes.c_void_p(targets.data_ptr()), feats.shape[0], quantile,
                                            ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                            self._stream()))
        return g, loss

    def pivot_train_step(self, feats, targets, quantile: float, lr: float):
        torch = _torch()
        loss = torch.empty((1,), dtype=torch.float32, device=feats.device)
        self._check(self.lib.knn_pivot_train_step(self.h, ctypes.c_void_p(feats.data_ptr()),
                                                  ctypes.c_void_p(targets.data_ptr()), feats.shape[0], quantile,
                                                  lr, ctypes.c_void_p(loss.data_ptr()), self._stream()))
        return loss

    def pivot_add_examples(self, dist, k: int):
        """Appends one training example (features, standardised exact k-th
        value) per row of a 2-D FP32 device matrix; returns the example count."""
        rows, cols = dist.shape
        self._check(self.lib.knn_pivot_add_examples(self.h, ctypes.c_void_p(dist.data_ptr()), rows, cols,
                                                    max(dist.stride(0), cols), k, self._stream()))
        return self.pivot_example_count()

    def pivot_example_count(self) -> int:
        c = ctypes.c_int64()
        self._check(self.lib.knn_pivot_example_count(self.h, ctypes.byref(c)))
        return int(c.value)

    def pivot_examples(self):
        """The stored examples: (features [n, 8], targets [n]) device tensors."""
        torch = _torch()
        n = self.pivot_example_count()
        f = torch.empty((max(n, 1), 8), dtype=torch.float32, device=f"cuda:{self.device}")
        y = torch.empty((max(n, 1),), dtype=torch.float32, device=f"cuda:{self.device}")
        torch.cuda.synchronize(self.device)
        self._check(self.lib.knn_pivot_get_examples(self.h, ctypes.c_void_p(f.data_ptr()),
                                                    ctypes.c_void_p(y.data_ptr()), max(n, 1)))
        return f[:n], y[:n]

    def pivot_clear_examples(self):
        self._check(self.lib.knn_pivot_clear_examples(self.h))

    def pivot_train(self, out_path=None, seed: int = 1000, steps: int = 3000):
        """Trains the pivot network on the stored examples (all on the device);
        writes the weights file when out_path is given."""
        torch = _torch()
        torch.cuda.synchronize(self.device)
        self._check(self.lib.knn_pivot_train(self.h, None if out_path is None else str(out_path).encode(),
                                             int(seed), int(steps)))

    def graph(self, points, k: int, pivot="sample", precision="fp32", oversample=4, flags=0,
              metric="sqeuclidean"):
        """k-NN graph of the rows of `points` (own index excluded).
        Returns (dist [n, k] f32, idx [n, k] i32)."""
        torch = _torch()
        if points.dim() != 2 or points.dtype != torch.float32 or not points.is_cuda or not points.is_contiguous():
            raise ValueError("points must be a contiguous 2-D float32 device tensor")
        n, d = points.shape
        dist = torch.empty((n, k), dtype=torch.float32, device=points.device)
        idx = torch.empty((n, k), dtype=torch.int32, device=points.device)
        o = self._opts(pivot, precision, oversample, flags, metric)
        self._check(self.lib.knn_graph(self.h, ctypes.c_void_p(points.data_ptr()), n, d, k,
                                       ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                       self._stream(), ctypes.byref(o)))
        return dist, idx


_default = {}


def handle(device: int = 0) -> Handle:
    if device not in _default:
        _default[device] = Handle(device)
    return _default[device]
