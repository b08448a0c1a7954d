"""CPU oracle for the quick multi-select k-NN hot path (arXiv:1309.5478).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.

* ``select_k``  -- plain definition of per-row k-smallest selection (the paper's
  brute-force description in the Introduction): stable sort of each row under
  the FP32 total order (-0 == +0, NaN == NaN > +inf), first k kept, values
  copied verbatim.  C, ``knn_oracle.c``.
* ``knn``       -- FP64 direct-form squared Euclidean distances (Methods,
  "Distance calculation") + stable sort, ties to the lower corpus index, own
  index excluded for the k-NNG.  C, ``knn_oracle.c``.
* ``partition`` -- one partition pass of a segment around a pivot as the
  "GPU-based quick multi-select" subsection describes it: elements below the
  pivot fill the output from the left in input order, the others fill it from
  the right end (so they appear in reverse input order).  numpy.
* ``mlp``       -- FP64 forward/backward of the pivot network (see ``mlp.py``).
* ``quant``     -- BF16 and OCP e4m3 conversions from the formats' definitions.
* ``nth_select_k`` -- not a reference: the std::nth_element CPU baseline the
  benchmark times beside the GPU selection (checked against ``select_k``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_NTH_SRC = os.path.join(_HERE, "nth_baseline.cpp")
_NTH_LIB = os.path.join(_HERE, "libnth.so")
_lib = None
_nth = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP contraction off), and the nth_element
    CPU baseline with g++."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-pthread",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    if force or not os.path.exists(_NTH_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _NTH_SRC, "-o", _NTH_LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_NTH_LIB + ".tmp", _NTH_LIB)
    return _LIB


def _load_nth():
    global _nth
    if _nth is None:
        if not os.path.exists(_NTH_LIB) or os.path.getmtime(_NTH_LIB) < os.path.getmtime(_NTH_SRC):
            build()
        lib = ctypes.CDLL(_NTH_LIB)
        P = ctypes.c_void_p
        lib.nth_select_k.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P,
                                     ctypes.c_int32]
        lib.nth_select_k.restype = ctypes.c_int
        _nth = lib
    return _nth


def nth_select_k(D: np.ndarray, k: int, nthreads: int = 0):
    """CPU comparison baseline (std::nth_element + sort of the first k per row;
    not the oracle).  Returns (values float32 [r, k], indices int32 [r, k])."""
    D = np.ascontiguousarray(D, dtype=np.float32)
    rows, cols = D.shape
    vals = np.empty((rows, k), np.float32)
    idx = np.empty((rows, k), np.int32)
    st = _load_nth().nth_select_k(_ptr(D), rows, cols, cols, k, _ptr(vals), _ptr(idx), nthreads)
    if st != 0:
        raise ValueError(f"nth_select_k failed with status {st}")
    return vals, idx


def bind(path: str):
    """Load an oracle shared library built from knn_oracle.c (or a test's variant of it)."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_select_k.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32, P, P, ctypes.c_int32]
    lib.oracle_select_k.restype = ctypes.c_int
    lib.oracle_knn.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, P, P, P, ctypes.c_int32]
    lib.oracle_knn.restype = ctypes.c_int
    lib.oracle_default_threads.restype = ctypes.c_int
    if hasattr(lib, "oracle_knn_metric"):
        lib.oracle_knn_metric.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                          P, P, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_knn_metric.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = bind(_LIB)
    return _lib


def default_threads() -> int:
    return int(_load().oracle_default_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def select_k(D: np.ndarray, k: int, rows=None, nthreads: int = 0, lib=None):
    """k smallest per row of FP32 matrix D (optionally only the listed rows).
    Returns (values float32 [r, k], indices int32 [r, k])."""
    D = np.ascontiguousarray(D, dtype=np.float32)
    if D.ndim == 1:
        D = D[None, :]
    nr, cols = D.shape
    rid = None
    if rows is not None:
        rid = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rid.shape[0]
    vals = np.empty((nr, k), np.float32)
    idx = np.empty((nr, k), np.int32)
    st = (lib or _load()).oracle_select_k(_ptr(D), nr, _ptr(rid), cols, cols, k, _ptr(vals), _ptr(idx), nthreads)
    if st != 0:
        raise ValueError(f"oracle_select_k failed with status {st}")
    return vals, idx


METRICS = {"sqeuclidean": 0, "cosine": 1, "pearson": 2}


def knn(Q: np.ndarray, C: np.ndarray, k: int, self_ids=None, nthreads: int = 0, lib=None, metric="sqeuclidean"):
    """k nearest rows of C to each row of Q by FP64 direct squared distance
    (or, with metric, cosine distance 1 - cos, or Pearson distance 1 - r: the
    cosine distance of the mean-centred vectors; NaN for a zero-norm vector).
    self_ids[i] (if given) is the corpus index excluded for query i.
    Returns (dist float64 [m, k], idx int32 [m, k]); missing entries (+inf, -1)."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    m, d = Q.shape
    n, d2 = C.shape
    if d != d2:
        raise ValueError("dimension mismatch")
    sid = None if self_ids is None else np.ascontiguousarray(self_ids, dtype=np.int64)
    dist = np.empty((m, k), np.float64)
    idx = np.empty((m, k), np.int32)
    st = (lib or _load()).oracle_knn_metric(_ptr(Q), m, _ptr(C), n, d, k, _ptr(sid), _ptr(dist), _ptr(idx),
                                            nthreads, METRICS[metric])
    if st != 0:
        raise ValueError(f"oracle_knn failed with status {st}")
    return dist, idx


def total_order_less(a: float, ia: int, b: float, ib: int) -> bool:
    """(a, ia) < (b, ib) under the FP32 total order, index breaking ties."""
    an, bn = np.isnan(a), np.isnan(b)
    if an != bn:
        return bool(bn)
    if not an and a != b:
        return bool(a < b)
    return ia < ib


def partition(seg_vals: np.ndarray, seg_idx: np.ndarray, piv_val: float, piv_idx: int):
    """One partition pass of a segment around a pivot key (value, index).

    Keys below the pivot go to the left of the output in input order; the other
    keys go to the right end, the first of them in the last slot, so the right
    side holds them in reverse input order.  Returns (out_vals, out_idx, L)."""
    n = seg_vals.shape[0]
    out_v = np.empty(n, np.float32)
    out_i = np.empty(n, np.int32)
    left, right = 0, n - 1
    for t in range(n):
        if total_order_less(float(seg_vals[t]), int(seg_idx[t]), piv_val, piv_idx):
            out_v[left], out_i[left] = seg_vals[t], seg_idx[t]
            left += 1
        else:
            out_v[right], out_i[right] = seg_vals[t], seg_idx[t]
            right -= 1
    return out_v, out_i, left
