"""ctypes prototypes for libknn.so (include/knn.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libknn.so")

KNN_SUCCESS = 0
KNN_ERROR_INVALID_VALUE = 1
KNN_ERROR_OUT_OF_MEMORY = 2
KNN_ERROR_UNSUPPORTED = 3
KNN_ERROR_DEVICE = 4
KNN_ERROR_IO = 5

PIVOT_PLAIN, PIVOT_SAMPLE, PIVOT_LEARNED = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP8_E4M3 = 0, 1, 2
METRIC_SQEUCLIDEAN, METRIC_COSINE, METRIC_PEARSON = 0, 1, 2
FLAG_FORCE_FALLBACK = 0x1
FLAG_UNFUSED = 0x2
FLAG_TIMING = 0x4
FLAG_NO_GRAPH = 0x8
FLAG_AUTOTUNE = 0x10
FLAG_FORCE_RERUN = 0x20
FLAG_NO_SPLIT = 0x40
FLAG_FORCE_SPLIT = 0x80
PIVOT_NPARAM = 4801


class Options(ctypes.Structure):
    _fields_ = [("pivot", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("metric", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_void_p), ("m", ctypes.c_int64), ("corpus", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32),
                ("out_dist", ctypes.c_void_p), ("out_idx", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("passes_total", ctypes.c_int64),
                ("passes_max", ctypes.c_int32), ("split_parts", ctypes.c_int32),
                ("stream_passes_total", ctypes.c_int64), ("spill_rows", ctypes.c_int64),
                ("first_pass_survivors", ctypes.c_int64), ("fallback_rows", ctypes.c_int64),
                ("candidates_total", ctypes.c_int64), ("phase_cycles", ctypes.c_int64 * 4),
                ("product_ms", ctypes.c_double), ("product_launches", ctypes.c_int64),
                ("product_flops", ctypes.c_double), ("rows_uncertified", ctypes.c_int64),
                ("rows_rerun", ctypes.c_int64)]

    def as_dict(self):
        d = {name: int(getattr(self, name)) for name, _ in self._fields_
             if name not in ("phase_cycles", "product_ms", "product_flops")}
        d["product_ms"] = float(self.product_ms)
        d["product_flops"] = float(self.product_flops)
        d["phase_cycles"] = [int(x) for x in self.phase_cycles]
        return d


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_ST = ctypes.c_int

PROTOTYPES = {
    "knn_create": (_ST, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "knn_destroy": (_ST, [_P]),
    "knn_status_string": (ctypes.c_char_p, [_ST]),
    "knn_last_error": (ctypes.c_char_p, [_P]),
    "knn_select_k": (_ST, [_P, _P, _I64, _I64, _I64, _I32, _P, _P, _P, ctypes.POINTER(Options)]),
    "knn_select_k_noalloc": (_ST, [_P, _P, _I64, _I64, _I64, _I32, _P, _P, _P, ctypes.POINTER(Options)]),
    "knn_partition": (_ST, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "knn_search": (_ST, [_P, _P, _I64, _P, _I64, _I32, _I32, _P, _P, _P, ctypes.POINTER(Options)]),
    "knn_search_host_corpus": (_ST, [_P, _P, _I64, _P, _I64, _I32, _I32, _I64, _P, _P, _P, ctypes.POINTER(Options)]),
    "knn_graph": (_ST, [_P, _P, _I64, _I32, _I32, _P, _P, _P, ctypes.POINTER(Options)]),
    "knn_batch_search": (_ST, [_P, ctypes.POINTER(Job), _I32, _P, ctypes.POINTER(Options)]),
    "knn_distances": (_ST, [_P, _P, _I64, _P, _I64, _I32, _P, _I64, _P]),
    "knn_get_stats": (_ST, [_P, ctypes.POINTER(Stats)]),
    "knn_quantize": (_ST, [_P, _P, _I64, _I32, _I32, _P, _P, _P]),
    "knn_pivot_set_weights": (_ST, [_P, _P, _I32]),
    "knn_pivot_get_weights": (_ST, [_P, _P, _I32]),
    "knn_pivot_save": (_ST, [_P, ctypes.c_char_p]),
    "knn_pivot_load": (_ST, [_P, ctypes.c_char_p]),
    "knn_pivot_features": (_ST, [_P, _P, _I64, _I64, _I64, _I32, _P, _P, _P]),
    "knn_pivot_predict": (_ST, [_P, _P, _I64, _P, _P]),
    "knn_pivot_grad": (_ST, [_P, _P, _P, _I64, ctypes.c_float, _P, _P, _P]),
    "knn_pivot_train_step": (_ST, [_P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, _P, _P]),
    "knn_pivot_add_examples": (_ST, [_P, _P, _I64, _I64, _I64, _I32, _P]),
    "knn_pivot_clear_examples": (_ST, [_P]),
    "knn_pivot_example_count": (_ST, [_P, ctypes.POINTER(_I64)]),
    "knn_pivot_get_examples": (_ST, [_P, _P, _P, _I64]),
    "knn_pivot_train": (_ST, [_P, ctypes.c_char_p, ctypes.c_uint64, _I32]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libknn.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(python paper_1309_5478_amd/build.py); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib
