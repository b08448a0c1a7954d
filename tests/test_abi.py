"""The C-ABI library loads, exports every symbol include/knn.h declares, and its
host-side argument checks answer without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1309_5478_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(knn_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("knn_create", "knn_destroy", "knn_select_k", "knn_partition", "knn_get_stats"):
        assert must in names


@pytest.mark.parametrize("name", declared_symbols())
def test_symbol_exported(lib, name):
    assert hasattr(lib, name), f"{name} declared in include/ but not exported by libknn.so"


def test_prototypes_cover_header():
    missing = [n for n in declared_symbols() if n not in _abi.PROTOTYPES]
    assert not missing, f"binding lacks prototypes for {missing}"


def test_status_strings(lib):
    assert lib.knn_status_string(0) == b"success"
    assert lib.knn_status_string(1) == b"invalid value"
    assert lib.knn_status_string(3) == b"unsupported"
    assert lib.knn_status_string(99) == b"unknown status"


def test_null_handle_rejected_without_launch(lib):
    st = lib.knn_select_k(None, None, 4, 8, 8, 2, None, None, None, None)
    assert st == _abi.KNN_ERROR_INVALID_VALUE
    assert b"handle is null" in lib.knn_last_error(None)
    st = lib.knn_partition(None, None, 1, 1, 1, None, None, None, None, None, None)
    assert st == _abi.KNN_ERROR_INVALID_VALUE
    jobs = (_abi.Job * 1)()
    st = lib.knn_batch_search(None, jobs, 1, None, None)
    assert st == _abi.KNN_ERROR_INVALID_VALUE
    assert lib.knn_destroy(None) == 0
    s = _abi.Stats()
    assert lib.knn_get_stats(None, ctypes.byref(s)) == _abi.KNN_ERROR_INVALID_VALUE


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.knn_create(ctypes.byref(h), 0) == _abi.KNN_ERROR_DEVICE
    assert not h.value
    assert lib.knn_create(None, 0) == _abi.KNN_ERROR_INVALID_VALUE


def test_job_struct_layout():
    # knn_job_t: pointer, int64, pointer, int64, int32, int32, pointer, pointer
    assert ctypes.sizeof(_abi.Job) == 56
    assert _abi.Job.d.offset == 32 and _abi.Job.k.offset == 36 and _abi.Job.out_idx.offset == 48
