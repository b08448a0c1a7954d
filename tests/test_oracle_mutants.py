"""The oracle's pins are strong enough: each plausible mistake planted in a copy of
the C oracle (built on the CPU, in a temporary directory) fails at least one pin."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from brute import knn_pairwise, select_by_subsets
from golden_io import lattice_cases, select_cases

SRC = os.path.join(os.path.dirname(oracle.__file__), "knn_oracle.c")

MUTANTS = {
    "ties_to_higher_index": ("if (key_cmp(keys, src[j], src[i]) < 0)", "if (key_cmp(keys, src[j], src[i]) <= 0)"),
    "nan_lowest": ("if (an || bn) return an - bn;          /* NaN above everything, NaN == NaN */",
                   "if (an || bn) return bn - an;"),
    "signed_zero_order": ("if (a < b) return -1;                  /* IEEE: -0 == +0 */",
                          "if (a < b || (a == b && signbit(a) && !signbit(b))) return -1;"),
    "self_not_excluded": ("if (c == self) continue;", "if (c == self && 0) continue;"),
    "dropped_square": ("s += diff * diff;", "s += fabs(diff);"),
    "sign_flip": ("double diff = (double)q[t] - (double)y[t];", "double diff = (double)q[t] + (double)y[t];"),
    "corpus_stride": ("const float *y = j->C + c * (int64_t)j->d;", "const float *y = j->C + c;"),
    "values_not_verbatim": ("memcpy(&j->out_val[p * j->k + t], &row[idx[t]], sizeof(float));",
                            "j->out_val[p * j->k + t] = row[idx[t]] + 0.0f;"),
    "dropped_last_term": ("for (int32_t t = 0; t < j->d; ++t) {\n            double diff",
                          "for (int32_t t = 0; t + 1 < j->d; ++t) {\n            double diff"),
    "pearson_not_centred": ("if (metric == 2) {", "if (metric == 3) {"),
    "cosine_similarity_not_distance": ("return 1.0 - dot / (qnorm * yn);", "return dot / (qnorm * yn);"),
    "cosine_norm_squared": ("*norm = sqrt(s);", "*norm = s;"),
    "pearson_norm_uncentred": ("double v = (double)x[t] - mu;", "double v = (double)x[t];"),
}


def _battery(lib):
    """Runs the oracle pins against `lib`; returns the names of the pins that fail."""
    failed = set()
    for vals, k, idx, vbits in select_cases():
        v, i = oracle.select_k(np.array([vals], np.float32), k, lib=lib)
        got = np.asarray(v[0], np.float32).view(np.uint32).tolist()
        nan_ok = all(np.isnan(np.float32(np.uint32(e).view(np.float32))) or g == e for g, e in zip(got, vbits))
        if i[0].tolist() != idx or not nan_ok:
            failed.add("select_hand")
    pool = np.array([0.0, -0.0, 1.0, 1.0, 2.5, -3.0, np.inf, -np.inf, np.nan, 7.0], np.float32)
    for seed in range(20):
        row = np.random.default_rng(seed).choice(pool, size=8).astype(np.float32)
        for k in range(1, 9):
            _, i = oracle.select_k(row[None], k, lib=lib)
            if i[0].tolist() != select_by_subsets([float(x) for x in row], k):
                failed.add("select_brute")
    P = np.arange(5, dtype=np.float32)[:, None]
    for k, node, idx, dist in lattice_cases():
        d, i = oracle.knn(P, P, k, self_ids=np.arange(5), lib=lib)
        if i[node].tolist() != idx or d[node].tolist() != dist:
            failed.add("lattice")
    rng = np.random.default_rng(1)
    Q = rng.integers(-3, 4, size=(4, 3)).astype(np.float32)
    C = rng.integers(-3, 4, size=(9, 3)).astype(np.float32)
    d, i = oracle.knn(Q, C, 5, lib=lib)
    bd, bi = knn_pairwise(Q.tolist(), C.tolist(), 5)
    if i.tolist() != bi or d.tolist() != bd:
        failed.add("knn_brute")
    Q = rng.random((6, 7)).astype(np.float32)
    C = rng.random((20, 7)).astype(np.float32)
    d, i = oracle.knn(Q, C, 20, lib=lib)
    ref = cdist(Q.astype(np.float64), C.astype(np.float64), "sqeuclidean")
    for r in range(6):
        if not np.allclose(d[r], ref[r, i[r]], rtol=1e-12, atol=0):
            failed.add("scipy")
    # cosine and Pearson distances against scipy's cosine and correlation
    Q = (rng.random((5, 9)) - 0.3).astype(np.float32)
    C = (rng.random((30, 9)) - 0.3).astype(np.float32)
    for metric, name in (("cosine", "cosine"), ("pearson", "correlation")):
        d, i = oracle.knn(Q, C, 30, lib=lib, metric=metric)
        ref = cdist(Q.astype(np.float64), C.astype(np.float64), name)
        for r in range(5):
            if not np.allclose(d[r], ref[r, i[r]], rtol=1e-10, atol=1e-14) or not (np.diff(d[r]) >= 0).all():
                failed.add("scipy_" + metric)
    return failed


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-pthread",
                           str(src), "-o", str(so), "-lm"])
    return oracle.bind(str(so))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_unmutated_oracle_passes_battery(tmp_path):
    lib = _build(tmp_path, "orig", open(SRC).read())
    assert _battery(lib) == set()


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert old in text, f"mutation site for {name} not found"
    lib = _build(tmp_path, name, text.replace(old, new, 1))
    assert _battery(lib), f"planted mistake {name} passed every pin"
