"""Brute-force definitions on tiny inputs, in pure Python, independent of the C oracle.

* ``select_by_subsets``: the k-smallest set of a row is the unique k-subset S such
  that every key in S is below every key outside S, keys being (value, index)
  under the FP32 total order (-0 == +0, NaN == NaN above +inf).  Found by
  enumerating all k-subsets.
* ``knn_pairwise``: squared Euclidean distances summed term by term in Python
  floats (FP64), neighbours found by repeatedly taking the minimum remaining key.
"""
from __future__ import annotations

import itertools
import math


def key_less(a, ia, b, ib):
    an, bn = math.isnan(a), math.isnan(b)
    if an != bn:
        return bn
    if not an and a != b:
        return a < b
    return ia < ib


def select_by_subsets(row, k):
    n = len(row)
    found = []
    for sub in itertools.combinations(range(n), k):
        s = set(sub)
        if all(key_less(row[i], i, row[j], j) for i in s for j in range(n) if j not in s):
            found.append(sub)
    assert len(found) == 1, "the k-smallest set must be unique under a total order"
    chosen = list(found[0])
    # order the chosen indices by key, by repeated minimum
    ordered = []
    while chosen:
        best = chosen[0]
        for c in chosen[1:]:
            if key_less(row[c], c, row[best], best):
                best = c
        ordered.append(best)
        chosen.remove(best)
    return ordered


def knn_pairwise(Q, C, k, self_ids=None):
    out_d, out_i = [], []
    for qi, q in enumerate(Q):
        cand = []
        for ci, c in enumerate(C):
            if self_ids is not None and ci == self_ids[qi]:
                continue
            s = 0.0
            for a, b in zip(q, c):
                s += (float(a) - float(b)) ** 2
            cand.append((s, ci))
        picked = []
        for _ in range(min(k, len(cand))):
            best = min(cand)          # tuple order: distance, then lower index
            picked.append(best)
            cand.remove(best)
        out_d.append([p[0] for p in picked])
        out_i.append([p[1] for p in picked])
    return out_d, out_i
