"""Row-by-row check of k-NN results against the FP64 oracle, shared by the GPU
test modules.

Bar: neighbour sets equal per row, except where the oracle's FP64 gap between
the k-th and the (k+1)-th distance is within the 1e-5 relative band (counted
and returned, not failed); returned squared distances within 1e-5 relative of
FP64 (1e-6 of ||q||^2 + ||c||^2 for exact zeros); rows in ascending
(distance, index) order."""
import numpy as np

import oracle

REL = 1e-5


def d64(q, c):
    diff = q.astype(np.float64) - c.astype(np.float64)
    return float(np.dot(diff, diff))


def compare(Q, C, k, gd, gi, rows, self_ids=None):
    """Compares GPU rows (gd, gi for the listed query rows) with the oracle.
    Returns the number of rows whose set differs only inside the near-tie band."""
    qs = Q[rows]
    sid = None if self_ids is None else np.asarray(self_ids)[rows]
    n_elig = C.shape[0] - (0 if sid is None else 1)
    kk = min(k + 1, n_elig)
    od, oi = oracle.knn(qs, C, kk, self_ids=sid)
    near = 0
    for t, r in enumerate(rows):
        g_idx = [int(x) for x in gi[t]]
        assert len(set(g_idx)) == k, f"row {r}: duplicate indices"
        assert all(0 <= j < C.shape[0] for j in g_idx), f"row {r}: index out of range"
        if sid is not None:
            assert int(sid[t]) not in g_idx, f"row {r}: own index returned"
        # distances against FP64 direct form, for whatever indices were returned
        for dist, j in zip(gd[t], g_idx):
            ref = d64(Q[r], C[j])
            if ref == 0.0:
                tol = 1e-6 * (d64(Q[r], 0 * Q[r]) + d64(C[j], 0 * C[j]))
                assert abs(float(dist)) <= tol, (r, j, dist)
            else:
                assert abs(float(dist) - ref) <= REL * ref, (r, j, float(dist), ref)
        # ascending (distance, index)
        for a in range(k - 1):
            assert (gd[t, a], g_idx[a]) <= (gd[t, a + 1], g_idx[a + 1]) or gd[t, a] < gd[t, a + 1], (r, a)
        want = [int(x) for x in oi[t, :k]]
        if set(g_idx) != set(want):
            kth = od[t, k - 1]
            diff = set(g_idx) ^ set(want)
            band = max(kth, 1e-30) * REL
            for j in diff:
                dj = d64(Q[r], C[j])
                assert abs(dj - kth) <= band, f"row {r}: set differs beyond the near-tie band ({j}: {dj} vs {kth})"
            near += 1
        elif g_idx != want:
            # same set, different order: only legal among FP32-equal distances
            for a in range(k):
                if g_idx[a] != want[a]:
                    assert abs(d64(Q[r], C[g_idx[a]]) - d64(Q[r], C[want[a]])) <= REL * max(od[t, a], 1e-30)
    return near


def metric_tol(ref, d):
    """Cosine / Pearson distance bar: 1e-5 relative, plus the FP32 error of the
    unit vectors the GPU ranks (per element at most eps_d relative, eps_d =
    (ceil(d / 64) + 16) 2^-24 for the norm's lane sums, the two divisions and
    the centring), which moves |u - v|^2 / 2 by at most 2 eps_d |u - v|."""
    eps = (np.ceil(d / 64.0) + 16.0) * 2.0 ** -24
    return REL * np.abs(ref) + 2.0 * eps * np.sqrt(2.0 * np.maximum(ref, 0.0)) + 4.0 * eps * np.abs(ref)


def compare_metric(Q, C, k, gd, gi, rows, metric, self_ids=None):
    """compare() for the cosine / Pearson distances (1 - similarity): sets equal
    outside the near-tie band of metric_tol at the k-th distance, distances of
    the returned points within metric_tol of the oracle's, NaN exactly where the
    oracle's is NaN, rows ascending.  Returns the near-tie row count."""
    qs = Q[rows]
    d = Q.shape[1]
    sid = None if self_ids is None else np.asarray(self_ids)[rows]
    n_elig = C.shape[0] - (0 if sid is None else 1)
    kk = min(k + 1, n_elig)
    od, oi = oracle.knn(qs, C, kk, self_ids=sid, metric=metric)
    near = 0
    for t, r in enumerate(rows):
        g_idx = [int(x) for x in gi[t]]
        assert len(set(g_idx)) == k, f"row {r}: duplicate indices"
        if sid is not None:
            assert int(sid[t]) not in g_idx, f"row {r}: own index returned"
        # the oracle's distances of exactly the returned points
        sub_d, sub_i = oracle.knn(Q[r:r + 1], C[g_idx], k, metric=metric)
        ref = np.empty(k)
        ref[sub_i[0]] = sub_d[0]
        g = gd[t].astype(np.float64)
        assert np.array_equal(np.isnan(g), np.isnan(ref)), f"row {r}: NaN pattern"
        fin = ~np.isnan(ref)
        assert np.all(np.abs(g[fin] - ref[fin]) <= metric_tol(ref[fin], d)), \
            (r, float(np.max(np.abs(g[fin] - ref[fin]))))
        for a in range(k - 1):   # ascending, NaN last, ties by index
            x, y = g[a], g[a + 1]
            assert np.isnan(y) or (not np.isnan(x) and (x < y or (x == y and g_idx[a] < g_idx[a + 1]))), (r, a)
        want = [int(x) for x in oi[t, :k]]
        if set(g_idx) != set(want):
            kth = od[t, k - 1]
            assert not np.isnan(kth), f"row {r}: set differs in the NaN class"
            band = metric_tol(np.array([kth]), d)[0]
            for j in set(g_idx) ^ set(want):
                dj = oracle.knn(Q[r:r + 1], C[j:j + 1], 1, metric=metric)[0][0, 0]
                assert abs(dj - kth) <= band, f"row {r}: set differs beyond the near-tie band ({j}: {dj} vs {kth})"
            near += 1
    return near
