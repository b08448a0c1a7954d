"""knn_batch_search: uneven jobs pooled into one grouped product launch with
captured HIP graphs.  Every job must give exactly the bits knn_search /
knn_graph give for it (same plan, same products, same selection), replays of
the captured graphs and the eager path must agree bit for bit, and sampled rows
are checked against the FP64 oracle."""
import os
import sys
import tempfile

import numpy as np
import pytest

import synth
from knn_check import compare

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def knn():
    import paper_1309_5478_amd as k
    return k


@pytest.fixture(scope="module")
def h(torch, knn):
    return knn.Handle(0)


# (kind, m, n, d, k, graph): uneven corpus sizes, dimensions (including ones
# that are not multiples of 4, which leave the grouped launch) and k, one empty
# job, k above the corpus size (padded rows), and graph jobs
JOBS = [
    ("gmm", 1024, 70000, 128, 64, False),
    ("uniform", 300, 1000, 64, 1, False),
    ("gmm", 1024, 20000, 768, 300, False),
    ("uniform", 77, 5000, 33, 16, False),
    ("gmm", 0, 4000, 64, 8, False),
    ("uniform", 1024, 900, 64, 1000, False),     # k > n: 124 padded columns
    ("gmm", 2000, 2000, 128, 32, True),          # graph job
    ("normal", 513, 33000, 17, 5, False),
    ("uniform", 1, 3000, 256, 1024, False),
    ("gmm", 1500, 1500, 64, 1024, True),          # graph job, k > n - 1
]


def points(kind, n, d, seed):
    if kind == "uniform":
        return synth.uniform_points(n, d, seed)
    if kind == "normal":
        return synth.normal_points(n, d, seed)
    return synth.gmm_points(n, d, seed)


@pytest.fixture(scope="module")
def data(torch):
    base = synth.SEEDS["batch"] * 1000
    out = []
    for t, (kind, m, n, d, k, graph) in enumerate(JOBS):
        C = points(kind, n, d, base + 2 * t)
        Q = None if graph else points(kind, m, d, base + 2 * t + 1)
        out.append(dict(kind=kind, m=m, n=n, d=d, k=k, graph=graph, C=C, Q=Q,
                        Cd=torch.from_numpy(C).cuda(), Qd=None if graph else torch.from_numpy(Q).cuda()))
    return out


def job_list(data):
    return [(None if j["graph"] else j["Qd"], j["Cd"], j["k"]) for j in data]


def reference(h, j, **kw):
    """Per-job knn_search / knn_graph with k capped to the eligible corpus;
    the capped-off columns are +inf / -1."""
    import torch
    n_elig = j["n"] - (1 if j["graph"] else 0)
    kc = min(j["k"], n_elig)
    m = j["m"]
    dist = torch.full((m, j["k"]), float("inf"), device="cuda")
    idx = torch.full((m, j["k"]), -1, dtype=torch.int32, device="cuda")
    if m:
        d, i = h.graph(j["Cd"], kc, **kw) if j["graph"] else h.search(j["Qd"], j["Cd"], kc, **kw)
        dist[:, :kc] = d
        idx[:, :kc] = i
    return dist, idx


def bits(t):
    return t.cpu().numpy().view(np.uint32)


def assert_same(got, want, what):
    for t, ((gd, gi), (wd, wi)) in enumerate(zip(got, want)):
        assert gd.shape == wd.shape, (what, t)
        assert np.array_equal(gi.cpu().numpy(), wi.cpu().numpy()), f"{what}: job {t} indices differ"
        assert np.array_equal(bits(gd), bits(wd)), f"{what}: job {t} distances differ"


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_batch_equals_per_job_calls(h, torch, data, precision):
    jobs = job_list(data)
    say(f"batch of {len(jobs)} jobs, {precision}")
    got = h.batch_search(jobs, precision=precision)
    torch.cuda.synchronize()
    st = h.stats()
    want = [reference(h, j, precision=precision) for j in data]
    torch.cuda.synchronize()
    assert_same(got, want, f"batch vs per-job ({precision})")
    assert st["rows"] >= sum(j["m"] for j in data)


def test_batch_rows_against_oracle(h, torch, data):
    jobs = job_list(data)
    got = h.batch_search(jobs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for t, j in enumerate(data):
        if j["m"] == 0:
            continue
        gd, gi = got[t][0].cpu().numpy(), got[t][1].cpu().numpy()
        n_elig = j["n"] - (1 if j["graph"] else 0)
        kc = min(j["k"], n_elig)
        if kc < j["k"]:  # padding
            assert np.all(np.isinf(gd[:, kc:])) and np.all(gi[:, kc:] == -1), f"job {t}: padding"
        rows = np.unique(rng.integers(0, j["m"], 6))
        Q = j["C"] if j["graph"] else j["Q"]
        sid = np.arange(j["n"]) if j["graph"] else None
        near = compare(Q, j["C"], kc, gd[rows, :kc], gi[rows, :kc], rows, self_ids=sid)
        say(f"job {t}: {len(rows)} rows vs oracle, near ties {near}")


def test_batch_replay_and_eager_agree(h, knn, torch, data):
    jobs = job_list(data)
    first = h.batch_search(jobs)                    # plans and captures
    torch.cuda.synchronize()
    snap = [(d.clone(), i.clone()) for d, i in first]
    for d, i in first:                              # poison the outputs, replay into them
        d.fill_(-1.0)
        i.fill_(7)
    for rep in range(3):
        again = h.batch_search(jobs, out=first)
        torch.cuda.synchronize()
        assert_same(again, snap, f"replay {rep}")
        x = torch.ones(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert float(x) == float(1 << 20)
    eager = h.batch_search(jobs, flags=knn.FLAG_NO_GRAPH)
    torch.cuda.synchronize()
    assert_same(eager, snap, "eager")


def test_batch_forced_fallback_and_unfused(h, knn, torch, data):
    jobs = job_list(data)
    base = h.batch_search(jobs)
    torch.cuda.synchronize()
    forced = h.batch_search(jobs, flags=knn.FLAG_FORCE_FALLBACK)
    torch.cuda.synchronize()
    st = h.stats()
    # every row on the filtering path is re-done; corpora of at most 2048 points
    # are their own threshold sample and never filter, corpora above 16384
    # points always do
    assert sum(j["m"] for j in data if j["n"] > 16384) <= st["fallback_rows"]
    assert st["fallback_rows"] <= sum(j["m"] for j in data if j["n"] > 2048)
    assert_same(forced, base, "forced fallback")
    unf = h.batch_search(jobs, flags=knn.FLAG_UNFUSED)
    torch.cuda.synchronize()
    assert_same(unf, base, "unfused")


def test_batch_timing_and_autotune(h, knn, torch, data):
    jobs = job_list(data)
    base = h.batch_search(jobs)
    torch.cuda.synchronize()
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        os.environ["KNN_AUTOTUNE_CACHE"] = path
        try:
            tuned = h.batch_search(jobs, flags=knn.FLAG_AUTOTUNE | knn.FLAG_TIMING)
            torch.cuda.synchronize()
            st = h.stats()
            assert_same(tuned, base, "autotuned + timed")
            assert st["product_launches"] == 1 and st["product_ms"] > 0
            text = open(path).read()
            assert "grouped|" in text, text
            say(f"autotune cache: {text.strip()}")
            again = h.batch_search(jobs, flags=knn.FLAG_AUTOTUNE | knn.FLAG_TIMING)
            torch.cuda.synchronize()
            assert_same(again, base, "autotuned replay")
        finally:
            del os.environ["KNN_AUTOTUNE_CACHE"]


def test_batch_queue_form_same_bits(knn, torch, data):
    """The product as a resident grid over per-XCD item queues gives the same
    bits as one workgroup per item, for every tile shape (small1: the
    single-stage tile, one workgroup per item only)."""
    jobs = job_list(data)
    want = None
    for tile in ("small", "small1", "wide", "big"):
        for queue in (("0",) if tile == "small1" else ("0", "1")):
            os.environ["KNN_GEMM_TILE"] = tile
            os.environ["KNN_BATCH_QUEUE"] = queue
            try:
                hq = knn.Handle(0)   # a fresh plan reads the settings
                got = hq.batch_search(jobs)
                torch.cuda.synchronize()
            finally:
                del os.environ["KNN_BATCH_QUEUE"]
                del os.environ["KNN_GEMM_TILE"]
            if want is None:
                want = got
            else:
                assert_same(got, want, f"tile {tile}, queue {queue}")
            del hq


def test_batch_learned_pivot(knn, torch, data):
    hl = knn.Handle(0)   # packaged pivot network
    jobs = job_list(data)
    got = hl.batch_search(jobs, pivot="learned")
    torch.cuda.synchronize()
    want = [reference(hl, j, pivot="learned") for j in data]
    torch.cuda.synchronize()
    assert_same(got, want, "learned pivot")


def test_batch_large_job_is_split(h, torch):
    """A graph job of more than 32768 points is split into row parts."""
    P = synth.gmm_points(40000, 64, seed=synth.SEEDS["batch"] * 1000 + 99)
    Pd = torch.from_numpy(P).cuda()
    got = h.batch_search([(None, Pd, 8)])
    want = h.graph(Pd, 8)
    torch.cuda.synchronize()
    assert_same(got, [want], "split job")


def test_batch_errors(h, knn, torch):
    C = torch.zeros((100, 8), device="cuda")
    Q = torch.zeros((10, 8), device="cuda")
    with pytest.raises(knn.KnnError) as ei:
        h.batch_search([(Q, C, 4), (Q, C, 0)])
    assert ei.value.status == 1 and "job 1" in str(ei.value)
    with pytest.raises(knn.KnnError) as ei:
        h.batch_search([(Q, C, 1025)])
    assert ei.value.status == 3
    assert h.batch_search([]) == []


def test_batch_full_workload(h, knn, torch):
    """The full batched workload as the benchmark runs it (512 jobs, about
    100 GB of corpora drawn on the device, learned pivots, autotuned tiles,
    graph replay): every job's output equals its own knn_search call bit for
    bit, and 16 sampled rows of each of 32 jobs agree with the FP64 oracle."""
    import oracle
    from synth.gpu import batch_jobs, job_points
    J = batch_jobs()
    data = [job_points(j) for j in J]
    jobs = [(q, c, j["k"]) for (q, c), j in zip(data, J)]
    say(f"full batch: {len(J)} jobs, {sum(j['n'] * j['d'] * 4 for j in J) / 1e9:.1f} GB")
    first = h.batch_search(jobs, pivot="learned", flags=knn.FLAG_AUTOTUNE)
    got = h.batch_search(jobs, pivot="learned", flags=knn.FLAG_AUTOTUNE, out=first)   # replay
    torch.cuda.synchronize()
    say("batch done; per-job calls")
    for t, ((q, c), j) in enumerate(zip(data, J)):
        kc = min(j["k"], j["n"])
        wd, wi = h.search(q, c, kc, pivot="learned")
        gd, gi = got[t]
        assert np.array_equal(gi[:, :kc].cpu().numpy(), wi.cpu().numpy()), f"job {t} indices"
        assert np.array_equal(bits(gd[:, :kc]), bits(wd)), f"job {t} distances"
        if kc < j["k"]:
            assert bool(torch.all(gi[:, kc:] == -1)), f"job {t} padding"
    say("per-job parity done; oracle rows")
    rng = np.random.default_rng(11)
    for t in rng.choice(len(J), 32, replace=False):
        q, c = data[t]
        rows = np.sort(rng.choice(J[t]["m"], 16, replace=False))
        kc = min(J[t]["k"], J[t]["n"])
        Qh = q.cpu().numpy()
        Ch = c.cpu().numpy()
        gd, gi = got[t][0].cpu().numpy(), got[t][1].cpu().numpy()
        near = compare(Qh, Ch, kc, gd[rows, :kc], gi[rows, :kc], rows)
        say(f"job {t} (n={J[t]['n']}, d={J[t]['d']}, k={J[t]['k']}): 16 rows vs oracle, near ties {near}")
        del Qh, Ch
