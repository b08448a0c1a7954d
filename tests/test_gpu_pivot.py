"""The pivot network's HIP kernels against the FP64 oracle (features, forward,
loss and gradients), training behaviour, exactness of selection whatever the
weights, and what the trained network gains over the method without it."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

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
    return knn.Handle(0, pivot_weights=None)


def rand_params(seed):
    from paper_1309_5478_amd.pivot_train import he_init
    return he_init(seed, b3=-1.5)


def test_features_match_oracle(h, torch):
    rng = np.random.default_rng(3)
    D = synth.sqdist_matrix_normal(40, 5000, 32, seed=5)
    D[3, :] = rng.integers(0, 9, 5000)               # ties
    D[4, :] = np.sort(D[4])                           # sorted row
    for k in (1, 7, 64, 1000):
        f, ms = h.pivot_features(torch.from_numpy(D).cuda(), k)
        f, ms = f.cpu().numpy(), ms.cpu().numpy()
        for r in range(D.shape[0]):
            x, m, s = mlp.features(mlp.row_sample(D[r]), D.shape[1], k)
            assert abs(ms[r, 0] - m) <= 1e-6 * abs(m) + 1e-6 and abs(ms[r, 1] - s) <= 1e-5 * s
            np.testing.assert_allclose(f[r], x, rtol=2e-4, atol=2e-5)


def test_forward_matches_oracle(h, torch):
    theta = rand_params(11)
    h.pivot_set_weights(theta)
    X = np.random.default_rng(1).normal(0, 1, (257, 8)).astype(np.float32)
    got = h.pivot_predict(torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = mlp.forward(mlp.bf16_round(theta), X.astype(np.float64))
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("q", [0.5, 0.95])
def test_gradient_matches_oracle(h, torch, q):
    theta = rand_params(12)
    h.pivot_set_weights(theta)
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1, (300, 8)).astype(np.float32)
    y = rng.normal(-1, 2, 300).astype(np.float32)
    g, loss = h.pivot_grad(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), q)
    g, loss = g.cpu().numpy().astype(np.float64), float(loss.cpu()[0])
    want_loss, want_g = mlp.loss_and_grad(mlp.bf16_round(theta), X.astype(np.float64), y.astype(np.float64), q)
    assert abs(loss - want_loss) <= 1e-5 * max(1.0, abs(want_loss))
    # per-parameter agreement relative to the gradient's scale
    scale = np.abs(want_g).max()
    assert np.abs(g - want_g).max() <= 1e-4 * scale
    assert np.linalg.norm(g - want_g) <= 1e-5 * np.linalg.norm(want_g) * 10


def test_training_steps_reduce_loss(h, torch):
    h.pivot_set_weights(rand_params(13))
    rng = np.random.default_rng(4)
    X = torch.from_numpy(rng.normal(0, 1, (2048, 8)).astype(np.float32)).cuda()
    y = (X[:, 2] * 3.0 - X[:, 5] + 0.5).contiguous()
    first = float(h.pivot_train_step(X, y, 0.9, 1e-2).cpu()[0])
    for _ in range(200):
        last = float(h.pivot_train_step(X, y, 0.9, 1e-2).cpu()[0])
    assert last < 0.3 * first, (first, last)


def test_training_examples_match_oracle(torch, knn):
    """Examples stored from distance rows: the features and the exact k-th
    value standardised, as the FP64 network oracle and the selection oracle
    compute them; rows with non-finite values are skipped, order kept."""
    hh = knn.Handle(0, pivot_weights=None)
    D = synth.sqdist_matrix_normal(30, 3000, 16, seed=8)
    D[4, 100] = np.nan                  # its k-th value stays finite at small k
    D[6, :] = np.inf                    # dropped: infinite location and target
    dev = torch.from_numpy(D).cuda()
    for k in (3, 40):
        hh.pivot_add_examples(dev, k)
    f, y = hh.pivot_examples()
    f, y = f.cpu().numpy(), y.cpu().numpy()
    t = 0
    for k in (3, 40):
        ov, _ = oracle.select_k(D, k)
        for r in range(D.shape[0]):
            x, m, s_ = mlp.features(mlp.row_sample(D[r]), D.shape[1], k)
            target = (float(ov[r, k - 1]) - m) / s_
            if not (np.all(np.isfinite(x)) and np.isfinite(target)):
                continue
            np.testing.assert_allclose(f[t], x, rtol=2e-4, atol=2e-5)
            assert abs(y[t] - target) <= 1e-4 * max(1.0, abs(target))
            t += 1
    assert t == len(y) and t < 2 * D.shape[0]


def test_train_is_deterministic_and_learns(torch, knn):
    """knn_pivot_train from stored examples: the same seed gives the same
    weights bit for bit, another seed other weights, and the trained network's
    pinball loss is well below the initial one."""
    from paper_1309_5478_amd import pivot_train
    cfgs = [("gmm", 16384, 64, 1500), ("uniform", 16384, 32, 1501), ("normal", 8192, 128, 1502)]
    ws = []
    for seed in (7, 7, 8):
        hh = knn.Handle(0, pivot_weights=None)
        pivot_train.add_rows(hh, cfgs, rows_per_set=64)
        hh.pivot_train(None, seed=seed, steps=0)
        X, y = hh.pivot_examples()
        _, loss0 = hh.pivot_grad(X.contiguous(), y.contiguous(), 0.99)
        hh.pivot_train(None, seed=seed, steps=300)
        _, loss1 = hh.pivot_grad(X.contiguous(), y.contiguous(), 0.99)
        say(f"seed {seed}: {X.shape[0]} examples, pinball loss {float(loss0[0]):.4f} -> {float(loss1[0]):.4f}")
        assert float(loss1[0]) < 0.5 * float(loss0[0])
        ws.append(hh.pivot_get_weights())
    assert np.array_equal(ws[0], ws[1])
    assert not np.array_equal(ws[0], ws[2])


def test_save_load_roundtrip(h, torch, knn):
    theta = rand_params(14)
    h.pivot_set_weights(theta)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "w.bin")
        h.pivot_save(p)
        h2 = knn.Handle(0, pivot_weights=p)
        assert np.array_equal(h2.pivot_get_weights(), theta)
        with open(p, "r+b") as f:
            f.write(b"XXXX")
        with pytest.raises(knn.KnnError) as ei:
            h2.pivot_load(p)
        assert ei.value.status == 5


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


@pytest.mark.parametrize("weights", ["random", "huge", "zero"])
def test_selection_exact_whatever_the_weights(h, torch, weights):
    theta = rand_params(15)
    if weights == "huge":
        theta = theta * 1e30          # predictions overflow: per-row fallback
    elif weights == "zero":
        theta = np.zeros_like(theta)  # predicts the sample median
    h.pivot_set_weights(theta)
    D = synth.sqdist_matrix_normal(64, 30000, 48, seed=6)
    adv = synth.adversarial_rows(30000, seed=7)
    D = np.concatenate([D, np.stack([adv[n] for n in sorted(adv)])])
    dev = torch.from_numpy(D).cuda()
    for k in (1, 32, 700):
        v, i = h.select_k(dev, k, pivot="learned")
        ov, oi = oracle.select_k(D, k)
        assert np.array_equal(i.cpu().numpy(), oi)
        assert np.array_equal(bits(v.cpu().numpy()), bits(ov))


def _trained_handle(knn, torch):
    from paper_1309_5478_amd import pivot_train
    if os.path.exists(pivot_train.DEFAULT_WEIGHTS):
        return knn.Handle(0)           # packaged weights
    say("no packaged pivot weights: training a small network")
    cfgs = [(kind, n, d, 1000 + i) for i, (kind, n, d) in enumerate(
        [(kd, n, d) for kd in pivot_train.KINDS for n in (16384, 65536) for d in (32, 256)])]
    return pivot_train.train(out_path=None, steps=800, configs=cfgs, log=say)


def test_learned_pivot_gain_over_plain(torch, knn):
    """Held-out rows (seeds never used in training): the trained network must
    cut partition passes and time against plain median-of-samples pivots, with
    identical output.  The sample-order-statistic rule is reported beside it."""
    h = _trained_handle(knn, torch)
    D = synth.sqdist_matrix_normal(4096, 65536, 256, seed=2024)
    dev = torch.from_numpy(D).cuda()
    res = {}
    for pivot in ("plain", "sample", "learned"):
        h.select_k(dev, 64, pivot=pivot)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        v, i = h.select_k(dev, 64, pivot=pivot)
        e1.record()
        torch.cuda.synchronize()
        st = h.stats()
        res[pivot] = dict(ms=e0.elapsed_time(e1), passes=st["passes_total"] / st["rows"],
                          stream=st["stream_passes_total"] / st["rows"],
                          first=st["first_pass_survivors"] / st["rows"], out=(bits(v.cpu().numpy()), i.cpu().numpy()))
        say(f"{pivot}: {res[pivot]['ms']:.3f} ms, passes/row {res[pivot]['passes']:.2f}, "
            f"streams/row {res[pivot]['stream']:.4f}, first-pass survivors/row {res[pivot]['first']:.1f}")
    for p in ("sample", "learned"):
        assert np.array_equal(res[p]["out"][0], res["plain"]["out"][0])
        assert np.array_equal(res[p]["out"][1], res["plain"]["out"][1])
    assert res["learned"]["passes"] < 0.5 * res["plain"]["passes"]
    assert res["learned"]["ms"] < 0.5 * res["plain"]["ms"]
    assert res["learned"]["stream"] < 1.03      # re-reads of a row stay rare
