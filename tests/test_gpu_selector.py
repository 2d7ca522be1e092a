"""The learned schedule selector's GPU kernels against the FP64 CPU oracle of
the same network: loss and gradient of one forward/backward pass, the Adam
update, and inference; plus the library's fall back to the fixed default."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _batch(B, seed):
    g = np.random.default_rng(seed)
    X = np.zeros((B, 4), dtype=np.float32)
    X[:, 0] = g.uniform(-1.5, 1.2, B)                 # (log2 n - 14) / 3
    X[np.arange(B), 1 + g.integers(0, 3, B)] = 1.0    # precision one-hot
    Y = np.stack([g.integers(0, 4, B), g.integers(0, 3, B), g.integers(0, 3, B)], axis=1).astype(np.int32)
    return X, Y


def _theta(seed):
    g = np.random.default_rng(seed)
    th = np.concatenate([g.uniform(-0.5, 0.5, 160), g.uniform(-0.18, 0.18, 330)])
    return th.astype(np.float32)


@pytest.fixture
def fresh(gpu):
    yield gpu
    assert gpu.lu_selector_load(None) == 0        # later tests see the fixed default again


@pytest.mark.parametrize("B,seed", [(1, 0), (37, 1), (144, 2), (256, 3)])
def test_gradient_matches_oracle(fresh, B, seed):
    gpu = fresh
    X, Y = _batch(B, seed)
    th = _theta(seed)
    assert gpu.lu_selector_set_params(th, 1024, 49152) == 0
    rc, loss, g = gpu.lu_selector_grad(X, Y)
    assert rc == 0
    th64 = th.astype(np.float64)
    want_loss = mlp.loss(th64, X, Y)
    want = mlp.grad(th64, X, Y)
    assert abs(loss - want_loss) <= 1e-5 * max(1.0, abs(want_loss))
    assert np.linalg.norm(g - want) <= 1e-4 * np.linalg.norm(want)
    assert np.abs(g - want).max() <= 1e-4 * np.abs(want).max() + 1e-7


def test_adam_steps_match_oracle(fresh):
    gpu = fresh
    X, Y = _batch(96, 5)
    th = _theta(5)
    lr = 1e-2
    assert gpu.lu_selector_set_params(th, 1024, 49152) == 0      # also resets the Adam moments
    steps = 3
    rc, losses = gpu.lu_selector_train(X, Y, steps, lr=lr)
    assert rc == 0
    rc, got = gpu.lu_selector_get_params()
    t64 = th.astype(np.float64)
    m = np.zeros_like(t64)
    v = np.zeros_like(t64)
    want_losses = []
    for t in range(1, steps + 1):
        want_losses.append(mlp.loss(t64, X, Y))
        g = mlp.grad(t64, X, Y)
        t64, m, v = mlp.adam(t64, g, m, v, t, lr=lr)
    # the reported loss is the one of the weights each step started from
    assert np.allclose(losses, want_losses, rtol=1e-5, atol=1e-6) or \
        np.allclose(losses[:-1], want_losses[1:], rtol=1e-5, atol=1e-6)
    # Adam's first steps move every weight by about lr * sign(g): FP32
    # gradients can flip the sign only where g is tiny, so compare elsewhere
    g0 = np.abs(mlp.grad(th.astype(np.float64), X, Y))
    sel = g0 > 1e-3 * g0.max()
    assert sel.mean() > 0.8
    assert np.abs(got[sel] - t64[sel]).max() <= 1e-3 * lr * steps + 1e-6


def test_training_decreases_loss_and_fits_labels(fresh):
    gpu = fresh
    # a learnable rule: b grows with n, depth from precision, CU share from n
    ns = np.array([1024 * k for k in range(1, 49)])
    X, Y = [], []
    for n in ns:
        for p in range(3):
            x = np.zeros(4, dtype=np.float32)
            x[0] = (np.log2(n) - 14.0) / 3.0
            x[1 + p] = 1.0
            X.append(x)
            Y.append([min(3, int(np.log2(n) - 10) // 2), p, 0 if n < 16384 else 2])
    X = np.array(X, dtype=np.float32)
    Y = np.array(Y, dtype=np.int32)
    th = _theta(9)
    assert gpu.lu_selector_set_params(th, 1024, 49152) == 0
    rc, losses = gpu.lu_selector_train(X, Y, 1500, lr=2e-2)
    assert rc == 0
    assert losses[-1] < 0.25 * losses[0]
    rc, th_new = gpu.lu_selector_get_params()
    acc = (mlp.predict(th_new.astype(np.float64), X) == Y).all(axis=1).mean()
    assert acc >= 0.9, acc
    # the library's own inference agrees with the oracle's on every training point
    kB, kP = [64, 128, 256, 512], [8, 16, 32]
    pred = mlp.predict(th_new.astype(np.float64), X)
    for i, n in enumerate(np.repeat(ns, 3)):
        prec = i % 3
        z = mlp.forward(th_new.astype(np.float64), X[i:i + 1])[2][0]
        margins = [np.sort(z[lo:hi])[-1] - np.sort(z[lo:hi])[-2] for lo, hi in mlp.HEADS]
        if min(margins) < 1e-4:
            continue                                   # FP32 vs FP64 tie: either answer is right
        rc, s = gpu.lu_selector_predict(int(n), prec)
        assert rc == 0
        assert s == (kB[pred[i, 0]], int(pred[i, 1]), kP[pred[i, 2]])


def test_selector_range_and_fallback(fresh):
    gpu = fresh
    assert gpu.lu_selector_set_params(_theta(1), 4096, 8192) == 0
    # outside [n_min / 2, 2 n_max] the fixed default is used
    rc, s = gpu.lu_selector_predict(100000, 0)
    assert rc == 1 and s == (256, 1, 16)
    rc, s = gpu.lu_selector_predict(1000, 0)
    assert rc == 1 and s == (256, 1, 16)
    rc, s = gpu.lu_selector_predict(6000, 0)
    assert rc == 0 and s[0] in (64, 128, 256, 512) and s[1] in (0, 1, 2) and s[2] in (8, 16, 32)


def test_library_inference_matches_oracle_on_committed_weights(fresh):
    """The weights shipped next to the library: the GPU forward kernel picks the
    schedule the FP64 oracle of the network picks, at every swept size."""
    import os
    from tests.test_selector_regret import PKG, choose, load_weights, sweep
    gpu = fresh
    theta, _, _ = load_weights()
    assert gpu.lu_selector_load(os.path.join(PKG, "selector_weights.bin")) == 0
    d, _ = sweep()
    from paper_1804_07017_amd import tune
    checked = 0
    for n in d["train_sizes"] + d["heldout_sizes"]:
        for prec in (0, 1, 2):
            z = mlp.forward(theta, np.array([tune.features(n, prec)]))[2][0]
            if min(np.sort(z[lo:hi])[-1] - np.sort(z[lo:hi])[-2] for lo, hi in mlp.HEADS) < 1e-4:
                continue
            rc, s = gpu.lu_selector_predict(n, prec)
            assert rc == 0 and s == choose(theta, n, prec), (n, prec, s)
            checked += 1
    assert checked >= 30
