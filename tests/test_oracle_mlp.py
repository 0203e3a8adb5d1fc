"""Pins for the MLP oracle: finite differences, Adam's closed-form first
step, and the network's affine regime."""
import numpy as np
import pytest

from oracle import mlp
from paper_1801_01134_amd import synth


def _setup(B=12, seed=0, n_out=6):
    rng = synth.rng_for(500, seed)
    P = mlp.init_params(rng, n_out)
    X = rng.normal(size=(B, 16))
    t = np.exp(rng.normal(size=(B, n_out)))
    return P, X, mlp.targets(t)


def test_parameter_counts():
    # 16*64 + 64 + 64*64 + 64 + K*64 + K: 5638 for the six shapes, 5768 with
    # the two test kernels
    assert mlp.n_params() == mlp.n_params(6) == 5638
    assert mlp.n_params(8) == 5768
    assert mlp.param_shapes(8)["W3"] == (8, 64) and mlp.param_shapes(8)["b3"] == (8,)


@pytest.mark.parametrize("n_out", [6, 8])
def test_gradients_match_central_differences(n_out):
    P, X, tau = _setup(n_out=n_out)
    _, G = mlp.loss_and_grad(P, X, tau)
    rng = synth.rng_for(501)
    for name in mlp.PARAM_NAMES:
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            w = flat[idx]
            h = 1e-6 * max(1.0, abs(w))
            flat[idx] = w + h
            lp, _ = mlp.loss_and_grad(P, X, tau)
            flat[idx] = w - h
            lm, _ = mlp.loss_and_grad(P, X, tau)
            flat[idx] = w
            fd = (lp - lm) / (2 * h)
            g = G[name].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1e-3, abs(g)) + 1e-9, (name, idx, fd, g)


def test_adam_first_step_is_lr_times_sign():
    P, X, tau = _setup()
    _, G = mlp.loss_and_grad(P, X, tau)
    before = {k: v.copy() for k, v in P.items()}
    opt = mlp.Adam(P, lr=1e-3)
    opt.step(P, G)
    for k in P:
        g = G[k]
        big = np.abs(g) > 1e-4
        step = before[k] - P[k]
        assert np.allclose(step[big], 1e-3 * np.sign(g[big]), rtol=1e-4)


@pytest.mark.parametrize("n_out", [6, 8])
def test_affine_regime_equals_matrix_chain(n_out):
    rng = synth.rng_for(502)
    P = {"W1": rng.uniform(0.1, 1, (64, 16)), "b1": rng.uniform(0.1, 1, 64),
         "W2": rng.uniform(0.1, 1, (64, 64)), "b2": rng.uniform(0.1, 1, 64),
         "W3": rng.uniform(-1, 1, (n_out, 64)), "b3": rng.uniform(-1, 1, n_out)}
    X = rng.uniform(0.1, 1, (5, 16))  # every pre-activation is positive
    o, _ = mlp.forward(P, X)
    want = np.zeros((5, n_out))
    for b in range(5):
        h1 = [sum(P["W1"][i, j] * X[b, j] for j in range(16)) + P["b1"][i] for i in range(64)]
        h2 = [sum(P["W2"][i, j] * h1[j] for j in range(64)) + P["b2"][i] for i in range(64)]
        want[b] = [sum(P["W3"][i, j] * h2[j] for j in range(64)) + P["b3"][i] for i in range(n_out)]
    assert np.allclose(o, want, rtol=1e-12)


def test_targets_and_training_reduces_loss():
    t = np.array([[2.0, 1.0, 4.0, 1.0, 8.0, 3.0]])
    assert np.array_equal(mlp.targets(t), np.log2(t / 1.0))
    rng = synth.rng_for(503)
    X = rng.normal(size=(256, 16))
    times = np.exp(0.3 * (X[:, :6] + 0.5 * X[:, 6:12]))  # learnable
    tau = mlp.targets(times)
    P = mlp.init_params(rng)
    order = np.concatenate([rng.permutation(256) for _ in range(30)])
    P2, losses = mlp.train(P, X, tau, order, batch=32, lr=3e-3)
    assert np.mean(losses[-10:]) < 0.3 * np.mean(losses[:10])


def test_standardizer_hand_computed():
    # column 0: 1, 3, 8 -> mean 4, population variance (9 + 1 + 16) / 3 = 26/3
    # (the sample variance would be 13); column 1 is constant -> spread 0,
    # replaced by 1; column 2: spread 1e-13 (below 1e-12) -> 1; column 3:
    # spread 2e-12 (kept)
    X = np.array([[1.0, 5.0, 1.0 + 1e-13, 2e-12],
                  [3.0, 5.0, 1.0 - 1e-13, -2e-12],
                  [8.0, 5.0, 1.0 + 1e-13, 2e-12]])
    mu, sd = mlp.standardize_stats(X)
    assert mu[0] == 4.0 and mu[1] == 5.0
    assert sd[0] == np.sqrt(26.0 / 3.0)
    assert sd[1] == 1.0
    assert sd[2] == 1.0                                  # population spread ~0.94e-13
    assert abs(sd[3] - np.sqrt(32.0 / 9.0) * 1e-12) <= 1e-24   # population spread ~1.89e-12, kept
