"""What the trained selector network gains over selection without it, on the
committed timing records (measured on one MI355X) and the committed model
(trained on the device by the library's own kernels).

Both selectors are evaluated here by the CPU oracle, in FP64: the network's
forward pass on the held-out matrices' features, and the paper's per-kernel
polynomial interpolation of speed against Avg(r,c) ("Performance polynomial
interpolation") fitted on the training matrices. The regret of a choice is
t_selected / t_best - 1 (the time form of Table 3's speed difference), with
the recorded times of all six kernels. The split is by matrix index, 80% of
each population for training and the rest held out, as at training time.
"""
import json
import os

import numpy as np
import pytest

import oracle.mlp as M
import oracle.select as S
from paper_1801_01134_amd import records as R

HERE = os.path.dirname(os.path.abspath(__file__))
REC = os.path.join(HERE, "..", "paper_1801_01134_amd", "records")
FILES = [os.path.join(REC, f) for f in ("selector_records_mi355x.jsonl", "structured_records_mi355x.jsonl")]
MODEL = os.path.join(REC, "selector_mlp_mi355x.json")


@pytest.fixture(scope="module")
def held_out():
    if not all(os.path.exists(f) for f in FILES + [MODEL]):
        pytest.skip("no committed records or model")
    train, test = R.split(R.load(*FILES))
    with open(MODEL) as f:
        model = json.load(f)
    return train, test, model


def _params(flat):
    """The device's flat parameter vector (W1, b1, W2, b2, W3, b3, weights
    row-major [out, in]) as the oracle's dictionary."""
    flat = np.asarray(flat, dtype=np.float64)
    P, o = {}, 0
    for name in M.PARAM_NAMES:
        shp = M.param_shapes()[name]
        n = int(np.prod(shp))
        P[name] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.size == M.n_params()
    return P


def _regrets(T, choice):
    return np.array([S.regret(T[i], int(choice[i])) for i in range(T.shape[0])])


def test_network_beats_interpolation_on_held_out_matrices(held_out):
    train, test, model = held_out
    Xtr, Ttr, Atr, Gtr = R.arrays(train)
    Xte, Tte, Ate, Gte = R.arrays(test)
    assert len(test) >= 400 and Tte.shape[1] == 6

    P = _params(model["params"])
    Xh = (Xte.astype(np.float64) - np.asarray(model["mu"], np.float64)) / np.asarray(model["sd"], np.float64)
    net = _regrets(Tte, M.predict(P, Xh))

    interp = S.fit_interpolation(Atr, Gtr, 3)
    itp = _regrets(Tte, np.array([interp.select(Ate[i]) for i in range(len(test))]))

    # always the single shape that is best on average over the training matrices
    fixed_k = int(np.argmin(np.mean(Ttr / Ttr.min(axis=1, keepdims=True), axis=0)))
    fixed = _regrets(Tte, np.full(len(test), fixed_k))

    print(f"held-out mean regret: network {net.mean():.4f}, interpolation {itp.mean():.4f}, "
          f"fixed shape {fixed.mean():.4f}; within 5%: {np.mean(net <= 0.05):.3f}, "
          f"{np.mean(itp <= 0.05):.3f}, {np.mean(fixed <= 0.05):.3f}")
    # the network is within 5% of the best kernel where the interpolation is not
    assert np.mean(net <= 0.05) >= 0.95
    assert np.mean(net <= 0.05) > np.mean(itp <= 0.05)
    # and its average loss against the best kernel is a fraction of the others'
    assert net.mean() < 0.01
    assert net.mean() < 0.5 * itp.mean()
    assert net.mean() < 0.5 * fixed.mean()


def test_network_picks_are_stable_under_float32_rounding(held_out):
    """The device runs the network in FP32; its picks agree with the FP64
    forward pass except where two kernels' scores nearly tie, and such
    disagreements cost almost nothing."""
    _, test, model = held_out
    Xte, Tte, _, _ = R.arrays(test)
    P = _params(model["params"])
    mu = np.asarray(model["mu"], np.float64)
    sd = np.asarray(model["sd"], np.float64)
    o64, _ = M.forward(P, (Xte.astype(np.float64) - mu) / sd)
    P32 = {k: v.astype(np.float32) for k, v in P.items()}
    Xh32 = ((Xte.astype(np.float32) - mu.astype(np.float32)) / sd.astype(np.float32)).astype(np.float32)
    h1 = np.maximum(Xh32 @ P32["W1"].T + P32["b1"], 0)
    h2 = np.maximum(h1 @ P32["W2"].T + P32["b2"], 0)
    o32 = h2 @ P32["W3"].T + P32["b3"]
    c64, c32 = o64.argmin(axis=1), o32.argmin(axis=1)
    differ = np.flatnonzero(c64 != c32)
    assert differ.size <= 0.02 * len(test)
    for i in differ:
        gap = abs(o64[i, c64[i]] - o64[i, c32[i]])
        assert gap < 1e-3, (i, gap)
