"""The selector network's device kernels against the FP64 oracle.

Tolerances. Gradients: FP32 sums of at most 64 products per entry, so the
norm-wise relative error of each parameter block stays near 1e-6; the test
allows 1e-4. Training: Adam moves a parameter by about lr per step, and an
FP32 gradient error of relative size e changes that move by about e*lr, so
after S steps |dP| <= 1e-3*lr*S + 1e-6 leaves two orders of margin while a
wrong sign or index shows up as ~lr*S. Inference: an FP32 dot product of m
terms errs by at most ~m*u times the sum of the terms' magnitudes; the bound
uses a forward pass on |W|, |x| to get those magnitudes.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import select as osel
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu
OUTS = pytest.mark.parametrize("k", [6, 8], ids=["6shapes", "8classes"])


def blocks(k=6):
    """(name, start, end) of each parameter block in the flat layout."""
    return [("W1", 0, 1024), ("b1", 1024, 1088), ("W2", 1088, 5184), ("b2", 5184, 5248),
            ("W3", 5248, 5248 + 64 * k), ("b3", 5248 + 64 * k, 5248 + 65 * k)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def flat(P):
    k = np.asarray(P["b3"]).size
    return np.concatenate([np.asarray(P[n], np.float64).reshape(-1) for n, _, _ in blocks(k)])


def unflat(v):
    k = 8 if v.size == M.n_params(8) else 6
    shapes = M.param_shapes(k)
    return {n: np.asarray(v[a:b], np.float64).reshape(shapes[n]) for n, a, b in blocks(k)}


def dataset(n, seed, k=6):
    """Feature rows with the spread of real features and times with a
    feature-dependent best class (inputs only; no method arithmetic)."""
    rng = synth.rng_for(510, seed)
    X = (rng.standard_normal((n, 16)) * rng.uniform(0.5, 5.0, 16) + rng.uniform(-3, 3, 16)).astype(np.float32)
    t = np.exp(0.5 * rng.standard_normal((n, k)) + 0.1 * X[:, :k]).astype(np.float32)
    return X, t


def prepared(n, seed, k=6):
    """Inputs both sides share: FP32 features and times, the oracle's
    standardizer rounded to FP32, targets rounded to FP32, FP32 params."""
    X, t = dataset(n, seed, k)
    mu, sd = M.standardize_stats(X.astype(np.float64))
    mu32, sd32 = mu.astype(np.float32), sd.astype(np.float32)
    tau32 = M.targets(t.astype(np.float64)).astype(np.float32)
    P32 = flat(M.init_params(synth.rng_for(511, seed), k)).astype(np.float32)
    Xh = (X.astype(np.float64) - mu32.astype(np.float64)) / sd32.astype(np.float64)
    return X, t, mu32, sd32, tau32, P32, Xh


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@OUTS
def test_standardizer_and_targets(k):
    say(f"[mlp] standardizer, targets K={k}")
    X, t = dataset(1000, 1, k)
    mu, sd = spc.mlp_standardizer(cuda(X))
    mu_r, sd_r = M.standardize_stats(X.astype(np.float64))
    assert np.allclose(mu.cpu().numpy(), mu_r, rtol=2**-23, atol=1e-6)
    assert np.allclose(sd.cpu().numpy(), sd_r, rtol=2**-22, atol=0)
    tau = spc.mlp_targets(cuda(t)).cpu().numpy()
    tau_r = M.targets(t.astype(np.float64))
    assert np.allclose(tau, tau_r, rtol=2**-23, atol=1e-7)
    assert np.all(tau.min(axis=1) == 0.0)


@OUTS
@pytest.mark.parametrize("batch", [1, 17, 64])
def test_loss_grad_matches_oracle(batch, k):
    say(f"[mlp] loss/grad batch={batch} K={k}")
    X, t, mu, sd, tau, P, Xh = prepared(300, 2, k)
    rows = synth.rng_for(512, batch).choice(300, size=batch, replace=False).astype(np.int32)
    loss, g = spc.mlp_loss_grad(cuda(P), cuda(mu), cuda(sd), cuda(X), cuda(tau), rows)
    g = g.cpu().numpy().astype(np.float64)
    L_ref, G_ref = M.loss_and_grad(unflat(P.astype(np.float64)), Xh[rows], tau[rows].astype(np.float64))
    assert g.size == M.n_params(k)
    assert abs(loss - L_ref) <= 1e-5 * L_ref
    for name, a, b in blocks(k):
        ref = np.asarray(G_ref[name]).reshape(-1)
        err = np.linalg.norm(g[a:b] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err <= 1e-4, (name, err)


@OUTS
def test_train_matches_oracle_and_resumes(k):
    say(f"[mlp] train 40 steps K={k}")
    n, B, S, lr = 256, 64, 40, 1e-3
    X, t, mu, sd, tau, P, Xh = prepared(n, 3, k)
    order = synth.rng_for(513).permutation(np.tile(np.arange(n), (S * B) // n + 1))[:S * B].astype(np.int32)
    p = cuda(P)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    args = (cuda(mu), cuda(sd), cuda(X), cuda(tau))
    losses = spc.mlp_train(p, m, v, 0, lr, *args, order, B).cpu().numpy()
    P_ref, L_ref = M.train(unflat(P.astype(np.float64)), Xh, tau.astype(np.float64), order, B, lr=lr)
    assert np.all(np.abs(losses - np.array(L_ref)) <= 1e-4 * np.array(L_ref))
    d = np.abs(p.cpu().numpy().astype(np.float64) - flat(P_ref))
    assert d.max() <= 1e-3 * lr * S + 1e-6, d.max()
    assert losses[-1] < losses[0]
    # the same 40 steps taken as 25 + 15 give the same bits
    p2 = cuda(P)
    m2 = torch.zeros_like(p2)
    v2 = torch.zeros_like(p2)
    spc.mlp_train(p2, m2, v2, 0, lr, *args, order[:25 * B], B)
    spc.mlp_train(p2, m2, v2, 25, lr, *args, order[25 * B:], B)
    assert torch.equal(p, p2) and torch.equal(m, m2) and torch.equal(v, v2)


@OUTS
def test_infer_and_selector_match_oracle(k):
    say(f"[mlp] inference K={k}")
    X, t, mu, sd, tau, P, Xh = prepared(2000, 4, k)
    scores, choice = spc.mlp_infer(cuda(P), cuda(mu), cuda(sd), cuda(X))
    scores = scores.cpu().numpy().astype(np.float64)
    choice = choice.cpu().numpy()
    Pd = unflat(P.astype(np.float64))
    o_ref, _ = M.forward(Pd, Xh)
    mag, _ = M.forward({k: np.abs(v) for k, v in Pd.items()}, np.abs(Xh))
    tol = 2 * 64 * 2.0**-24 * (mag + 1.0)
    assert np.all(np.abs(scores - o_ref) <= tol)
    srt = np.sort(o_ref, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 2 * tol.max(axis=1)
    assert clear.mean() > 0.9
    assert np.array_equal(choice[clear], np.argmin(o_ref, axis=1)[clear])
    # the selector object gives the same choice for single vectors
    sel = spc.Selector()
    with pytest.raises(spc.SpcError) as e:
        sel.select(X[0], spc.SEL_MLP)
    assert e.value.code == -7
    sel.set_mlp(P, mu, sd)
    assert sel.n_classes(spc.SEL_MLP) == k
    for b in range(0, 2000, 199):
        s, sc = sel.select(X[b], spc.SEL_MLP)
        assert s == choice[b] and np.array_equal(sc, scores[b].astype(np.float32))


def test_argument_checks():
    X, t, mu, sd, tau, P, Xh = prepared(50, 5)
    with pytest.raises(spc.SpcError) as e:
        spc.mlp_loss_grad(cuda(P), cuda(mu), cuda(sd), cuda(X), cuda(tau), np.array([0, 50], np.int32))
    assert e.value.code == -4
    with pytest.raises(spc.SpcError) as e:
        spc.mlp_loss_grad(cuda(P), cuda(mu), cuda(sd), cuda(X), cuda(tau), np.zeros(65, np.int32))
    assert e.value.code == -8
    # oracle feature vectors go through the same path (feature scale check)
    f = osel.features(synth.band_plus_uniform()).astype(np.float32)
    s, _ = spc.Selector().set_mlp(P, mu, sd).select(f, spc.SEL_MLP)
    assert 0 <= s < 6
    # an output count other than 6 or 8 is refused
    from paper_1801_01134_amd import _binding as bb
    Xd, Pd, mud, sdd = cuda(X), cuda(P), cuda(mu), cuda(sd)
    ch = torch.empty(X.shape[0], dtype=torch.int32, device="cuda")
    with pytest.raises(spc.SpcError) as e:
        bb.check(spc.lib().spc_mlp_infer(bb._ptr(Pd), bb._ptr(mud), bb._ptr(sdd), bb._ptr(Xd), X.shape[0], 7,
                                         None, bb._ptr(ch), bb.stream_ptr()))
    assert e.value.code == -1
    with pytest.raises(ValueError):
        spc.mlp_infer(cuda(P[:-1]), cuda(mu), cuda(sd), cuda(X))
