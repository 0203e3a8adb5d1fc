"""FP64 oracle of the learned kernel selector: a 16 -> 64 -> 64 -> K ReLU
network trained by Adam on recorded kernel times, K = 6 (the block shapes)
or 8 (the shapes and the two "test" kernels of Algorithm 2). TEST
INFRASTRUCTURE ONLY.

The paper selects kernels by per-kernel polynomial interpolation of recorded
speeds and names selection from several matrix statistics as future work
(Conclusions); this network is that extension. Its reference is written out
here step by step:

  x^   = (x - mu) / sigma            (training-set mean and spread per feature)
  z1   = W1 x^ + b1,  h1 = relu(z1)
  z2   = W2 h1 + b2,  h2 = relu(z2)
  o    = W3 h2 + b3                  (one score per kernel class)
  tau  = log2(t / min_k t_k)         (target: time relative to the best kernel)
  L    = mean over batch and classes of (o - tau)^2
  pick = argmin_k o_k

Weights are row-major [out, in]. Gradients come from the chain rule; Adam
uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8 with bias correction.
"""
from __future__ import annotations

import numpy as np

DIMS = (16, 64, 64, 6)
PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def param_shapes(n_out: int = DIMS[3]):
    d0, d1, d2 = DIMS[:3]
    return {"W1": (d1, d0), "b1": (d1,), "W2": (d2, d1), "b2": (d2,), "W3": (n_out, d2), "b3": (n_out,)}


def n_params(n_out: int = DIMS[3]) -> int:
    return int(sum(int(np.prod(s)) for s in param_shapes(n_out).values()))


def init_params(rng: np.random.Generator, n_out: int = DIMS[3]) -> dict:
    """He-uniform weights, zero biases (the random draw is an input to both sides)."""
    P = {}
    for name, shp in param_shapes(n_out).items():
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            P[name] = rng.uniform(-lim, lim, size=shp)
        else:
            P[name] = np.zeros(shp)
    return P


def standardize_stats(X):
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 1e-12, sd, 1.0)
    return mu, sd


def targets(times) -> np.ndarray:
    t = np.asarray(times, dtype=np.float64)
    return np.log2(t / t.min(axis=1, keepdims=True))


def forward(P, Xh):
    Xh = np.asarray(Xh, dtype=np.float64)
    z1 = Xh @ np.asarray(P["W1"], np.float64).T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ np.asarray(P["W2"], np.float64).T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ np.asarray(P["W3"], np.float64).T + P["b3"]
    return o, {"x": Xh, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(o, tau) -> float:
    return float(np.mean((np.asarray(o) - np.asarray(tau)) ** 2))


def backward(P, cache, o, tau) -> dict:
    B = o.shape[0]
    dO = 2.0 * (o - tau) / (B * o.shape[1])
    G = {"W3": dO.T @ cache["h2"], "b3": dO.sum(axis=0)}
    dh2 = dO @ np.asarray(P["W3"], np.float64)
    dz2 = dh2 * (cache["z2"] > 0.0)
    G["W2"] = dz2.T @ cache["h1"]
    G["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ np.asarray(P["W2"], np.float64)
    dz1 = dh1 * (cache["z1"] > 0.0)
    G["W1"] = dz1.T @ cache["x"]
    G["b1"] = dz1.sum(axis=0)
    return G


def loss_and_grad(P, Xh, tau):
    o, cache = forward(P, Xh)
    return loss(o, tau), backward(P, cache, o, tau)


class Adam:
    def __init__(self, P, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in P.items()}
        self.v = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in P.items()}
        self.t = 0

    def step(self, P, G):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in P:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * G[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * G[k] * G[k]
            mh = self.m[k] / c1
            vh = self.v[k] / c2
            P[k] = np.asarray(P[k], np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps)
        return P


def train(P, Xh, tau, order, batch: int, lr: float = 1e-3):
    """Mini-batch Adam over rows of Xh taken in the given index order (an
    input, so that both implementations visit the same batches). Returns the
    trained parameters and the loss of every step."""
    P = {k: np.array(v, dtype=np.float64) for k, v in P.items()}
    opt = Adam(P, lr=lr)
    losses = []
    order = np.asarray(order)
    for s in range(0, order.size, batch):
        idx = order[s:s + batch]
        if idx.size < batch:
            break
        L, G = loss_and_grad(P, Xh[idx], tau[idx])
        losses.append(L)
        opt.step(P, G)
    return P, losses


def predict(P, Xh) -> np.ndarray:
    o, _ = forward(P, Xh)
    return np.argmin(o, axis=1)
