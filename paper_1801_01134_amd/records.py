"""Timing records of the beta(r,c) kernels and the selectors built on them.

The paper chooses a kernel from timings recorded on earlier runs (its
record-based strategy): one polynomial per kernel of speed against Avg(r,c)
(section "Performance polynomial interpolation"). This module

  * collects records: for each matrix of a seeded population, the 16 device
    features (spc_matrix_features), and for each of the six shapes the
    device conversion followed by the autotuner (spc_autotune: every plan
    candidate timed with HIP events); one JSON line per matrix with the best
    time of each shape's own kernels (modes 0, 1 and 3) and, for beta(1,8) and
    beta(2,4), the best time of the test kernel of Algorithm 2 (mode 2);
  * fits the interpolation selector (spc_selector_fit_interp) and trains the
    network on the device (spc_mlp_standardizer / spc_mlp_targets /
    spc_mlp_train) from a training split of the records, over 6 classes
    (the shapes) or 8 (the shapes and the two test kernels);
  * evaluates both on the held-out split by regret = t_selected / t_best - 1
    using the recorded times, against the best of the classes the selector
    knows and against the best of all eight kernels.

Command line:
  python -m paper_1801_01134_amd.records collect --first 0 --count 2000 --out recs.jsonl
  python -m paper_1801_01134_amd.records train --records recs.jsonl --out model.json [--classes 8]
  python -m paper_1801_01134_amd.records evaluate --records recs.jsonl --model model.json
  python -m paper_1801_01134_amd.records compare-classes --records recs.jsonl

Matrix generation is CPU work (numpy); a pool of worker processes, started
before this process touches the GPU, keeps the device busy.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

SHAPES = [(1, 8), (2, 4), (2, 8), (4, 4), (4, 8), (8, 4)]
DEFAULT_MIN_ROWS = 50_000
DEFAULT_MAX_ROWS = 1_000_000
TRAIN_FRACTION = 0.8


# ---------------------------------------------------------------------------
# collection

POPULATIONS = ("selector", "structured", "large")
LARGE_MIN_ROWS, LARGE_MAX_ROWS = 1_000_000, 4_000_000


def generator(population: str):
    """The seeded matrix generator of a population: (index, min_rows,
    max_rows) -> (family, CSR)."""
    from . import synth
    return {"selector": synth.selector_matrix, "structured": synth.structured_matrix,
            "large": synth.large_matrix}[population]


def _generate(args):
    """Worker: build matrix `index` and park its CSR structure in files."""
    index, min_rows, max_rows, tmp, population = args
    t0 = time.perf_counter()
    fam, A = generator(population)(index, min_rows, max_rows)
    base = os.path.join(tmp, f"m{index}")
    np.save(base + "_rp.npy", A.rowptr)
    np.save(base + "_ci.npy", A.colidx)
    return index, fam, A.n_rows, A.n_cols, base, time.perf_counter() - t0


class _Ready:
    """A result computed in this process, read like a pool's async result."""

    def __init__(self, value):
        self.value = value

    def get(self):
        return self.value


def collect(first: int, count: int, out_path: str, reps: int = 5, workers: int = 12,
            min_rows: int = DEFAULT_MIN_ROWS, max_rows: int = DEFAULT_MAX_ROWS, population: str = "selector",
            log=sys.stderr):
    if population not in POPULATIONS:
        raise ValueError(f"population must be one of {POPULATIONS}")
    import multiprocessing as mp
    # the pool is forked before this process initialises the GPU; workers = 0
    # generates the matrices in this process instead (no fork)
    ctx = mp.get_context("fork")
    tmp = tempfile.mkdtemp(prefix="spc_records_")
    pool = ctx.Pool(workers) if workers > 0 else None
    try:
        import torch

        from . import _binding as b
        dev = torch.device("cuda")
        gen = torch.Generator(device=dev)
        pending = []
        todo = list(range(first, first + count))
        window = max(1, 2 * workers)
        t_start = time.perf_counter()
        with open(out_path, "a") as out:
            while todo or pending:
                while todo and len(pending) < window:
                    i = todo.pop(0)
                    job = (i, min_rows, max_rows, tmp, population)
                    pending.append(pool.apply_async(_generate, (job,)) if pool else _Ready(_generate(job)))
                index, fam, n_rows, n_cols, base, t_gen = pending.pop(0).get()
                rp = torch.from_numpy(np.load(base + "_rp.npy")).to(dev)
                ci = torch.from_numpy(np.load(base + "_ci.npy")).to(dev)
                os.remove(base + "_rp.npy")
                os.remove(base + "_ci.npy")
                nnz = ci.numel()
                gen.manual_seed(1801 * 100003 + index)
                vals = torch.empty(max(1, nnz), dtype=torch.float64, device=dev).uniform_(-1.0, 1.0,
                                                                                        generator=gen)[:nnz]
                x = torch.empty(n_cols, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=gen)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                feat, nb = b.matrix_features(rp, ci, n_cols)
                t_feat = time.perf_counter() - t0
                us, dflt, params, ntiles, us_test, params_test = [], [], [], [], [], []
                for (r, c) in SHAPES:
                    B = b.csr_to_beta(r, c, rp, ci, vals, n_cols)
                    _, _, recs = b.autotune(B, reps=reps, x=x)
                    # the shape's own kernels (modes 0, 1 and 3) and, for the
                    # one-byte-mask shapes, the test kernel (mode 2: Algorithm 2)
                    # as a class of its own
                    plain = min((q for q in recs if q["mode"] != 2), key=lambda q: q["us"])
                    us.append(float(plain["us"]))
                    params.append({k: v for k, v in plain.items() if k not in ("us", "n_tiles")})
                    ntiles.append(int(plain["n_tiles"]))
                    test = [q for q in recs if q["mode"] == 2]
                    if test:
                        bt = min(test, key=lambda q: q["us"])
                        us_test.append(float(bt["us"]))
                        params_test.append({k: v for k, v in bt.items() if k not in ("us", "n_tiles")})
                    d = [q["us"] for q in recs if q["mode"] == 0 and q["wave_chunks"] in (0, 4)
                         and q["tile_order"] == 0 and not q.get("cu_groups") and not q.get("wave_tiles")
                         and not q["pipeline"]]
                    dflt.append(float(d[0]) if d else float("nan"))
                    del B
                rec = {"population": population, "index": index, "family": fam, "n_rows": n_rows,
                       "n_cols": n_cols, "nnz": nnz,
                       "features": [float(v) for v in feat], "n_blocks": [int(v) for v in nb],
                       "us": us, "us_default_plan": dflt, "params": params, "n_tiles": ntiles,
                       "us_test": us_test, "params_test": params_test,
                       "gflops": [2.0 * nnz / (t * 1e-6) / 1e9 for t in us],
                       "features_ms": t_feat * 1e3, "gen_s": t_gen}
                out.write(json.dumps(rec) + "\n")
                out.flush()
                print(f"[records] {index} {fam} n={n_rows} nnz={nnz} best={int(np.argmin(us))} "
                      f"us={[round(t, 1) for t in us]} ({time.perf_counter() - t_start:.0f}s)",
                      file=log, flush=True)
                del rp, ci, vals, x
    finally:
        if pool is not None:
            pool.terminate()
            pool.join()
        for f in os.listdir(tmp):
            os.remove(os.path.join(tmp, f))
        os.rmdir(tmp)


SHARES = (32, 64, 128, 256)   # compute units a product runs on (of 256)


def collect_shares(first: int, count: int, out_path: str, population: str = "selector",
                   shares=SHARES, reps: int = 5, workers: int = 12, min_rows: int = DEFAULT_MIN_ROWS,
                   max_rows: int = DEFAULT_MAX_ROWS, log=sys.stderr):
    """Records for the 2-D model: each matrix of the population in each of
    the six shapes (library default plan) timed on streams restricted to
    `shares` compute units. One JSON line per matrix with us[share][shape]."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    tmp = tempfile.mkdtemp(prefix="spc_shares_")
    pool = ctx.Pool(workers) if workers > 0 else None
    try:
        import torch

        from . import _binding as b
        dev = torch.device("cuda")
        total = b.device_cu_count()
        streams = [b.CUStream(min(int(n), total)) for n in shares]
        gen = torch.Generator(device=dev)
        todo = list(range(first, first + count))
        pending = []
        window = max(1, 2 * workers)
        t_start = time.perf_counter()
        with open(out_path, "a") as out:
            while todo or pending:
                while todo and len(pending) < window:
                    i = todo.pop(0)
                    job = (i, min_rows, max_rows, tmp, population)
                    pending.append(pool.apply_async(_generate, (job,)) if pool else _Ready(_generate(job)))
                index, fam, n_rows, n_cols, base, _ = pending.pop(0).get()
                rp = torch.from_numpy(np.load(base + "_rp.npy")).to(dev)
                ci = torch.from_numpy(np.load(base + "_ci.npy")).to(dev)
                os.remove(base + "_rp.npy")
                os.remove(base + "_ci.npy")
                nnz = ci.numel()
                gen.manual_seed(1801 * 100003 + index)
                vals = torch.empty(max(1, nnz), dtype=torch.float64, device=dev).uniform_(-1.0, 1.0,
                                                                                        generator=gen)[:nnz]
                feat, nb = b.matrix_features(rp, ci, n_cols)
                us = [[0.0] * 6 for _ in shares]
                for k, (r, c) in enumerate(SHAPES):
                    B = b.csr_to_beta(r, c, rp, ci, vals, n_cols)
                    P = B.default_plan()
                    for q, cs in enumerate(streams):
                        with torch.cuda.stream(cs.stream):
                            us[q][k] = float(b.time_spmv(B, P, reps=reps, warmup=2))
                    del B, P
                rec = {"population": population, "index": index, "family": fam, "n_rows": n_rows,
                       "n_cols": n_cols, "nnz": nnz, "features": [float(v) for v in feat],
                       "n_blocks": [int(v) for v in nb], "cu_counts": [cs.n_cus for cs in streams],
                       "cu_total": total, "us": us}
                out.write(json.dumps(rec) + "\n")
                out.flush()
                print(f"[shares] {index} {fam} n={n_rows} nnz={nnz} best per share="
                      f"{[int(np.argmin(u)) for u in us]} ({time.perf_counter() - t_start:.0f}s)", file=log,
                      flush=True)
                del rp, ci, vals
        for cs in streams:
            cs.close()
    finally:
        if pool is not None:
            pool.terminate()
            pool.join()
        for f in os.listdir(tmp):
            os.remove(os.path.join(tmp, f))
        os.rmdir(tmp)


def share_rows(recs: list[dict]):
    """Flattened (matrix, share) rows: features [m, 16], log2 share [m],
    times [m, 6], speeds [m, 6], matrix index [m]."""
    X, U, T, G, I = [], [], [], [], []
    for j, r in enumerate(recs):
        for n, us in zip(r["cu_counts"], r["us"]):
            X.append(r["features"])
            U.append(np.log2(n / r["cu_total"]))
            T.append(us)
            G.append([2.0 * r["nnz"] / (t * 1e-6) / 1e9 for t in us])
            I.append(j)
    return (np.array(X, dtype=np.float32), np.array(U), np.array(T), np.array(G), np.array(I))


def evaluate_shares(train: list[dict], test: list[dict]):
    """Held-out regret per share of the 2-D fit (speed against Avg and the
    share), of the sequential per-kernel polynomial fitted at the full share
    only, and of the best fixed shape on the training records."""
    from . import _binding as b
    Xtr, Utr, Ttr, Gtr, _ = share_rows(train)
    Xte, Ute, Tte, Gte, _ = share_rows(test)
    sel = b.Selector()
    sel.fit_interp2d(Xtr[:, 8:14].astype(np.float64), Utr, Gtr, 3, 2)
    full = Utr == 0.0
    sel.fit_interp(Xtr[full, 8:14].astype(np.float64), Gtr[full], 3)
    out = {"n_train_matrices": len(train), "n_test_matrices": len(test), "per_share": {}}
    for u in sorted(set(Ute.tolist())):
        m = Ute == u
        share = float(2.0 ** u)
        ch2 = np.array([sel.select_at(x, share)[0] for x in Xte[m]], dtype=np.int64)
        ch1 = np.array([sel.select(x, b.SEL_INTERP)[0] for x in Xte[m]], dtype=np.int64)
        mt = Utr == u
        fixed = int(np.argmin(np.mean(Ttr[mt] / Ttr[mt].min(axis=1, keepdims=True), axis=0)))
        out["per_share"][f"{share:g}"] = {
            "n": int(m.sum()),
            "interp2d": summary(regrets(Tte[m], ch2)),
            "interp1d_full_share": summary(regrets(Tte[m], ch1)),
            f"fixed_best_on_train_{SHAPES[fixed][0]}x{SHAPES[fixed][1]}":
                summary(regrets(Tte[m], np.full(int(m.sum()), fixed, np.int64))),
            "best_shape_share": np.bincount(Tte[m].argmin(axis=1), minlength=6).tolist()}
    return out


def load(*paths: str) -> list[dict]:
    recs = []
    for path in paths:
        with open(path) as f:
            recs += [json.loads(line) for line in f if line.strip()]
    for r in recs:
        r.setdefault("population", "selector")
    recs.sort(key=lambda r: (POPULATIONS.index(r["population"]), r["index"]))
    return recs


def split(recs: list[dict], train_fraction: float = TRAIN_FRACTION):
    """Deterministic split of each population by matrix index: the lowest
    indices train, the rest are held out."""
    train, test = [], []
    for pop in POPULATIONS:
        part = [r for r in recs if r["population"] == pop]
        n_train = int(round(train_fraction * len(part)))
        train += part[:n_train]
        test += part[n_train:]
    return train, test


# Avg(r,c) feature of each kernel class: the six shapes, then the test
# kernels of beta(1,8) and beta(2,4)
CLASS_FEATURE = (8, 9, 10, 11, 12, 13, 8, 9)
CLASS_NAMES = [f"{r}x{c}" for r, c in SHAPES] + ["1x8_test", "2x4_test"]


def has_test(recs: list[dict]) -> bool:
    return all(len(r.get("us_test", [])) == 2 for r in recs)


def arrays(recs: list[dict], n_classes: int = 6):
    """Features [n, 16], times [n, K], Avg per class [n, K], speeds [n, K]
    (GFlop/s) for K = 6 (the shapes) or 8 (with the test kernels)."""
    if n_classes not in (6, 8):
        raise ValueError("n_classes must be 6 or 8")
    if n_classes == 8 and not has_test(recs):
        raise ValueError("8 classes need records with the test kernels' times (us_test)")
    X = np.array([r["features"] for r in recs], dtype=np.float32)
    T = np.array([r["us"] + (r["us_test"] if n_classes == 8 else []) for r in recs], dtype=np.float64)
    avg = X[:, list(CLASS_FEATURE[:n_classes])].astype(np.float64)
    nnz = np.array([r["nnz"] for r in recs], dtype=np.float64)
    G = 2.0 * nnz[:, None] / (T * 1e-6) / 1e9
    return X, T, avg, G


# ---------------------------------------------------------------------------
# selectors

def train_mlp(X: np.ndarray, T: np.ndarray, epochs: int = 400, batch: int = 64, lr: float = 2e-3,
              seed: int = 0):
    """Trains the network (T.shape[1] outputs) on the device. Returns
    (params, mu, sd, losses) as numpy arrays. Learning rate: lr for the
    first half of the epochs, then lr/4 and lr/16 (Adam's step count
    continues across the stages)."""
    import torch

    from . import _binding as b
    from . import synth
    dev = torch.device("cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(dev)
    mu, sd = b.mlp_standardizer(Xd)
    tau = b.mlp_targets(Td)
    rng = synth.rng_for(60, seed)
    K = T.shape[1]
    P = np.zeros(b.mlp_n_params(K), dtype=np.float32)
    # He-uniform weights, zero biases (same recipe as the oracle's init)
    o = 0
    for (n_out, n_in) in ((64, 16), (64, 64), (K, 64)):
        lim = np.sqrt(6.0 / n_in)
        P[o:o + n_out * n_in] = rng.uniform(-lim, lim, size=n_out * n_in)
        o += n_out * n_in + n_out
    p = torch.from_numpy(P).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    n = X.shape[0]
    steps_per_epoch = n // batch
    stages = [(epochs // 2, lr), (epochs // 4, lr / 4), (epochs - epochs // 2 - epochs // 4, lr / 16)]
    step0 = 0
    losses = []
    for ep, lr_s in stages:
        order = np.concatenate([rng.permutation(n)[:steps_per_epoch * batch] for _ in range(ep)]).astype(np.int32)
        L = b.mlp_train(p, m, v, step0, lr_s, mu, sd, Xd, tau, order, batch)
        losses.append(L.cpu().numpy())
        step0 += ep * steps_per_epoch
    return (p.cpu().numpy(), mu.cpu().numpy(), sd.cpu().numpy(),
            np.concatenate(losses) if losses else np.zeros(0))


def regrets(T: np.ndarray, choice: np.ndarray) -> np.ndarray:
    return T[np.arange(T.shape[0]), choice] / T.min(axis=1) - 1.0


def summary(reg: np.ndarray) -> dict:
    return {"mean": float(reg.mean()), "geomean_ratio_minus_1": float(np.exp(np.mean(np.log1p(reg))) - 1.0),
            "p90": float(np.quantile(reg, 0.9)), "max": float(reg.max()),
            "within_5pct": float(np.mean(reg <= 0.05)), "exact": float(np.mean(reg == 0.0))}


def _choices(sel, model, Xte, n_classes):
    """(network choices or None, interpolation choices) for the test rows."""
    import torch

    from . import _binding as b
    ch_mlp = None
    if model is not None:
        dev = torch.device("cuda")
        P = torch.tensor(model["params"], dtype=torch.float32, device=dev)
        mu = torch.tensor(model["mu"], dtype=torch.float32, device=dev)
        sd = torch.tensor(model["sd"], dtype=torch.float32, device=dev)
        _, ch = b.mlp_infer(P, mu, sd, torch.from_numpy(Xte).to(dev))
        ch_mlp = ch.cpu().numpy().astype(np.int64)
    ch_int = np.array([sel.select(x, b.SEL_INTERP)[0] for x in Xte], dtype=np.int64)
    return ch_mlp, ch_int


def fit(train: list[dict], n_classes: int = 6, epochs: int = 400, with_mlp: bool = True):
    """(interpolation selector, network model dict or None) fitted on train."""
    from . import _binding as b
    Xtr, Ttr, Atr, Gtr = arrays(train, n_classes)
    sel = b.Selector().fit_interp(Atr, Gtr, 3)
    model = None
    if with_mlp:
        t0 = time.perf_counter()
        P, mu, sd, losses = train_mlp(Xtr, Ttr, epochs=epochs)
        model = {"params": P.tolist(), "mu": mu.tolist(), "sd": sd.tolist(), "n_out": n_classes,
                 "final_loss": float(losses[-1]) if losses.size else None,
                 "train_s": time.perf_counter() - t0, "epochs": epochs, "n_train": len(train)}
    return sel, model


def evaluate(train: list[dict], test: list[dict], model: dict | None = None, epochs: int = 400,
             n_classes: int | None = None):
    """Fits both selectors on `train` (or uses `model` for the network) and
    reports held-out regrets for the network, the interpolation, and fixed
    kernels. With records that hold the test kernels' times, regrets are
    also given against the best of all eight kernels ("vs_all8")."""
    if n_classes is None:
        n_classes = int(model.get("n_out", 6)) if model else 6
    from . import _binding as b
    Xtr, Ttr, Atr, Gtr = arrays(train, n_classes)
    Xte, Tte, Ate, Gte = arrays(test, n_classes)
    sel = b.Selector().fit_interp(Atr, Gtr, 3)
    if model is None:
        _, model = fit(train, n_classes, epochs)
    ch_mlp, ch_int = _choices(sel, model, Xte, n_classes)
    T8 = arrays(test, 8)[1] if has_test(test) else None
    best_avg = int(np.argmin(np.mean(Ttr / Ttr.min(axis=1, keepdims=True), axis=0)))
    pops = np.array([r["population"] for r in test])

    def block(m):
        n = int(m.sum())
        d = {"n": n, "mlp": summary(regrets(Tte[m], ch_mlp[m])),
             "interpolation": summary(regrets(Tte[m], ch_int[m])),
             "fixed_b1x8": summary(regrets(Tte[m], np.zeros(n, np.int64))),
             f"fixed_best_on_train_{CLASS_NAMES[best_avg]}":
                 summary(regrets(Tte[m], np.full(n, best_avg, np.int64)))}
        if T8 is not None:
            d["vs_all8"] = {"mlp": summary(regrets(T8[m], ch_mlp[m])),
                            "interpolation": summary(regrets(T8[m], ch_int[m]))}
        return d

    out = {"n_classes": n_classes, "n_train": len(train), "n_test": len(test)}
    out.update(block(np.ones(len(test), bool)))
    out["best_class_share"] = np.bincount(Tte.argmin(axis=1), minlength=n_classes).tolist()
    out["mlp_choice_share"] = np.bincount(ch_mlp, minlength=n_classes).tolist()
    out["interp_choice_share"] = np.bincount(ch_int, minlength=n_classes).tolist()
    out["by_population"] = {pop: block(pops == pop) for pop in POPULATIONS if (pops == pop).any()}
    return out, model


def compare_classes(train: list[dict], test: list[dict], epochs: int = 400):
    """Held-out regret with and without the two test kernels as classes of
    their own, all against the best of the eight kernels: the 6-class and
    8-class network and interpolation, trained on the same split. Also the
    large population with a network that never saw it (trained on the
    other populations only)."""
    out = {}
    for k in (6, 8):
        res, _ = evaluate(train, test, None, epochs, k)
        out[f"classes_{k}"] = res
    tr_small = [r for r in train if r["population"] != "large"]
    large = [r for r in train + test if r["population"] == "large"]
    if large and tr_small:
        out["large_unseen"] = {}
        for k in (6, 8):
            res, _ = evaluate(tr_small, large, None, epochs, k)
            out["large_unseen"][f"classes_{k}"] = {key: res[key] for key in
                                                  ("n_classes", "n_train", "n_test", "mlp", "interpolation",
                                                   "vs_all8", "mlp_choice_share", "best_class_share")
                                                  if key in res}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--first", type=int, default=0)
    c.add_argument("--count", type=int, default=2000)
    c.add_argument("--out", required=True)
    c.add_argument("--reps", type=int, default=5)
    c.add_argument("--workers", type=int, default=12)
    c.add_argument("--min-rows", type=int, default=None,
                   help="default: 50k (1M for the large population)")
    c.add_argument("--max-rows", type=int, default=None,
                   help="default: 1M (4M for the large population)")
    c.add_argument("--population", default="selector", choices=POPULATIONS)
    t = sub.add_parser("train")
    t.add_argument("--records", required=True, nargs="+")
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--classes", type=int, default=6, choices=(6, 8))
    cc = sub.add_parser("compare-classes")
    cc.add_argument("--records", required=True, nargs="+")
    cc.add_argument("--epochs", type=int, default=400)
    cc.add_argument("--out", default=None)
    cs = sub.add_parser("collect-shares")
    cs.add_argument("--first", type=int, default=0)
    cs.add_argument("--count", type=int, default=320)
    cs.add_argument("--out", required=True)
    cs.add_argument("--reps", type=int, default=5)
    cs.add_argument("--workers", type=int, default=12)
    cs.add_argument("--population", default="selector", choices=POPULATIONS)
    es = sub.add_parser("evaluate-shares")
    es.add_argument("--records", required=True, nargs="+")
    e = sub.add_parser("evaluate")
    e.add_argument("--records", required=True, nargs="+")
    e.add_argument("--model", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        large = a.population == "large"
        lo = a.min_rows if a.min_rows is not None else (LARGE_MIN_ROWS if large else DEFAULT_MIN_ROWS)
        hi = a.max_rows if a.max_rows is not None else (LARGE_MAX_ROWS if large else DEFAULT_MAX_ROWS)
        collect(a.first, a.count, a.out, a.reps, a.workers, lo, hi, a.population)
    elif a.cmd == "collect-shares":
        collect_shares(a.first, a.count, a.out, a.population, reps=a.reps, workers=a.workers)
    elif a.cmd == "evaluate-shares":
        tr, te = split(load(*a.records))
        print(json.dumps(evaluate_shares(tr, te)))
    elif a.cmd == "compare-classes":
        tr, te = split(load(*a.records))
        res = compare_classes(tr, te, a.epochs)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        print(json.dumps(res))
    elif a.cmd == "train":
        tr, te = split(load(*a.records))
        res, model = evaluate(tr, te, epochs=a.epochs, n_classes=a.classes)
        with open(a.out, "w") as f:
            json.dump(model, f)
        print(json.dumps(res))
    else:
        tr, te = split(load(*a.records))
        model = None
        if a.model:
            with open(a.model) as f:
                model = json.load(f)
        res, _ = evaluate(tr, te, model)
        print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
