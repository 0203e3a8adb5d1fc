#!/usr/bin/env python3
"""Benchmark: SpMV over beta(r,c) on the 27-point stencil of a 128^3 grid.

Headline workload (synthetic, seeded): 2,097,152 rows, 55,742,968 nonzeros,
natural ordering, diagonal 27, off-diagonals and x drawn from U[-1, 1]. Every
block shape (1,8) (2,4) (2,8) (4,4) (4,8) (8,4) is converted on the device
and timed in FP64 and FP32, each autotuned over its plan candidates; the
headline is the FP64 product with the fastest of the six (the kernel the
timing records select for this matrix). A step is one y = A x with that
kernel, inputs resident in HBM.

Flop count per product: 2 * nnz (the paper's GFlop/s definition). The
roofline figure divides the algorithmic bytes of one launch (values, block
columns, masks, interval pointers, tile descriptors, x and y, each once) by
the average kernel duration measured with HIP events on the launch stream,
against the MI355X HBM peak of 8 TB/s.

Further sections of the same JSON line (each can be switched off):
  selection   the learned selector (network) and the interpolation pick a
              shape for the headline matrix from its features alone; their
              kernel's time over the best kernel's time; held-out regrets
              of both on the recorded selector population
  batched     64 matrices (rows log-uniform in [10k, 500k], Poisson(16.8)
              uniform columns + Poisson(2.4) dense 3x3 blocks per block row),
              each in the shape the selector picks, as one launch versus 64
              launches (plain and graph-captured); and the same for 512
              small matrices (rows log-uniform in [500, 20k])
  reorder     the 27-point stencil with randomly numbered grid points, each
              shape autotuned before and after the reverse Cuthill-McKee
              renumbering (values per block, times, cost of the order and
              of the permutations)
  parallel_estimation
              the headline product on 1/8, 1/4, 1/2 and all of the compute
              units, and the held-out regrets of the 2-D (Avg, share) model
  cg          CG on the SPD 27-point matrix of a 192^3 grid (7,077,888 rows,
              189,119,224 nonzeros) with k = 1, 4, 8, 16 right-hand sides,
              FP64 to 1e-8 and FP32 to 1e-5, true residuals recomputed by
              the FP64 CSR oracle on the host

Prints one JSON line. --gpus N with N > 1 is refused: this build runs one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # dense FP32 vector peak of the part
MODEL_DIR = os.path.join(ROOT, "paper_1801_01134_amd", "records")
RECORDS = [os.path.join(MODEL_DIR, f) for f in ("selector_records_mi355x.jsonl", "structured_records_mi355x.jsonl",
                                                "large_records_mi355x.jsonl")]
MODEL = os.path.join(MODEL_DIR, "selector_mlp_mi355x.json")
MODEL8 = os.path.join(MODEL_DIR, "selector_mlp8_mi355x.json")


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(B, n_tiles: int, k: int = 1, accumulate: bool = False) -> int:
    es = B.values.element_size()
    n_int = B.block_rowptr.numel()
    b = (B.nnz * es + B.n_blocks * 4 + B.n_blocks * B.r * B.c // 8 + n_int * 4 + n_tiles * 32
         + k * B.n_cols * es + k * B.n_rows * es)
    if accumulate:
        b += k * B.n_rows * es
    return b


PLAN_KEYS = ("mode", "wave_chunks", "tile_bits", "tile_order", "pipeline", "cu_groups", "wave_tiles")


def committed_profile(kind: str, kname: str, shape, params: dict, m: int):
    """The committed profile summary (profiles/*.<kind>.json: 'traffic' for
    the memory counters, 'trace' for the kernel trace) of this kernel and
    plan on the m^3 stencil, if the kernel sources still hash to the ones
    that were measured; else None."""
    import glob
    import hashlib
    if m != 128:
        return None
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", f"*.{kind}.json"))):
        with open(f) as fh:
            rec = json.load(fh)
        if rec.get("kernel") != kname or rec.get("shape") != list(shape):
            continue
        if {k: rec["plan"].get(k, 0) for k in PLAN_KEYS} != {k: params.get(k, 0) for k in PLAN_KEYS}:
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() == rec["sha256"]:
            rec["source"] = os.path.relpath(f, ROOT)
            return rec
    return None


def event_time(torch, fn, steps: int, warmup: int, stream=None) -> float:
    """Average seconds per call of fn, HIP events on the stream it launches on."""
    s = stream or torch.cuda.current_stream()
    with torch.cuda.stream(s):
        for _ in range(warmup):
            fn()
        s.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        s.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def small_case(spc, torch, steps: int = 2000):
    """The small square matrix (n = 4096, 8 band + 8 uniform columns per row,
    FP64, beta(1,8)): 0.8 MB, cache-resident, so a product is bound by launch
    and latency, not by HBM. Reported in microseconds beside the FP64 CSR
    oracle on the same matrix."""
    import oracle
    from paper_1801_01134_amd import synth
    A = synth.band_plus_uniform(4096, seed=0)
    x = synth.dense_vector(A.n_cols, 1)
    dev = torch.device("cuda")
    B = spc.csr_to_beta(1, 8, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    params, us_tuned, _ = spc.autotune(B, reps=200, x=xd)
    P = spc.plan_from(B, params)
    t = event_time(torch, lambda: spc.spmv(B, xd, yd, plan=P), steps, 50)
    y_ref, s_ref = oracle.csr_spmv(A, x)
    ok = bool((abs(yd.cpu().numpy() - y_ref) <= 1e-13 * s_ref).all())
    oracle.csr_spmv(A, x)
    reps = 2000
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.csr_spmv(A, x)
    tc = (time.perf_counter() - t0) / reps
    return {"n": A.n_rows, "nnz": A.nnz, "n_blocks": B.n_blocks, "plan": params,
            "us_per_product_launched": round(t * 1e6, 2), "us_device_tuned": round(us_tuned, 2),
            "gflops": round(2.0 * A.nnz / t / 1e9, 2), "matches_oracle": ok,
            "oracle_us": round(tc * 1e6, 1), "oracle_threads": oracle.threads(),
            "note": "back-to-back launches from Python; us_device_tuned is the autotuner's device time"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(A, x, label: str, budget_s: float = 10.0):
    """The FP64 CSR oracle (plain C, OpenMP over rows) on the host cores.

    value: consecutive full products for budget_s seconds on all host
    threads. Beside it, the paper's protocol (16 consecutive products, the
    first one on a matrix not read since it was built; mean and median) on
    all threads and on one thread."""
    import numpy as np

    import oracle
    n_all = oracle.threads()

    def sixteen(threads):
        oracle.set_threads(threads)
        # fresh copies of the arrays: the first product reads them cold
        from paper_1801_01134_amd import synth
        Ac = synth.CSR(A.n_rows, A.n_cols, A.rowptr.copy(), A.colidx.copy(), A.values.copy())
        ts = []
        for _ in range(16):
            t0 = time.perf_counter()
            oracle.csr_spmv(Ac, x)
            ts.append(time.perf_counter() - t0)
        ts = np.array(ts)
        return {"threads": threads, "mean_ms": round(float(ts.mean()) * 1e3, 3),
                "median_ms": round(float(np.median(ts)) * 1e3, 3), "first_ms": round(float(ts[0]) * 1e3, 3),
                "gflops_mean": round(2.0 * A.nnz / ts.mean() / 1e9, 3),
                "gflops_median": round(2.0 * A.nnz / float(np.median(ts)) / 1e9, 3)}

    protocol = {"all_threads": sixteen(n_all), "one_thread": sixteen(1)}
    oracle.set_threads(n_all)
    t0 = time.perf_counter()
    runs = 0
    while True:
        oracle.csr_spmv(A, x)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    per = el / runs
    return {"value": round(2.0 * A.nnz / per / 1e9, 3), "unit": "GFlop/s", "cores": n_all,
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "kind": "oracle",
            "sample": f"{runs} consecutive FP64 CSR products of the full {label} on {n_all} "
                      f"threads (mean {per * 1e3:.1f} ms each, {el:.1f} s total)",
            "paper_protocol_16_runs": protocol}


# ---------------------------------------------------------------------------
# workload generation in worker processes (forked before the GPU is touched)

def _gen_batched(args):
    i, tmp, lo, hi = args
    import numpy as np

    from paper_1801_01134_amd import synth
    A = synth.batched_matrix(i, lo, hi)
    base = os.path.join(tmp, f"b{lo}_{i}")
    np.save(base + "_rp.npy", A.rowptr)
    np.save(base + "_ci.npy", A.colidx)
    np.save(base + "_v.npy", A.values)
    return i, A.n_rows, A.n_cols, base


def _gen_cg(args):
    m, tmp = args
    import numpy as np

    from paper_1801_01134_amd import synth
    A = synth.stencil27(m, diag=26.1, offdiag=-1.0)
    base = os.path.join(tmp, f"cg{m}")
    np.save(base + "_rp.npy", A.rowptr)
    np.save(base + "_ci.npy", A.colidx)
    np.save(base + "_v.npy", A.values)
    return m, A.n_rows, A.n_cols, base


def _gen_scrambled(args):
    m, tmp = args
    import numpy as np

    from paper_1801_01134_amd import synth
    A = synth.grid_scrambled(m, m, m, "27pt", seed=9)
    base = os.path.join(tmp, f"scr{m}")
    np.save(base + "_rp.npy", A.rowptr)
    np.save(base + "_ci.npy", A.colidx)
    np.save(base + "_v.npy", A.values)
    return m, A.n_rows, A.n_cols, base


def _load_csr(base, n_rows, n_cols):
    import numpy as np

    from paper_1801_01134_amd import synth
    A = synth.CSR(n_rows, n_cols, np.load(base + "_rp.npy"), np.load(base + "_ci.npy"), np.load(base + "_v.npy"))
    for suf in ("_rp.npy", "_ci.npy", "_v.npy"):
        os.remove(base + suf)
    return A


# ---------------------------------------------------------------------------
# sections

def load_selectors(spc):
    """{"classes_6": (Selector, model), "classes_8": ...} fitted on the
    training split of the committed records (interpolation) with the
    committed network of that class count, and the held-out evaluation of
    each. The 8-class entry needs records with the test kernels' times."""
    from paper_1801_01134_amd import records as R
    paths = [p for p in RECORDS if os.path.exists(p)]
    if not paths:
        return {}, {}
    recs = R.load(*paths)
    train, test = R.split(recs)
    sels, held = {}, {}
    for k, path in ((6, MODEL), (8, MODEL8)):
        if k == 8 and not R.has_test(recs):
            continue
        _, _, Atr, Gtr = R.arrays(train, k)
        sel = spc.Selector().fit_interp(Atr, Gtr, 3)
        model = None
        if os.path.exists(path):
            with open(path) as f:
                model = json.load(f)
            if int(model.get("n_out", 6)) != k:
                model = None
            else:
                sel.set_mlp(model["params"], model["mu"], model["sd"])
        sels[f"classes_{k}"] = (sel, model)
        held[f"classes_{k}"] = R.evaluate(train, test, model, n_classes=k)[0] if model else None
    return sels, held


def main_selector(sels):
    """The selector the bench reports: 8 classes when available."""
    for name in ("classes_8", "classes_6"):
        if name in sels:
            return sels[name]
    return None, None


def select_class(spc, sel, model, feat):
    """(network's class or None, interpolation's class)."""
    if sel is None:
        return None, None
    si = sel.select(feat, spc.SEL_INTERP)[0]
    sm = sel.select(feat, spc.SEL_MLP)[0] if model else None
    return sm, si


def steps_section(spc, torch, A, rp, ci, v64, sel, model, reps: int = 5):
    """The other steps of the path, each timed on the device against its own
    bound: conversion (HBM: CSR read once, beta arrays written once),
    feature extraction (HBM: CSR structure read once), network training and
    inference (FP32 vector peak) and one selection."""
    import numpy as np
    out = {}
    n, nnz = A.n_rows, A.nnz

    def wall(fn):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts[1:]))

    conv = {}
    for (r, c) in spc.SHAPES:
        B = spc.csr_to_beta(r, c, rp, ci, v64, A.n_cols)
        nb = B.n_blocks
        del B
        t = wall(lambda: spc.csr_to_beta(r, c, rp, ci, v64, A.n_cols))
        ab = (4 * (n + 1) + 4 * nnz + 8 * nnz                     # CSR read
              + 4 * ((n + r - 1) // r + 1) + 4 * nb + nb * r * c // 8 + 8 * nnz)   # beta written
        conv[f"b{r}x{c}"] = {"us": round(t * 1e6, 1), "alg_bytes": ab, "alg_GBs": round(ab / t / 1e9, 1),
                             "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4)}
    out["conversion_f64"] = {"note": "count pass, scan, host read of the block count, fill pass; the CSR "
                                     "structure is read twice (count and fill)", "shapes": conv}
    t = wall(lambda: spc.matrix_features(rp, ci, A.n_cols))
    ab = 4 * (n + 1) + 4 * nnz
    out["features"] = {"us": round(t * 1e6, 1), "alg_bytes": ab, "alg_GBs": round(ab / t / 1e9, 1),
                       "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4),
                       "note": "all six block counts and the row statistics in one pass; includes the copy "
                               "of 16 floats and 6 counts to the host"}
    if model is not None and os.path.exists(RECORDS[0]):
        from paper_1801_01134_amd import records as R
        recs = R.load(*[p for p in RECORDS if os.path.exists(p)])
        train, test = R.split(recs)
        K = int(model.get("n_out", 6))
        Xtr, Ttr, _, _ = R.arrays(train, K)
        Xte, _, _, _ = R.arrays(test, K)
        dev = torch.device("cuda")
        Xd = torch.from_numpy(np.ascontiguousarray(Xtr, dtype=np.float32)).to(dev)
        Td = torch.from_numpy(np.ascontiguousarray(Ttr, dtype=np.float32)).to(dev)
        mu, sd = spc.mlp_standardizer(Xd)
        tau = spc.mlp_targets(Td)
        p = torch.tensor(model["params"], dtype=torch.float32, device=dev)
        m_ = torch.zeros_like(p)
        v_ = torch.zeros_like(p)
        batch = 64
        steps = Xtr.shape[0] // batch
        order = np.random.default_rng(0).permutation(Xtr.shape[0])[:steps * batch].astype(np.int32)
        spc.mlp_train(p, m_, v_, 0, 1e-4, mu, sd, Xd, tau, order, batch)
        t = wall(lambda: spc.mlp_train(p, m_, v_, 0, 1e-4, mu, sd, Xd, tau, order, batch))
        layer = 16 * 64 + 64 * 64 + 64 * K
        fl = 3 * 2 * layer * batch           # forward, and a backward of twice its cost
        out["mlp_train"] = {"steps": steps, "batch": batch, "us_per_step": round(t / steps * 1e6, 2),
                            "flops_per_step": fl, "achieved_TFLOPs": round(fl * steps / t / 1e12, 5),
                            "peak_TFLOPs_fp32": FP32_PEAK_TFLOPS,
                            "frac": round(fl * steps / t / 1e12 / FP32_PEAK_TFLOPS, 7),
                            "bound": "latency: one workgroup per step (the steps depend on each other)"}
        Xq = torch.from_numpy(np.ascontiguousarray(Xte, dtype=np.float32)).to(dev)
        t = wall(lambda: spc.mlp_infer(p, mu, sd, Xq))
        out["mlp_infer"] = {"rows": int(Xte.shape[0]), "us": round(t * 1e6, 1),
                            "flops": 2 * layer * int(Xte.shape[0])}
        feat, _ = spc.matrix_features(rp, ci, A.n_cols)
        t = wall(lambda: sel.select(feat, spc.SEL_MLP))
        out["select_one_matrix_us"] = {"mlp": round(t * 1e6, 1),
                                       "interpolation": round(wall(lambda: sel.select(feat, spc.SEL_INTERP)) * 1e6, 1)}
    return out


def batch_plan(spc, B, modes, cache: dict, key) -> dict:
    """The matrix's fastest plan in one of the given modes among the
    autotuner's records that a batch can run (one tile per wavefront, no
    pipeline)."""
    if key not in cache:
        _, _, recs = spc.autotune(B, reps=3)
        cache[key] = recs
    ok = [q for q in cache[key] if q["mode"] in modes and not q.get("pipeline") and q.get("wave_tiles", 0) <= 1]
    best = min(ok, key=lambda q: q["us"])
    return {"mode": best["mode"], "wave_chunks": best["wave_chunks"]}


def batched_section(spc, torch, selectors, pool, tmp, n_mat: int, steps: int, warmup: int,
                    min_rows: int = 10_000, max_rows: int = 500_000):
    """A batch of n_mat matrices, each in the kernel class a selector picks
    from its features (the network when trained, else the interpolation),
    with the mode and chunk count the autotuner finds fastest for that class
    (a shape's class: modes 0, 3 and 4; a test class: mode 2). For each
    selector (6 classes: the shapes; 8: the shapes and the test kernels),
    the grouped batch (one launch per (mode, shape, chunks) group) against
    one launch per matrix with the same plans, both also as captured graphs."""
    import numpy as np
    dev = torch.device("cuda")
    results = pool.map(_gen_batched, [(i, tmp, min_rows, max_rows) for i in range(n_mat)])
    from paper_1801_01134_amd import synth
    mats, feats, xs = [], [], []
    total_nnz = 0
    for i, n_rows, n_cols, base in results:
        A = _load_csr(base, n_rows, n_cols)
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.colidx).to(dev)
        feat, _ = spc.matrix_features(rp, ci, A.n_cols)
        mats.append((rp, ci, torch.from_numpy(A.values).to(dev), A.n_cols, A.n_rows))
        feats.append(feat)
        xs.append(torch.from_numpy(synth.dense_vector(A.n_cols, 400 + i)).to(dev))
        total_nnz += A.nnz
    flops = 2.0 * total_nnz
    out = {"matrices": n_mat, "rows_range": [min_rows, max_rows], "nnz_total": total_nnz,
           "rows_total": sum(m[4] for m in mats)}
    betas, tune_cache = {}, {}

    def beta(i, shape):
        if (i, shape) not in betas:
            rp, ci, v, n_cols, _ = mats[i]
            r, c = spc.SHAPES[shape]
            betas[(i, shape)] = spc.csr_to_beta(r, c, rp, ci, v, n_cols)
        return betas[(i, shape)]

    def timed(fn, stream=None):
        t = event_time(torch, fn, steps, warmup, stream)
        return t

    def row(t, ab):
        return {"us": round(t * 1e6, 1), "gflops": round(flops / t / 1e9, 1), "alg_GBs": round(ab / t / 1e9, 1),
                "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4)}

    for name, (sel, model) in selectors.items():
        if sel is None:
            continue
        method = spc.SEL_MLP if model else spc.SEL_INTERP
        classes = [sel.select(f, method)[0] for f in feats]
        Bs, params = [], []
        for i, k in enumerate(classes):
            shape = spc.class_shape(k)
            # a shape's own class runs its fastest of modes 0, 3 and 4; a test class, mode 2
            modes = (2,) if spc.class_mode(k) == 2 else (0, 3, 4)
            B = beta(i, shape)
            Bs.append(B)
            params.append(batch_plan(spc, B, modes, tune_cache, (i, shape)))
        ys = [torch.empty(m[4], dtype=torch.float64, device=dev) for m in mats]
        batch = spc.Batch(Bs, params=params).set_vectors(xs, ys)
        plans = [spc.plan_from(B, p) for B, p in zip(Bs, params)]
        ab = sum(algorithmic_bytes(B, P.info()["n_tiles"]) for B, P in zip(Bs, plans))
        info = batch.info()
        res = {"selector": "mlp" if model else "interpolation", "n_classes": sel.n_classes(method),
               "class_share": np.bincount(classes, minlength=8).tolist(), "n_groups": info["n_groups"],
               "n_tiles": info["n_tiles"], "alg_bytes": ab,
               "chunks_share": {str(q): sum(1 for p in params if p["wave_chunks"] == q) for q in (2, 4, 6, 8)},
               "mode_share": {str(m): sum(1 for p in params if p["mode"] == m) for m in (0, 2, 3, 4)}}

        def sep():
            for B, x, y, P in zip(Bs, xs, ys, plans):
                spc.spmv(B, x, y, plan=P)

        sep()
        torch.cuda.synchronize()
        ref = [y.clone() for y in ys]
        side = torch.cuda.Stream()
        res["grouped"] = row(timed(lambda: batch.run()), ab)
        res["grouped_persistent_2048wg"] = row(timed(lambda: batch.run(grid_blocks=2048)), ab)
        res["grouped_graph"] = row(timed(lambda: batch.run(use_graph=True), side), ab)
        res["separate_launches"] = row(timed(sep), ab)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            sep()
        res["separate_launches_graph"] = row(timed(g.replay, side), ab)
        # each matrix alone in its plan, summed: what the batch's tiles cost without any overlap
        res["sum_of_single_launches_us"] = round(sum(
            spc.time_spmv(B, P, reps=max(3, steps // 2)) for B, P in zip(Bs, plans)), 1)
        batch.run()
        torch.cuda.synchronize()
        res["bitwise_equal_to_separate"] = all(torch.equal(a, b) for a, b in zip(ys, ref))
        res["speedup_grouped_vs_separate"] = round(res["separate_launches"]["us"] / res["grouped"]["us"], 3)
        out[name] = res
        del batch, plans, g
    # the earlier single-launch form: every matrix in mode 0 with 4 chunks, one
    # launch of the shape-switching kernel, shapes as the 6-class selector picks
    ref_name = "classes_6" if "classes_6" in out else next((k for k in out if k.startswith("classes_")), None)
    if ref_name is not None:
        sel, model = selectors[ref_name]
        method = spc.SEL_MLP if model else spc.SEL_INTERP
        Bs = [beta(i, spc.class_shape(sel.select(f, method)[0])) for i, f in enumerate(feats)]
        ys = [torch.empty(m[4], dtype=torch.float64, device=dev) for m in mats]
        batch = spc.Batch(Bs, wave_chunks=4).set_vectors(xs, ys).set_kernel(True)
        ab = sum(algorithmic_bytes(B, B.plan(0, 0, 0, 4).info()["n_tiles"]) for B in Bs)
        out["shape_switching_one_launch_kq4"] = row(timed(lambda: batch.run()), ab)
    best = out.get("classes_8") or out.get("classes_6")
    if best is not None:
        out["speedup_one_launch_vs_separate"] = best["speedup_grouped_vs_separate"]
    if "classes_8" in out and "classes_6" in out:
        out["time_8_classes_over_6_classes"] = round(out["classes_8"]["grouped"]["us"]
                                                     / out["classes_6"]["grouped"]["us"], 4)
    return out


def reorder_section(spc, torch, pool, tmp, m: int):
    """Reordering before conversion on the 27-point stencil of an m^3 grid
    whose points are numbered at random: values per block, and the fastest
    product of each shape (autotuned), before and after the reverse
    Cuthill-McKee renumbering; the cost of the order (host walk), of the
    device permutation and of permuting x and y per product."""
    import numpy as np

    import oracle
    dev = torch.device("cuda")
    _, n_rows, n_cols, base = pool.apply(_gen_scrambled, ((m, tmp),))
    A = _load_csr(base, n_rows, n_cols)
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colidx).to(dev)
    v = torch.from_numpy(A.values).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm = spc.rcm_order(rp, ci)
    torch.cuda.synchronize()
    t_order = time.perf_counter() - t0
    t0 = time.perf_counter()
    rp2, ci2, v2 = spc.csr_permute(rp, ci, v, perm)
    torch.cuda.synchronize()
    t_perm = time.perf_counter() - t0
    from paper_1801_01134_amd import synth
    x = torch.from_numpy(synth.dense_vector(A.n_cols, 5)).to(dev)
    out = {"workload": f"27-point stencil {m}^3 with randomly numbered grid points (n={A.n_rows}, nnz={A.nnz})",
           "rcm_order_ms": round(t_order * 1e3, 1), "csr_permute_ms": round(t_perm * 1e3, 2),
           "order_on": "host (breadth-first walk); permutation on the device", "shapes": {}}
    xp = spc.permute_vector(x, perm)
    t = event_time(torch, lambda: spc.permute_vector(x, perm), 20, 3)
    out["permute_vector_us"] = round(t * 1e6, 2)
    best = {}
    for label, (a_, b_, c_) in (("random_numbering", (rp, ci, v)), ("rcm", (rp2, ci2, v2))):
        for (r, c) in spc.SHAPES:
            B = spc.csr_to_beta(r, c, a_, b_, c_, A.n_cols)
            params, us, _ = spc.autotune(B, reps=10, x=x if label != "rcm" else xp)
            key = f"b{r}x{c}"
            out["shapes"].setdefault(key, {})[label] = {"avg_nnz_per_block": round(A.nnz / B.n_blocks, 3),
                                                        "us": round(us, 2), "plan": params}
            best[label] = min(best.get(label, 1e30), us)
            del B
            torch.cuda.empty_cache()
    out["best_us"] = {k: round(v_, 2) for k, v_ in best.items()}
    out["speedup_best_shape"] = round(best["random_numbering"] / best["rcm"], 3)
    # the fastest reordered product, mapped back, against the oracle on the original matrix
    fastest = min(out["shapes"], key=lambda k: out["shapes"][k]["rcm"]["us"])
    r, c = (int(t_) for t_ in fastest[1:].split("x"))
    out["rcm_fastest_shape"] = [r, c]
    B = spc.csr_to_beta(r, c, rp2, ci2, v2, A.n_cols)
    y = spc.permute_vector(spc.spmv(B, xp), perm, scatter=True).cpu().numpy()
    y_ref, s_ref = oracle.csr_spmv(A, x.cpu().numpy())
    out["rcm_product_matches_oracle"] = bool((np.abs(y - y_ref) <= 1e-13 * s_ref).all())
    return out


def shares_section(spc, torch, rp, ci, v64, n_cols, nnz, params, r, c):
    """The headline product on streams restricted to a share of the compute
    units, and the held-out regrets of the 2-D (Avg, share) model against
    the sequential per-kernel polynomial, from the committed share records."""
    out = {}
    B = spc.csr_to_beta(r, c, rp, ci, v64, n_cols)
    P = spc.plan_from(B, params)
    total = spc.device_cu_count()
    live = {}
    for n in (total // 8, total // 4, total // 2, total):
        cs = spc.CUStream(n)
        with torch.cuda.stream(cs.stream):
            us = spc.time_spmv(B, P, reps=20, warmup=3)
        cs.close()
        live[str(n)] = {"us": round(us, 2), "gflops": round(2.0 * nnz / (us * 1e-6) / 1e9, 1)}
    out["headline_kernel_by_cu_count"] = live
    path = os.path.join(MODEL_DIR, "selector_shares_mi355x.jsonl")
    if os.path.exists(path):
        from paper_1801_01134_amd import records as R
        recs = R.load(path)
        tr, te = R.split(recs)
        out["held_out"] = R.evaluate_shares(tr, te)
    return out


def cg_section(spc, torch, pool, tmp, m: int, ks, fp32_ks):
    import numpy as np

    from oracle import cg as ocg
    from paper_1801_01134_amd import synth
    dev = torch.device("cuda")
    _, n_rows, n_cols, base = pool.apply(_gen_cg, ((m, tmp),))
    A = _load_csr(base, n_rows, n_cols)
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colidx).to(dev)
    out = {"grid": m, "n": A.n_rows, "nnz": A.nnz, "runs": []}
    for dt, kset, tol in ((torch.float64, ks, 1e-8), (torch.float32, fp32_ks, 1e-5)):
        vals = torch.from_numpy(A.values).to(dev).to(dt)
        # per k: the fastest SpMM among two shapes x four chunk counts x four
        # caps on resident workgroups per compute unit x the two SpMM kernels
        # (mask-bit lanes; the row path where the columns come in 16-byte groups)
        Bs = {rc: spc.csr_to_beta(rc[0], rc[1], rp, ci, vals, A.n_cols) for rc in ((2, 4), (4, 8))}
        for k in kset:
            Bm = synth.dense_block(A.n_cols, k, 701 + k)
            Bd = torch.from_numpy(Bm).to(dev).to(dt)
            X = torch.from_numpy(synth.dense_block(A.n_cols, k, 702)).to(dev).to(dt)
            best = None
            grouped = (k * X.element_size()) % 16 == 0
            for rc, Bc in Bs.items():
                for kq in (2, 4, 6, 8):
                    for cap in (0, 2, 3, 4):
                        for path in ((spc.SPMM_BITS, spc.SPMM_ROWS) if grouped else (spc.SPMM_BITS,)):
                            Pc = Bc.plan(0, 0, 0, kq, 0, cap, 0, path)
                            t = event_time(torch, lambda: spc.spmm(Bc, X, plan=Pc), 10, 2)
                            if best is None or t < best[0]:
                                best = (t, rc, kq, cap, path)
            t_spmm, (r, c), kq, cap, path = best
            B = Bs[(r, c)]
            P = B.plan(0, 0, 0, kq, 0, cap, 0, path)
            s = torch.cuda.Stream()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(s):
                Xs, its, res, total = spc.cg(B, Bd, rel_tol=tol, max_iter=5000, check_every=25, plan=P)
            s.synchronize()
            wall = time.perf_counter() - t0
            Xh = Xs.cpu().numpy().astype(np.float64)
            Bh = Bd.cpu().numpy().astype(np.float64)
            true = ocg.true_residual(A, Xh, Bh) / np.linalg.norm(Bh, axis=0)
            ab = algorithmic_bytes(B, P.info()["n_tiles"], k=k)
            out["runs"].append({
                "dtype": "f64" if dt == torch.float64 else "f32", "k": k, "shape": [r, c], "wave_chunks": kq,
                "cu_groups": cap, "spmm_path": "rows" if path == spc.SPMM_ROWS else "mask-bit lanes",
                "rel_tol": tol, "iterations": its, "iterations_run": total,
                "true_rel_residual_max": float(true.max()),
                "converged": bool(all(i > 0 for i in its) and true.max() <= 10 * tol),
                "cg_ms": round(wall * 1e3, 2), "ms_per_iteration": round(wall * 1e3 / max(1, total), 4),
                "spmm_us": round(t_spmm * 1e6, 1), "spmm_gflops": round(2.0 * A.nnz * k / t_spmm / 1e9, 1),
                "spmm_alg_GBs": round(ab / t_spmm / 1e9, 1),
                "spmm_hbm_frac": round(ab / t_spmm / 1e9 / HBM_PEAK_GBS, 4),
                "spmm_share_of_iteration": round(t_spmm * total / wall, 3) if total else None})
            log(f"cg {out['runs'][-1]}")
            del X, Xs, Bd
        del B, P, Bs, vals
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=128, help="stencil grid edge (128 -> 2.1M rows)")
    ap.add_argument("--sweep-steps", type=int, default=20, help="timed launches per autotune candidate")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--shape", default="auto", help="r,c of the headline kernel, or auto")
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"),
                    help="arithmetic of the headline product (f64; f32 is for profiling the FP32 kernels)")
    ap.add_argument("--only-headline", action="store_true", help="skip the sweep and every extra section")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-reorder", action="store_true")
    ap.add_argument("--no-shares", action="store_true")
    ap.add_argument("--no-select", action="store_true")
    ap.add_argument("--batched-matrices", type=int, default=64)
    ap.add_argument("--cg-grid", type=int, default=192)
    ap.add_argument("--plan", default="", help="mode,wave_chunks_or_tile_bits,tile_order[,pipeline[,cu_groups[,wave_tiles]]]: force "
                    "the headline plan (skips autotuning; used for profiling)")
    ap.add_argument("--spmm", default="",
                    help="k,dtype(64|32),wave_chunks,cu_groups[,spmm_path]: time only Y = A X on the CG matrix "
                         "(used for profiling the multi-RHS kernels; spmm_path 1 = mask-bit lanes, 2 = rows)")
    ap.add_argument("--only-steps", action="store_true",
                    help="run only the other steps (conversion, features, network) and print them")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run only a plain 256 MiB copy (memory-counter calibration)")
    args = ap.parse_args(argv)

    if args.copy_ref:
        # a plain copy of known size: calibrates the memory counters
        import torch
        n = 256 * 2**20 // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4}))
        return 0
    if args.spmm:
        return spmm_only(args)
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} refused: this build measures one GPU only "
              "(the multi-GPU sharding is described in DESIGN.md, not run)", file=sys.stderr)
        return 2
    extras = not args.only_headline
    do_batched = extras and not args.no_batched
    do_cg = extras and not args.no_cg
    args.do_reorder = extras and not args.no_reorder
    args.do_shares = extras and not args.no_shares
    do_select = extras and not args.no_select

    # worker processes for the CPU-side matrix generation, forked before any GPU call
    pool = None
    tmp = tempfile.mkdtemp(prefix="spc_bench_")
    if do_batched or do_cg or args.do_reorder:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(12)

    try:
        return run(args, pool, tmp, do_batched, do_cg, do_select)
    finally:
        if pool is not None:
            pool.terminate()
            pool.join()
        for f in os.listdir(tmp):
            os.remove(os.path.join(tmp, f))
        os.rmdir(tmp)


def spmm_only(args):
    """Y = A X on the SPD 27-point matrix of the CG section (beta(2,4)), one
    plan, `steps` timed launches after `warmup`; one JSON line."""
    import torch

    import paper_1801_01134_amd as spc
    from paper_1801_01134_amd import synth
    fields = [int(t) for t in args.spmm.split(",")]
    k, bits, kq, cap = fields[:4]
    path = fields[4] if len(fields) > 4 else 0
    dt = torch.float64 if bits == 64 else torch.float32
    dev = torch.device("cuda:0")
    A = synth.stencil27(args.cg_grid, diag=26.1, offdiag=-1.0)
    B = spc.csr_to_beta(2, 4, torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colidx).to(dev),
                        torch.from_numpy(A.values).to(dev).to(dt), A.n_cols)
    X = torch.from_numpy(synth.dense_block(A.n_cols, k, 702)).to(dev).to(dt)
    Y = torch.empty(A.n_rows, k, dtype=dt, device=dev)
    P = B.plan(0, 0, 0, kq, 0, cap, 0, path)
    t = event_time(torch, lambda: spc.spmm(B, X, Y, plan=P), args.steps, args.warmup)
    ab = algorithmic_bytes(B, P.info()["n_tiles"], k=k)
    print(json.dumps({"workload": f"27-point SPD stencil {args.cg_grid}^3 (n={A.n_rows}, nnz={A.nnz}), "
                                  f"beta(2,4), Y = A X, k = {k}, FP{bits}",
                      "plan": {"wave_chunks": kq, "cu_groups": cap, "spmm_path": path}, "us": round(t * 1e6, 1),
                      "alg_bytes_per_launch": ab, "alg_GBs": round(ab / t / 1e9, 1),
                      "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4)}), flush=True)
    return 0


def run(args, pool, tmp, do_batched, do_cg, do_select):
    import torch

    import paper_1801_01134_amd as spc
    from paper_1801_01134_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m = args.grid
    t_gen = time.perf_counter()
    A = synth.stencil27(m, diag=27.0)
    x64 = synth.dense_vector(A.n_cols, 1)
    log(f"generated {m}^3 stencil: n={A.n_rows} nnz={A.nnz} in {time.perf_counter() - t_gen:.1f}s")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colidx).to(dev)
    v64 = torch.from_numpy(A.values).to(dev)
    flops = 2.0 * A.nnz
    csr_bytes = {8: A.nnz * 12 + (A.n_rows + 1) * 4, 4: A.nnz * 8 + (A.n_rows + 1) * 4}
    if args.only_steps:
        sel, model = main_selector(load_selectors(spc)[0])
        print(json.dumps({"step_timings": steps_section(spc, torch, A, rp, ci, v64, sel, model)}), flush=True)
        return 0

    sweep = {}
    best_params = {}
    top_params = {}
    for dt in (torch.float64, torch.float32):
        if args.only_headline:
            break
        xd = torch.from_numpy(x64).to(dev).to(dt)
        for (r, c) in spc.SHAPES:
            B = spc.csr_to_beta(r, c, rp, ci, v64.to(dt), A.n_cols)
            _, us_tune, records = spc.autotune(B, reps=args.sweep_steps, x=xd)
            # the three fastest candidates of the shape's own kernels and the
            # fastest test-kernel candidate, timed again with more launches
            own = sorted((q for q in records if q["mode"] != 2), key=lambda q: q["us"])[:3]
            tst = sorted((q for q in records if q["mode"] == 2), key=lambda q: q["us"])[:1]

            def retime(q):
                p_ = {k: v for k, v in q.items() if k not in ("us", "n_tiles")}
                P_ = spc.plan_from(B, p_)
                return min(spc.time_spmv(B, P_, reps=100, warmup=5) for _ in range(2)), p_

            own_t = sorted((retime(q) for q in own), key=lambda tp: tp[0])
            tst_t = [retime(q) for q in tst]
            us, params = min(own_t + tst_t, key=lambda tp: tp[0])
            t = us * 1e-6
            P = spc.plan_from(B, params)
            info = P.info()
            ab = algorithmic_bytes(B, info["n_tiles"])
            key = f"{'f64' if dt == torch.float64 else 'f32'}_b{r}x{c}"
            best_params[key] = params
            top_params[key] = [p_ for _, p_ in sorted(own_t + tst_t, key=lambda tp: tp[0])]
            sweep[key] = {"us": round(us, 2), "gflops": round(flops / t / 1e9, 1),
                          "us_own_kernels": round(own_t[0][0], 2),
                          "us_test_kernel": round(tst_t[0][0], 2) if tst_t else None,
                          "us_autotuner": round(us_tune, 2),
                          "alg_GBs": round(ab / t / 1e9, 1), "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4),
                          "alg_bytes": ab, "matrix_bytes": B.nbytes(),
                          "matrix_vs_csr": round(B.nbytes() / csr_bytes[B.values.element_size()], 4),
                          "n_blocks": B.n_blocks, "avg_nnz_per_block": round(A.nnz / B.n_blocks, 3),
                          "n_tiles": info["n_tiles"], "n_long": info["n_long"], "plan": params,
                          "candidates": len(records)}
            log(f"{key}: {sweep[key]}")
            del B, P
            torch.cuda.empty_cache()

    # headline kernel: FP64, the fastest in the records above (or forced)
    if args.shape == "auto" and not sweep:
        r, c = 2, 4
    elif args.shape == "auto":
        f64 = {k: v for k, v in sweep.items() if k.startswith("f64_")}
        best = min(f64, key=lambda k: f64[k]["us"])
        r, c = (int(s) for s in best[5:].split("x"))
    else:
        r, c = (int(s) for s in args.shape.split(","))
    hdt = torch.float64 if args.dtype == "f64" else torch.float32
    tname = "double" if args.dtype == "f64" else "float"
    xd = torch.from_numpy(x64).to(dev).to(hdt)
    yd = torch.empty(A.n_rows, dtype=hdt, device=dev)
    B = spc.csr_to_beta(r, c, rp, ci, v64.to(hdt), A.n_cols)
    if args.plan:
        fields = [int(t) for t in args.plan.split(",")]
        m_, v_, o_ = fields[:3]
        params = {"mode": m_, "wave_chunks": v_ if m_ != 1 else 0, "tile_bits": v_ if m_ == 1 else 0,
                  "tile_order": o_, "pipeline": fields[3] if len(fields) > 3 else 0}
        if len(fields) > 4 and fields[4]:
            params["cu_groups"] = fields[4]
        if len(fields) > 5 and fields[5]:
            params["wave_tiles"] = fields[5]
    else:
        params = best_params.get(f"{args.dtype}_b{r}x{c}") or spc.autotune(B, reps=args.sweep_steps, x=xd)[0]
        # the sweep's three fastest plans of this kernel, timed again with more
        # launches: near-ties between them are decided on a longer sample
        cands = top_params.get(f"{args.dtype}_b{r}x{c}", [])
        if len(cands) > 1:
            timed = [(spc.time_spmv(B, spc.plan_from(B, p_), reps=100), i) for i, p_ in enumerate(cands)]
            params = cands[min(timed)[1]]
    P = spc.plan_from(B, params)
    info = P.info()
    kname = ({0: f"k_spmv_wave{'_pipe' if params.get('pipeline') else ('2' if params.get('wave_tiles') == 2 else '')}"
                 f"<{r},{c},{tname},{params['wave_chunks'] or 4}>",
              2: f"k_spmv_test<{r},{c},{tname},{params['wave_chunks'] or 4}>",
              3: f"k_spmv_brow<{r},{c},{tname},{params['wave_chunks'] or 4}>",
              4: f"k_spmv_vlane<{tname},{params['wave_chunks'] or 4}>"}.get(
                 params["mode"], f"k_spmv_wg<{r},{c},{tname},{info['tile_bits']}>"))
    for _ in range(args.warmup):
        spc.spmv(B, xd, yd, plan=P)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        spc.spmv(B, xd, yd, plan=P)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_kernel = e0.elapsed_time(e1) * 1e-3 / args.steps
    ms_per_step = wall / args.steps * 1e3
    ab = algorithmic_bytes(B, info["n_tiles"])
    achieved = ab / t_kernel / 1e9
    value = flops / (wall / args.steps) / 1e9
    traffic = committed_profile("traffic", kname, (r, c), params, m)
    trace = committed_profile("trace", kname, (r, c), params, m)
    # the timed launches' result against the CSR oracle, per row (FP64; FP32
    # from the FP32-rounded inputs)
    import numpy as np

    import oracle
    if args.dtype == "f64":
        y_ref, s_ref = oracle.csr_spmv(A, x64)
        tol = 1e-13
    else:
        y_ref, s_ref = oracle.csr_spmv(A.astype(np.float32), x64.astype(np.float32))
        tol = 2e-6
    err = abs(yd.cpu().numpy().astype(np.float64) - y_ref)
    matches = bool((err <= tol * s_ref).all())
    worst = float((err / (tol * s_ref + 1e-300)).max())
    del B, P

    # selection: kernel classes picked from the matrix's features alone; the
    # time of a class is its shape's own kernels (classes 0-5) or its test
    # kernel (6, 7), each autotuned in the sweep above
    selection = None
    ratio = None
    sels = {}
    sel = model = None
    if do_select:
        sels, held_out = load_selectors(spc)
        sel, model = main_selector(sels)
        feat, nb = spc.matrix_features(rp, ci, A.n_cols)
        cls_times = []
        for k in range(spc.N_CLASSES):
            r_, c_ = spc.SHAPES[spc.class_shape(k)]
            e = sweep.get(f"f64_b{r_}x{c_}")
            cls_times.append(None if e is None else (e["us_test_kernel"] if k >= 6 else e["us_own_kernels"]))
        selection = {"features": [round(float(v), 5) for v in feat], "held_out_regret": held_out}
        if sels and all(t is not None for t in cls_times):
            t_best = min(cls_times)
            selection["class_times_us"] = cls_times
            for name, (sel_, model_) in sels.items():
                sm, si = select_class(spc, sel_, model_, feat)
                d = {}
                for meth, k in (("mlp", sm), ("interpolation", si)):
                    if k is not None:
                        d[meth] = {"class": k, "shape": list(spc.SHAPES[spc.class_shape(k)]),
                                   "test_kernel": k >= 6, "time_ratio": round(cls_times[k] / t_best, 4)}
                selection[name] = d
            main = selection.get("classes_8", selection.get("classes_6", {}))
            ratio = main.get("mlp", main.get("interpolation", {})).get("time_ratio")
        elif not sweep:
            selection["note"] = "no sweep (only-headline): ratios need every kernel's time"

    out = {
        "metric": "SpMV GFlop/s + HBM GB/s % of peak; selected-vs-best kernel time ratio",
        "value": round(value, 2), "unit": "GFlop/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"27-point stencil {m}^3 (n={A.n_rows}, nnz={A.nnz}), {args.dtype.upper()} y=A*x, "
                               f"beta({r},{c}) kernel", "shape": [r, c], "n_rows": A.n_rows,
                   "nnz": A.nnz, "tile_bits": info.get("tile_bits"), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic["traffic_bytes_per_launch"] if traffic else None,
                     "traffic_source": traffic["source"] if traffic else "no counter record for this kernel build",
                     "kernel": kname, "plan": params,
                     "alg_bytes_per_launch": ab, "kernel_us": round(t_kernel * 1e6, 2),
                     "kernel_us_source": f"HIP events around {args.steps} back-to-back launches on the launch stream",
                     "kernel_us_trace": trace["avg_ns"] / 1e3 if trace else None,
                     "frac_trace": round(ab / (trace["avg_ns"] * 1e-9) / 1e9 / HBM_PEAK_GBS, 4) if trace else None,
                     "trace_source": trace["source"] if trace else "no kernel trace for this kernel build and plan",
                     "target_frac": 0.70,
                     "matches_oracle": matches, "max_err_over_bound": round(worst, 4)},
        "selected_vs_best_time_ratio": ratio,
        "headline_selection": "fastest of the six beta kernels on this matrix, each autotuned over its plan "
                              "candidates (records taken in this run)" if args.shape == "auto" else "forced",
        "selection": selection,
        "per_kernel": sweep,
    }
    if do_select:
        out["step_timings"] = steps_section(spc, torch, A, rp, ci, v64, sel, model)
        log(f"step timings: {out['step_timings']}")
        torch.cuda.empty_cache()
    if do_batched:
        if not sels:
            sels, _ = load_selectors(spc)
        out["batched"] = batched_section(spc, torch, sels, pool, tmp, args.batched_matrices,
                                         max(5, args.steps // 10), 3)
        log(f"batched: {out['batched']}")
        torch.cuda.empty_cache()
        out["batched_small"] = batched_section(spc, torch, sels, pool, tmp, 512, max(5, args.steps // 10), 3,
                                               min_rows=500, max_rows=20_000)
        log(f"batched small: {out['batched_small']}")
        torch.cuda.empty_cache()
    if do_cg:
        out["cg"] = cg_section(spc, torch, pool, tmp, args.cg_grid, (1, 4, 8, 16), (1, 16))
        torch.cuda.empty_cache()
    if args.do_reorder:
        out["reorder"] = reorder_section(spc, torch, pool, tmp, m)
        log(f"reorder: {out['reorder']}")
        torch.cuda.empty_cache()
    if args.do_shares:
        out["parallel_estimation"] = shares_section(spc, torch, rp, ci, v64, A.n_cols, A.nnz, params, r, c)
        log(f"parallel estimation: {out['parallel_estimation']}")
        torch.cuda.empty_cache()
    if not args.only_headline:
        out["small_case"] = small_case(spc, torch)
        log(f"small case: {out['small_case']}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, x64, f"{m}^3 27-point matrix")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
