"""The autotuner and the timing records it writes (the paper's record-based
strategy: kernels and their parameters are chosen from timings of earlier
runs). Checks that spc_autotune returns the fastest of the candidates it
timed, that every candidate plan computes the product the oracle computes,
and that records.collect writes complete, self-consistent lines whose block
counts equal the oracle's for the same seeded matrices."""
import json
import os
import sys
import tempfile

import numpy as np
import pytest
import torch

import oracle
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import records as R
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _key(p):
    return tuple(sorted((k, v) for k, v in p.items() if v))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 8)], ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("name", ["stencil24", "powerlaw"])
def test_autotune_best_is_fastest_record_and_matches_oracle(name, rc, dtype):
    r, c = rc
    say(f"[tune] {name} beta{rc} {dtype}")
    A = (synth.stencil27(24) if name == "stencil24" else synth.powerlaw(30000, 30000, seed=8)).astype(NP[dtype])
    x = synth.dense_vector(A.n_cols, 61, dtype=NP[dtype])
    y_ref, s_ref = oracle.csr_spmv(A, x)
    B = spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    xd = torch.from_numpy(x).cuda()
    best, best_us, recs = spc.autotune(B, reps=3, x=xd)
    assert len(recs) >= 30
    assert sum(q["mode"] == 3 for q in recs) == 4
    assert sum(q["mode"] == 4 for q in recs) == (4 if rc == (1, 8) else 0)
    keys = [_key({k: v for k, v in q.items() if k not in ("us", "n_tiles")}) for q in recs]
    assert len(set(keys)) == len(keys), "a candidate was timed twice"
    # the headline launch's plan is among the candidates
    assert _key(dict(mode=0, wave_chunks=8, cu_groups=4)) in keys
    i_min = int(np.argmin([q["us"] for q in recs]))
    assert best_us == recs[i_min]["us"] and best_us > 0
    assert _key(best) == keys[i_min]
    for q in recs:
        p = {k: v for k, v in q.items() if k not in ("us", "n_tiles")}
        P = spc.plan_from(B, p)
        assert P.info()["n_tiles"] == q["n_tiles"]
        y = spc.spmv(B, xd, plan=P).cpu().numpy().astype(np.float64)
        bad = np.flatnonzero(~(np.abs(y - y_ref) <= TOL[dtype] * s_ref))
        assert bad.size == 0, (p, bad[:5])


def test_records_collect_writes_complete_lines():
    say("[tune] records.collect, two small matrices of each population")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "recs.jsonl")
        for pop in R.POPULATIONS:
            R.collect(0, 2, out, reps=2, workers=0, min_rows=3000, max_rows=6000, population=pop,
                      log=sys.stdout)
        with open(out) as f:
            lines = [json.loads(s) for s in f if s.strip()]
    assert len(lines) == 2 * len(R.POPULATIONS)
    for rec in lines:
        fam, A = R.generator(rec["population"])(rec["index"], 3000, 6000)
        assert rec["family"] == fam and rec["n_rows"] == A.n_rows and rec["nnz"] == A.nnz
        assert len(rec["features"]) == 16 and all(np.isfinite(rec["features"]))
        nb = [int(oracle.beta_count(A, r, c).sum()) for (r, c) in spc.SHAPES]
        assert rec["n_blocks"] == nb
        for k in range(6):
            assert rec["features"][8 + k] == pytest.approx(A.nnz / nb[k], rel=1e-6)
        assert len(rec["us"]) == 6 and all(t > 0 for t in rec["us"])
        assert rec["gflops"] == pytest.approx([2.0 * A.nnz / (t * 1e-6) / 1e9 for t in rec["us"]])
        assert len(rec["params"]) == 6 and all(p["mode"] in (0, 1, 3, 4) for p in rec["params"])
        assert all(n > 0 for n in rec["n_tiles"])
        # the test kernels (Algorithm 2) of beta(1,8) and beta(2,4) as classes of their own
        assert len(rec["us_test"]) == 2 and all(t > 0 for t in rec["us_test"])
        assert all(p["mode"] == 2 for p in rec["params_test"])


def _synthetic_records(n, seed):
    """Records whose fastest class follows the features: features are
    random, times depend on them (inputs only; no method arithmetic)."""
    rng = synth.rng_for(520, seed)
    recs = []
    for i in range(n):
        f = rng.uniform(0.5, 8.0, 16)
        t = np.exp(0.4 * rng.standard_normal(8) + 0.3 * f[:8] - 0.3 * f[8:16])
        recs.append({"population": R.POPULATIONS[i % 3], "index": i // 3, "features": f.tolist(),
                     "us": t[:6].tolist(), "us_test": t[6:].tolist(), "nnz": 1000 + i})
    return recs


@pytest.mark.parametrize("k", [6, 8])
def test_records_evaluate_classes(k):
    """records.evaluate on synthetic records: the device-trained network and
    the interpolation are judged with the recorded times; the regrets it
    reports equal the oracle's regret of the same choices."""
    say(f"[records] evaluate {k} classes")
    recs = _synthetic_records(450, k)
    train, test = R.split(recs)
    res, model = R.evaluate(train, test, epochs=30, n_classes=k)
    assert res["n_classes"] == k and model["n_out"] == k and len(model["params"]) == spc.mlp_n_params(k)
    assert res["n_test"] == len(test) and sum(res["mlp_choice_share"]) == len(test)
    assert len(res["best_class_share"]) == k
    # the reported mean regret of the network is the oracle's regret of its choices
    Xte, Tte, _, _ = R.arrays(test, k)
    P = torch.tensor(model["params"], dtype=torch.float32, device="cuda")
    mu = torch.tensor(model["mu"], dtype=torch.float32, device="cuda")
    sd = torch.tensor(model["sd"], dtype=torch.float32, device="cuda")
    _, ch = spc.mlp_infer(P, mu, sd, torch.from_numpy(Xte).cuda())
    ch = ch.cpu().numpy()
    from oracle import select as osel
    reg = np.array([osel.regret(Tte[i], int(ch[i])) for i in range(len(test))])
    assert res["mlp"]["mean"] == pytest.approx(reg.mean(), rel=1e-12, abs=1e-15)
    if k == 8:
        T8 = R.arrays(test, 8)[1]
        assert res["vs_all8"]["mlp"]["mean"] == pytest.approx(
            np.mean([osel.regret(T8[i], int(ch[i])) for i in range(len(test))]), rel=1e-12)
