"""Streams restricted to a share of the compute units (the second input of
the paper's parallel performance estimation): a product run on a share
gives the same bits as on the whole device, a smaller share is not faster
on a matrix that fills the device, and the share records collected on the
device are complete and consistent with the oracle's block counts."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_cu_count_and_refusals():
    n = spc.device_cu_count()
    assert n >= 8
    for bad in (0, -1, n + 1) + ((12,) if n == 256 else ()):
        with pytest.raises(spc.SpcError):
            spc.CUStream(bad)


@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 8)], ids=lambda s: f"b{s[0]}x{s[1]}")
def test_share_gives_the_same_bits(rc):
    r, c = rc
    say(f"[cu] same bits beta{rc}")
    A = synth.stencil27(40)
    x = synth.dense_vector(A.n_cols, 3)
    y_ref, s_ref = oracle.csr_spmv(A, x)
    B = spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    xd = torch.from_numpy(x).cuda()
    P = B.default_plan()
    y0 = spc.spmv(B, xd, plan=P)
    torch.cuda.synchronize()
    for n in (8, 32, 64, spc.device_cu_count()):
        cs = spc.CUStream(n)
        with torch.cuda.stream(cs.stream):
            y = spc.spmv(B, xd, plan=P)
        cs.stream.synchronize()
        assert torch.equal(y, y0), n
        cs.close()
    assert np.all(np.abs(y0.cpu().numpy() - y_ref) <= 1e-13 * s_ref)


def test_fewer_units_take_longer():
    say("[cu] timing on 16 and all units")
    A = synth.stencil27(96)
    B = spc.csr_to_beta(2, 4, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    P = B.default_plan()
    t = {}
    for n in (16, spc.device_cu_count()):
        cs = spc.CUStream(n)
        with torch.cuda.stream(cs.stream):
            t[n] = spc.time_spmv(B, P, reps=10, warmup=2)
        cs.close()
    assert t[16] > 2.0 * t[spc.device_cu_count()], t


def test_share_records_are_complete():
    say("[cu] collect_shares on two small matrices")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "shares.jsonl")
        R.collect_shares(0, 2, out, "selector", shares=(16, 64, 256), reps=2, workers=0, min_rows=3000,
                         max_rows=6000, log=sys.stdout)
        with open(out) as f:
            lines = [json.loads(s) for s in f if s.strip()]
    assert len(lines) == 2
    for rec in lines:
        fam, A = synth.selector_matrix(rec["index"], 3000, 6000)
        assert rec["family"] == fam and rec["nnz"] == A.nnz
        assert rec["n_blocks"] == [int(oracle.beta_count(A, r, c).sum()) for (r, c) in spc.SHAPES]
        assert rec["cu_counts"] == [16, 64, min(256, rec["cu_total"])]
        assert len(rec["us"]) == 3 and all(len(u) == 6 and min(u) > 0 for u in rec["us"])
