"""GPU parity of the multi-RHS product and of the CG driver against the CPU
oracle. SpMM: per entry |Y - Y_ref| <= tol * sum_j |a_ij X[j][q]| (1e-13
FP64, 2e-6 FP32). CG: the true residual, recomputed by the oracle from the
GPU's X, meets the tolerance; manufactured solutions are recovered."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import cg as ocg
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-13, torch.float32: 2e-6}
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dense_rows():
    a = synth.uniform_random(300, 5000, 4.0, seed=5)
    rows = np.repeat(np.arange(300), a.row_lengths())
    extra_r = np.repeat(np.array([3, 4, 150, 299]), 5000)
    extra_c = np.tile(np.arange(5000), 4)
    return synth._from_keys(300, 5000, np.concatenate([rows, extra_r]),
                            np.concatenate([a.colidx.astype(np.int64), extra_c]), synth.rng_for(56))


CASES = {
    "stencil13": lambda: synth.stencil27(13),
    "powerlaw": lambda: synth.powerlaw(2001, 2001, seed=2),
    "dense_rows": _dense_rows,
    "fem6": lambda: synth.fem_blocks(200, 6, 5.0, 10, seed=3),
    "tall": lambda: synth.uniform_random(9000, 37, 3.0, seed=9),
    # one entry per row: tiles at their cap of 127 intervals / 128 pairs
    "diagonal": lambda: synth.from_keys_sorted(6007, 6007, np.arange(6007), np.arange(6007), 11),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


def to_beta(A, r, c, dtype):
    return spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values).to(dtype), A.n_cols)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("k", [1, 3, 4, 8, 16])
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_spmm_parity(rc, name, k, dtype):
    r, c = rc
    A = case(name).astype(NP[dtype])
    say(f"[spmm] {name} beta{rc} k={k} {dtype}")
    X = synth.dense_block(A.n_cols, k, 31, dtype=NP[dtype])
    Y_ref, S_ref = oracle.csr_spmm(A, X)
    B = to_beta(A, r, c, dtype)
    Y = spc.spmm(B, torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(Y.astype(np.float64) - Y_ref)
    bad = np.argwhere(~(err <= TOL[dtype] * S_ref))
    assert bad.size == 0, f"{bad.shape[0]} entries off, first {bad[0]}: {Y[tuple(bad[0])]} vs {Y_ref[tuple(bad[0])]}"


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_spmm_strided_and_accumulate(rc):
    r, c = rc
    say(f"[spmm strided] beta{rc}")
    A = case("powerlaw")
    k = 5
    big = synth.dense_block(A.n_cols, 11, 32)
    X = torch.from_numpy(big).cuda()[:, 2:2 + k]          # leading dimension 11
    Y0 = synth.dense_block(A.n_rows, 9, 33)
    Yt = torch.from_numpy(Y0.copy()).cuda()
    Yv = Yt[:, 1:1 + k]                                     # leading dimension 9
    B = to_beta(A, r, c, torch.float64)
    spc.spmm(B, X, Yv, accumulate=True)
    Y_ref, S_ref = oracle.csr_spmm(A, big[:, 2:2 + k])
    got = Yt.cpu().numpy()
    want = Y0.copy()
    want[:, 1:1 + k] += Y_ref
    assert np.all(np.abs(got - want) <= 1e-13 * (S_ref.max() + np.abs(Y0).max()))
    # untouched columns stay bit for bit
    assert np.array_equal(got[:, :1], Y0[:, :1]) and np.array_equal(got[:, 1 + k:], Y0[:, 1 + k:])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_spmm_grouped_columns_strided(rc, dtype):
    """k a multiple of the 16-byte column group, X and Y views with aligned
    leading dimensions: the grouped gathers, checked against the oracle and
    against the same product taken one column at a time."""
    r, c = rc
    say(f"[spmm grouped] beta{rc} {dtype}")
    A = case("powerlaw").astype(NP[dtype])
    k = 8
    big = synth.dense_block(A.n_cols, 12, 34, dtype=NP[dtype])
    X = torch.from_numpy(big).cuda()[:, 4:4 + k]           # leading dimension 12, 16-byte aligned start
    Y0 = synth.dense_block(A.n_rows, 12, 35, dtype=NP[dtype])
    Yt = torch.from_numpy(Y0.copy()).cuda()
    B = to_beta(A, r, c, dtype)
    spc.spmm(B, X, Yt[:, 4:4 + k], accumulate=True)
    Y_ref, S_ref = oracle.csr_spmm(A, big[:, 4:4 + k])
    got = Yt.cpu().numpy().astype(np.float64)
    want = Y0.astype(np.float64)
    want[:, 4:4 + k] += Y_ref
    tol = TOL[dtype] * (S_ref + np.abs(Y0[:, 4:4 + k]))
    assert np.all(np.abs(got[:, 4:4 + k] - want[:, 4:4 + k]) <= tol)
    assert np.array_equal(got[:, :4], Y0[:, :4].astype(np.float64))
    # column by column through the one-column path (a strided view of X, so
    # not the single-vector kernel, which sums long rows in its own order):
    # the same bits as the grouped pass of the mask-bit kernel
    bits = B.plan(0, 0, 0, 0, 0, 0, 0, spc.SPMM_BITS)
    Yg = spc.spmm(B, X.contiguous(), plan=bits)
    for q in range(k):
        yq = spc.spmm(B, X[:, q:q + 1], plan=bits)
        assert torch.equal(yq[:, 0], Yg[:, q]), q
    # a contiguous single column runs the single-vector kernel: same values
    # within the tolerance
    y1 = spc.spmm(B, X[:, :1].contiguous())[:, 0].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(y1 - Y_ref[:, 0]) <= TOL[dtype] * S_ref[:, 0])


@pytest.mark.parametrize("dtype,k", [(torch.float64, 2), (torch.float64, 8), (torch.float64, 12),
                                     (torch.float64, 16), (torch.float32, 4), (torch.float32, 16)],
                         ids=["f64k2", "f64k8", "f64k12", "f64k16", "f32k4", "f32k16"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_spmm_row_path_matches_oracle_and_bit_lanes(rc, dtype, k):
    """The row path (values sorted by row in LDS, lanes on rows and 16-byte
    column groups) forced on, on every case matrix (long intervals, tiles of
    127 one-entry intervals, empty rows): each entry within the bound of the
    oracle, repeated calls bit for bit, y += A X leaving empty rows alone,
    and the mask-bit kernel within the same bound."""
    r, c = rc
    for name in CASES:
        A = case(name).astype(NP[dtype])
        say(f"[spmm rows] {name} beta{rc} {dtype} k={k}")
        B = to_beta(A, r, c, dtype)
        X = torch.from_numpy(synth.dense_block(A.n_cols, k, 37, dtype=NP[dtype])).cuda()
        Y_ref, S_ref = oracle.csr_spmm(A, X.cpu().numpy())
        for kq in (2, 4, 8):
            rows = B.plan(0, 0, 0, kq, 0, 0, 0, spc.SPMM_ROWS)
            bits = B.plan(0, 0, 0, kq, 0, 0, 0, spc.SPMM_BITS)
            Yr = spc.spmm(B, X, plan=rows)
            assert torch.equal(spc.spmm(B, X, plan=rows), Yr)
            for Y in (Yr, spc.spmm(B, X, plan=bits)):
                err = np.abs(Y.cpu().numpy().astype(np.float64) - Y_ref)
                bad = np.argwhere(~(err <= TOL[dtype] * S_ref))
                assert bad.size == 0, (name, kq, bad[:3])
            # accumulate: rows without entries keep their value bit for bit
            Y0 = torch.from_numpy(synth.dense_block(A.n_rows, k, 38, dtype=NP[dtype])).cuda()
            Ya = Y0.clone()
            spc.spmm(B, X, Ya, accumulate=True, plan=rows)
            empty = np.diff(A.rowptr) == 0
            assert torch.equal(Ya[torch.from_numpy(empty).cuda()], Y0[torch.from_numpy(empty).cuda()])
            err = np.abs(Ya.cpu().numpy().astype(np.float64) - (Y0.cpu().numpy().astype(np.float64) + Y_ref))
            assert np.all(err <= TOL[dtype] * (S_ref + np.abs(Y0.cpu().numpy()))), (name, kq)


def test_spmm_row_path_needs_grouped_columns():
    A = case("powerlaw")
    B = to_beta(A, 2, 4, torch.float64)
    X = torch.from_numpy(synth.dense_block(A.n_cols, 5, 39)).cuda()
    with pytest.raises(spc.SpcError):
        spc.spmm(B, X, plan=B.plan(0, 0, 0, 4, 0, 0, 0, spc.SPMM_ROWS))
    with pytest.raises(spc.SpcError):
        B.plan(0, 0, 0, 4, 0, 0, 0, 3)


def _spd(m):
    return synth.stencil27(m, diag=26.1, offdiag=-1.0)


@pytest.mark.parametrize("k", [1, 4])
@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 8)], ids=lambda s: f"b{s[0]}x{s[1]}")
def test_cg_fp64_manufactured(rc, k):
    r, c = rc
    say(f"[cg f64] beta{rc} k={k}")
    A = _spd(12)
    xs = synth.dense_block(A.n_cols, k, 40)
    Bm, _ = oracle.csr_spmm(A, xs)
    B = to_beta(A, r, c, torch.float64)
    X, its, res, total = spc.cg(B, torch.from_numpy(Bm).cuda(), rel_tol=1e-10, check_every=5)
    X = X.cpu().numpy()
    assert all(i > 0 for i in its) and all(v <= 1e-10 for v in res)
    true = ocg.true_residual(A, X, Bm)
    assert np.all(true <= 1e-9 * np.linalg.norm(Bm, axis=0))
    assert np.max(np.abs(X - xs)) <= 1e-7 * np.max(np.abs(xs))
    # the oracle's CG stops within a couple of iterations of the GPU's
    _, it_ref, _ = ocg.cg(A, Bm, tol=1e-10)
    assert np.all(np.abs(np.array(its) - it_ref) <= 2)


def test_cg_graph_equals_direct_and_fp32():
    say("[cg graph vs direct, fp32]")
    A = _spd(14)
    Bm = synth.dense_block(A.n_cols, 3, 41)
    B = to_beta(A, 2, 4, torch.float64)
    Bt = torch.from_numpy(Bm).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        X1, it1, r1, t1 = spc.cg(B, Bt, rel_tol=1e-8, use_graph=True, check_every=7)
        X2, it2, r2, t2 = spc.cg(B, Bt, rel_tol=1e-8, use_graph=False, check_every=7)
    s.synchronize()
    assert torch.equal(X1, X2) and it1 == it2 and t1 == t2
    assert np.all(ocg.true_residual(A, X1.cpu().numpy(), Bm) <= 2e-8 * np.linalg.norm(Bm, axis=0))
    A32 = A.astype(np.float32)
    B32 = to_beta(A32, 2, 4, torch.float32)
    X3, it3, r3, _ = spc.cg(B32, Bt.float(), rel_tol=1e-5)
    assert all(i > 0 for i in it3)
    true = ocg.true_residual(A32, X3.cpu().numpy().astype(np.float64), Bm.astype(np.float32).astype(np.float64))
    assert np.all(true <= 1e-4 * np.linalg.norm(Bm, axis=0))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 8), (8, 4)], ids=lambda s: f"b{s[0]}x{s[1]}")
def test_resident_group_cap_same_bits(rc, dtype):
    """A plan's cu_groups cap (LDS reserved at launch so that at most that
    many workgroups share a compute unit) changes only where tiles run: SpMM
    and SpMV give the same bits as without it, and match the oracle."""
    r, c = rc
    for name in ("powerlaw", "dense_rows", "diagonal"):
        A = case(name).astype(NP[dtype])
        say(f"[cap] {name} beta{rc} {dtype}")
        B = to_beta(A, r, c, dtype)
        X = synth.dense_block(A.n_cols, 16, 36, dtype=NP[dtype])
        Xd = torch.from_numpy(X).cuda()
        Y_ref, S_ref = oracle.csr_spmm(A, X)
        for kq in (2, 6, 8):
            Y0 = spc.spmm(B, Xd, plan=B.plan(0, 0, 0, kq))
            y0 = spc.spmv(B, Xd[:, 0].contiguous(), plan=B.plan(0, 0, 0, kq))
            for cap in (2, 3, 4, 8):
                P = B.plan(0, 0, 0, kq, 0, cap)
                assert torch.equal(spc.spmm(B, Xd, plan=P), Y0), (name, kq, cap)
                assert torch.equal(spc.spmv(B, Xd[:, 0].contiguous(), plan=P), y0), (name, kq, cap)
        err = np.abs(Y0.cpu().numpy().astype(np.float64) - Y_ref)
        assert np.all(err <= TOL[dtype] * S_ref), name


def test_resident_group_cap_is_checked():
    say("[cap] invalid values")
    A = case("powerlaw")
    B = to_beta(A, 2, 4, torch.float64)
    for bad in (1, 9, -1):
        with pytest.raises(spc.SpcError):
            B.plan(0, 0, 0, 4, 0, bad)
    with pytest.raises(spc.SpcError):
        B.plan(2048, 0, 1, 0, 0, 2)      # mode 1 takes no cap
