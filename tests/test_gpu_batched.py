"""Batched products: one launch per group of matrices (same mode, shape and
chunk count) over the tiles of many matrices of different sizes and shapes,
or one launch of the shape-switching kernel. Each y_i is checked against the
oracle with the per-row tolerance; a batched launch runs the same tiles in
the same order of operations as one launch per matrix with the same plan, so
its results are also bit-identical to the single-matrix kernels (mode 0
wavefront tiles and mode 2 test tiles), with or without a persistent grid
and with or without graph replay."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _long_rows():
    a = synth.uniform_random(40, 30000, 3.0, seed=71)
    rows = np.repeat(np.arange(40), a.row_lengths())
    r2 = np.repeat(np.array([5, 6, 7, 8]), 30000)
    c2 = np.tile(np.arange(30000), 4)
    return synth._from_keys(40, 30000, np.concatenate([rows, r2]), np.concatenate([a.colidx, c2]),
                            synth.rng_for(72))


def population():
    """(matrix, shape) pairs: uneven sizes, all six shapes, an empty matrix,
    a matrix with no entries, intervals longer than a tile."""
    mats = [synth.batched_matrix(i, 2_000, 40_000) for i in range(6)]
    mats += [synth.stencil27(9), synth.powerlaw(3000, 2500, seed=3), _long_rows(),
             synth.from_dense(np.array([[1.5, 0, 2.0]])),
             synth.CSR(17, 5, np.zeros(18, np.int32), np.zeros(0, np.int32), np.zeros(0)),
             synth.fem_blocks(400, 6, 4.0, 9, seed=8)]
    shapes = [spc.SHAPES[i % 6] for i in range(len(mats))]
    return mats, shapes


_pop = None


def pop():
    global _pop
    if _pop is None:
        _pop = population()
    return _pop


def build(dtype):
    mats, shapes = pop()
    Bs, xs, ys, refs = [], [], [], []
    for k, (A, (r, c)) in enumerate(zip(mats, shapes)):
        A = A.astype(NP[dtype])
        Bs.append(spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values).to(dtype), A.n_cols))
        x = synth.dense_vector(A.n_cols, 80 + k).astype(NP[dtype])
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.full((A.n_rows,), 7.0, dtype=dtype, device="cuda"))
        refs.append(oracle.csr_spmv(A, x))
    return Bs, xs, ys, refs


@pytest.mark.parametrize("kq", [2, 4, 6, 8])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_matches_oracle_and_single_launches(dtype, kq):
    say(f"[batched] {dtype} kq={kq}")
    Bs, xs, ys, refs = build(dtype)
    batch = spc.Batch(Bs, wave_chunks=kq).set_vectors(xs, ys)
    info = batch.info()
    assert info["n_tiles"] == sum(B.plan(0, 0, 0, kq).info()["n_tiles"] for B in Bs)
    assert info["n_long"] >= 1
    batch.run()
    torch.cuda.synchronize()
    first = [y.clone() for y in ys]
    for y, (y_ref, s) in zip(ys, refs):
        got = y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - y_ref) <= TOL[dtype] * s)
    # one launch per matrix with the same tiles: the same bits
    for B, x, y0 in zip(Bs, xs, first):
        assert torch.equal(spc.spmv(B, x, plan=B.plan(0, 0, 0, kq)), y0)
    # a persistent grid and graph replays give the same bits
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for grid, graph in [(7, False), (0, True), (0, True), (3, True), (3, True)]:
            for y in ys:
                y.fill_(-1.0)
            batch.run(grid_blocks=grid, use_graph=graph)
            s.synchronize()
            for y, y0 in zip(ys, first):
                assert torch.equal(y, y0)


def test_batched_accumulate():
    say("[batched] accumulate")
    Bs, xs, ys, refs = build(torch.float64)
    y0 = [y.clone() for y in ys]
    spc.Batch(Bs).set_vectors(xs, ys).run(accumulate=True)
    torch.cuda.synchronize()
    for y, base, (y_ref, s) in zip(ys, y0, refs):
        got = y.cpu().numpy()
        assert np.all(np.abs(got - (base.cpu().numpy() + y_ref)) <= 1e-13 * (s + 7.0))


def test_batch_refuses_bad_arguments():
    mats, shapes = pop()
    A = mats[0]
    B64 = spc.csr_to_beta(1, 8, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    B32 = spc.csr_to_beta(2, 4, A.rowptr, A.colidx, torch.from_numpy(A.values).float(), A.n_cols)
    with pytest.raises(spc.SpcError):
        spc.Batch([B64, B32])
    b = spc.Batch([B64])
    with pytest.raises(spc.SpcError):
        b.run()  # vectors not set
    with pytest.raises(ValueError):
        b.set_vectors([torch.zeros(3, dtype=torch.float64, device="cuda")],
                      [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")])
    B44 = spc.csr_to_beta(4, 4, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    for params, mats_ in [({"mode": 1}, [B64]), ({"mode": 2}, [B44]), ({"mode": 4}, [B44]), ({"mode": 5}, [B64]),
                          ({"mode": 0, "pipeline": 1}, [B64]), ({"mode": 0, "wave_tiles": 2}, [B64])]:
        with pytest.raises(spc.SpcError):
            spc.Batch(mats_, params=params)
    with pytest.raises(ValueError):
        spc.Batch([B64, B44], params=[{"mode": 0}])
    # the shape-switching kernel needs one mode-0 chunk count
    mixed = spc.Batch([B64, B44], params=[{"mode": 2, "wave_chunks": 4}, {"mode": 0, "wave_chunks": 4}])
    assert mixed.info()["n_groups"] == 2
    with pytest.raises(spc.SpcError):
        mixed.set_kernel(True)
    with pytest.raises(spc.SpcError):
        spc.Batch([B64, B44], params=[{"mode": 0, "wave_chunks": 2}, {"mode": 0, "wave_chunks": 4}]).set_kernel(True)
    with pytest.raises(spc.SpcError):
        spc.Batch([B64, B44], params=[{"mode": 4, "wave_chunks": 4}, {"mode": 3, "wave_chunks": 4}]).set_kernel(True)


def _mixed_params(shapes):
    """Per matrix: test tiles (mode 2) for every other one-byte-mask matrix,
    value lanes (mode 4) for the other beta(1,8) ones, block-row lanes
    (mode 3) for every third of the rest, wavefront tiles (mode 0)
    otherwise; chunk counts cycling over 2, 4, 6, 8."""
    out = []
    for k, (r, c) in enumerate(shapes):
        if r * c == 8 and k % 2 == 0:
            mode = 2
        elif (r, c) == (1, 8):
            mode = 4
        elif k % 3 == 1:
            mode = 3
        else:
            mode = 0
        out.append({"mode": mode, "wave_chunks": (2, 4, 6, 8)[k % 4]})
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_grouped_batch_mixed_modes_and_chunks(dtype):
    say(f"[batched] grouped, mixed modes {dtype}")
    mats, _ = pop()
    # more one-byte-mask matrices than the six-shape cycle gives
    shapes = [spc.SHAPES[(0, 1, 0, 1, 2, 3, 4, 5, 0, 1, 1, 0)[k]] for k in range(len(mats))]
    Bs, xs, ys, refs = [], [], [], []
    for k, (A, (r, c)) in enumerate(zip(mats, shapes)):
        A = A.astype(NP[dtype])
        Bs.append(spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values).to(dtype), A.n_cols))
        x = synth.dense_vector(A.n_cols, 95 + k).astype(NP[dtype])
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.full((A.n_rows,), 7.0, dtype=dtype, device="cuda"))
        refs.append(oracle.csr_spmv(A, x))
    params = _mixed_params(shapes)
    assert {p["mode"] for p in params} == {0, 2, 3, 4}
    batch = spc.Batch(Bs, params=params).set_vectors(xs, ys)
    info = batch.info()
    keys = {(p["mode"], shapes[k], p["wave_chunks"]) for k, p in enumerate(params)}
    assert info["n_groups"] == len(keys) and info["single_shape"] == -1
    plans = [spc.plan_from(B, p) for B, p in zip(Bs, params)]
    assert info["n_tiles"] == sum(P.info()["n_tiles"] for P in plans)
    batch.run()
    torch.cuda.synchronize()
    first = [y.clone() for y in ys]
    for y, (y_ref, s) in zip(ys, refs):
        got = y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - y_ref) <= TOL[dtype] * s)
    for B, x, y0, P in zip(Bs, xs, first, plans):
        assert torch.equal(spc.spmv(B, x, plan=P), y0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for grid, graph in [(5, False), (0, True), (0, True), (2, True), (2, True)]:
            for y in ys:
                y.fill_(-1.0)
            batch.run(grid_blocks=grid, use_graph=graph)
            s.synchronize()
            for y, y0 in zip(ys, first):
                assert torch.equal(y, y0)


@pytest.mark.parametrize("shape", [0, 1, 5])
def test_single_shape_kernel_equals_general_kernel(shape):
    say(f"[batched] single shape {shape}")
    mats, _ = pop()
    r, c = spc.SHAPES[shape]
    Bs, xs, ys, refs = [], [], [], []
    for k, A in enumerate(mats):
        Bs.append(spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols))
        x = synth.dense_vector(A.n_cols, 90 + k)
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.zeros(A.n_rows, dtype=torch.float64, device="cuda"))
        refs.append(oracle.csr_spmv(A, x))
    batch = spc.Batch(Bs).set_vectors(xs, ys)
    assert batch.info()["single_shape"] == shape
    batch.run()
    torch.cuda.synchronize()
    fixed = [y.clone() for y in ys]
    for y, (y_ref, s) in zip(fixed, refs):
        assert np.all(np.abs(y.cpu().numpy() - y_ref) <= 1e-13 * s)
    batch.set_kernel(True).run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ys, fixed))
    for B, x, y0 in zip(Bs, xs, fixed):
        # without parameters the batch plans each matrix with its default
        assert torch.equal(spc.spmv(B, x, plan=B.default_plan()), y0)
