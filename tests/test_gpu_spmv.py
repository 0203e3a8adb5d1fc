"""GPU parity of conversion and SpMV against the CPU oracle.

Bars: conversion and decoding bit-exact; SpMV per row |y - y_ref| <= 1e-13 *
sum_j |a_ij x_j| (FP64) and <= 2e-6 * sum_j |a_ij x_j| (FP32, with y_ref and
the bound computed in FP64 from the FP32-rounded inputs); integer-valued
inputs bit-exact.
"""
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


def _empty_rows():
    A = synth.uniform_random(3000, 3000, 3.0, seed=4)
    lens = A.row_lengths()
    keep = np.ones(A.n_rows, bool)
    keep[100:1900] = False  # 1800 empty rows in a run
    rows = np.repeat(np.arange(A.n_rows), lens)
    m = keep[rows]
    counts = np.bincount(rows[m], minlength=A.n_rows)
    rp = np.zeros(A.n_rows + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    return synth.CSR(A.n_rows, A.n_cols, rp, A.colidx[m], A.values[m])


def _dense_rows():
    # a few rows far longer than a tile (the long path), among short rows
    a = synth.uniform_random(600, 9000, 4.0, seed=5)
    rows = np.repeat(np.arange(600), a.row_lengths())
    cols = a.colidx.astype(np.int64)
    extra_r = np.repeat(np.array([3, 4, 5, 250, 599]), 9000)
    extra_c = np.tile(np.arange(9000), 5)
    R = np.concatenate([rows, extra_r])
    Cc = np.concatenate([cols, extra_c])
    return synth._from_keys(600, 9000, R, Cc, synth.rng_for(55))


CASES = {
    "band4096": lambda: synth.band_plus_uniform(4096, seed=0),
    "stencil13": lambda: synth.stencil27(13),                  # 2197 rows: ragged for every r
    "stencil16": lambda: synth.stencil27(16),
    "powerlaw": lambda: synth.powerlaw(3001, 3001, seed=2),     # rows up to 2000 entries
    "fem3": lambda: synth.fem_blocks(700, 3, 6.0, 20, seed=3),
    "fem6": lambda: synth.fem_blocks(300, 6, 5.0, 10, seed=3),
    "banded": lambda: synth.banded(2500, 64, 0.4, seed=6),
    "uniform": lambda: synth.uniform_random(5000, 4000, 12.0, seed=7),
    "wide": lambda: synth.uniform_random(97, 20000, 300.0, seed=8),
    "tall": lambda: synth.uniform_random(20000, 37, 3.0, seed=9),
    "empty_rows": _empty_rows,
    "dense_rows": _dense_rows,
    "tiny1x1": lambda: synth.from_dense(np.array([[2.5]])),
    "tiny3x5": lambda: synth.random_small(3, 5, 0.6, seed=10),
    "all_empty": lambda: synth.CSR(10, 10, np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0)),
    # one entry per row: tiles reach their cap of (interval, block row) pairs
    # (127 intervals for r = 1, 128 pairs otherwise), so every lane takes two
    "diagonal": lambda: synth.from_keys_sorted(6007, 6007, np.arange(6007), np.arange(6007), 11),
    # two entries per row, 8 columns apart: one value per beta(1,8) block
    "two_per_row": lambda: synth.from_keys_sorted(
        5003, 5003, np.repeat(np.arange(5003), 2),
        np.stack([np.arange(5003), (np.arange(5003) + 8) % 5003], axis=1).reshape(-1), 12),
}

_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


def to_beta(A, r, c, dtype):
    return spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values).to(dtype), A.n_cols)


def check_rows(y, y_ref, s_ref, tol, label):
    err = np.abs(y.astype(np.float64) - y_ref)
    bad = np.flatnonzero(~(err <= tol * s_ref))
    assert bad.size == 0, (f"{label}: {bad.size} rows out of bound, e.g. row {bad[0]}: "
                           f"y={y[bad[0]]!r} ref={y_ref[bad[0]]!r} bound={tol * s_ref[bad[0]]!r}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_conversion_bit_exact(name, rc):
    r, c = rc
    A = case(name)
    say(f"[conv] {name} beta{rc} n={A.n_rows} nnz={A.nnz}")
    ref = oracle.csr_to_beta(A, r, c)
    B = to_beta(A, r, c, torch.float64)
    assert B.n_blocks == ref.n_blocks
    assert np.array_equal(B.block_rowptr.cpu().numpy(), ref.block_rowptr)
    assert np.array_equal(B.block_colidx.cpu().numpy(), ref.block_colidx)
    mb = B.block_masks.cpu().numpy()
    assert np.array_equal(mb[:ref.n_blocks * r * c // 8], ref.mask_bytes())
    assert not mb[ref.n_blocks * r * c // 8:].any()  # padding zeroed
    assert np.array_equal(B.values.cpu().numpy().view(np.uint64), ref.values.view(np.uint64))
    # device decoding returns the CSR arrays bit for bit
    rp, ci, v = spc.beta_to_csr(B)
    assert np.array_equal(rp.cpu().numpy(), A.rowptr)
    assert np.array_equal(ci.cpu().numpy(), A.colidx)
    assert np.array_equal(v.cpu().numpy().view(np.uint64), A.values.view(np.uint64))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_conversion_values_aligned_and_not(rc, dtype):
    """Conversion into a values output on a 16-byte boundary and into one
    that is not (one element past it): both give the oracle's values bit for
    bit, and nothing outside the output is written."""
    from paper_1801_01134_amd import _binding as bb
    r, c = rc
    npd = np.float64 if dtype == torch.float64 else np.float32
    ubits = np.uint64 if dtype == torch.float64 else np.uint32
    for name in ("powerlaw", "fem6", "empty_rows"):
        A = case(name).astype(npd)
        say(f"[conv values] {name} beta{rc} {dtype}")
        ref = oracle.csr_to_beta(A, r, c)
        B = to_beta(A, r, c, dtype)                    # aligned output
        assert np.array_equal(B.values.cpu().numpy().view(ubits), ref.values.view(ubits))
        # the same conversion into an output one element past a 16-byte boundary
        rp = torch.from_numpy(A.rowptr).cuda()
        ci = torch.from_numpy(A.colidx if A.nnz else np.zeros(1, np.int32)).cuda()
        v = torch.from_numpy(A.values if A.nnz else np.zeros(1, npd)).cuda()
        store = torch.zeros(max(A.nnz, 1) + 4, dtype=dtype, device="cuda")
        vout = store[1:1 + max(A.nnz, 1)]
        bcol = torch.zeros(max(B.n_blocks, 1), dtype=torch.int32, device="cuda")
        masks = torch.zeros(B.block_masks.numel(), dtype=torch.uint8, device="cuda")
        bb.check(spc.lib().spc_csr_to_beta(r, c, bb._dtype_code(dtype), A.n_rows, A.n_cols, bb._ptr(rp),
                                           bb._ptr(ci), bb._ptr(v), bb._ptr(B.block_rowptr), bb._ptr(bcol),
                                           bb._ptr(masks), bb._ptr(vout), bb.stream_ptr()))
        torch.cuda.synchronize()
        assert np.array_equal(vout[:A.nnz].cpu().numpy().view(ubits), ref.values.view(ubits))
        assert torch.equal(bcol[:B.n_blocks], B.block_colidx) and torch.equal(masks, B.block_masks)
        assert store[0].item() == 0 and torch.all(store[1 + max(A.nnz, 1):] == 0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_spmv_parity(name, rc, dtype):
    r, c = rc
    A = case(name).astype(NP[dtype])
    say(f"[spmv] {name} beta{rc} {dtype} n={A.n_rows} nnz={A.nnz}")
    x = synth.dense_vector(A.n_cols, 21, dtype=NP[dtype])
    y_ref, s_ref = oracle.csr_spmv(A, x)
    B = to_beta(A, r, c, dtype)
    xd = torch.from_numpy(x).cuda()
    y = spc.spmv(B, xd).cpu().numpy()
    check_rows(y, y_ref, s_ref, TOL[dtype], f"{name} beta{rc}")
    # accumulate: y0 + A x; rows without entries keep y0 exactly
    y0 = synth.dense_vector(A.n_rows, 22, dtype=NP[dtype])
    ya = spc.spmv(B, xd, torch.from_numpy(y0.copy()).cuda(), accumulate=True).cpu().numpy()
    s_acc = s_ref + np.abs(y0.astype(np.float64))
    check_rows(ya, y_ref + y0.astype(np.float64), s_acc, TOL[dtype], f"{name} beta{rc} accumulate")
    empty = A.row_lengths() == 0
    assert np.array_equal(ya[empty], y0[empty])
    if empty.any():
        assert np.all(y[empty] == 0) and not np.signbit(y[empty]).any()


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("mode,tile_bits,chunks,order", [
    (0, 0, 2, 0), (0, 0, 4, 1), (0, 0, 6, 0), (0, 0, 8, 1),
    (1, 1024, 0, 0), (1, 2048, 0, 1), (1, 3072, 0, 0), (1, 4032, 0, 1)])
@pytest.mark.parametrize("name", ["powerlaw", "stencil13", "fem6", "dense_rows", "empty_rows"])
def test_plan_variants_and_determinism(rc, mode, tile_bits, chunks, order, name):
    r, c = rc
    say(f"[plan] {name} beta{rc} mode={mode} tile_bits={tile_bits} chunks={chunks} order={order}")
    A = case(name)
    x = synth.dense_vector(A.n_cols, 23)
    y_ref, s_ref = oracle.csr_spmv(A, x)
    B = to_beta(A, r, c, torch.float64)
    P = B.plan(tile_bits, order, mode, chunks)
    info = P.info()
    want_bits = tile_bits if mode == 1 else (64 * chunks - 1) * 2
    assert info["tile_bits"] == want_bits and info["n_tiles"] > 0
    xd = torch.from_numpy(x).cuda()
    y1 = spc.spmv(B, xd, plan=P)
    y2 = spc.spmv(B, xd, plan=P)
    check_rows(y1.cpu().numpy(), y_ref, s_ref, 1e-13, f"beta{rc} tb{tile_bits}")
    assert torch.equal(y1.view(torch.int64), y2.view(torch.int64))


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_integer_inputs_bit_exact(rc, dtype):
    r, c = rc
    say(f"[int] beta{rc} {dtype}")
    A = synth.powerlaw(1500, 1500, seed=11)
    A.values = np.round(A.values * 16)      # |a| <= 16
    x = np.round(synth.dense_vector(A.n_cols, 24) * 16)
    y_ref, _ = oracle.csr_spmv(A, x)        # exact: every partial sum is an integer < 2^24
    B = to_beta(A.astype(NP[dtype]), r, c, dtype)
    y = spc.spmv(B, torch.from_numpy(x.astype(NP[dtype])).cuda()).cpu().numpy()
    assert np.array_equal(y.astype(np.float64), y_ref)


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_nonfinite_x_under_unset_bits_does_not_leak(rc):
    r, c = rc
    say(f"[inf] beta{rc}")
    A = synth.random_small(64, 64, 0.15, seed=12)
    j = 9
    x = synth.dense_vector(64, 25)
    x[j] = np.inf
    B = to_beta(A, r, c, torch.float64)
    y = spc.spmv(B, torch.from_numpy(x).cuda()).cpu().numpy()
    has_j = np.zeros(A.n_rows, bool)
    for i in range(A.n_rows):
        has_j[i] = j in A.colidx[A.rowptr[i]:A.rowptr[i + 1]]
    assert np.all(np.isfinite(y[~has_j]))
    assert not np.any(np.isfinite(y[has_j]))


def test_invalid_csr_is_refused():
    say("[err] invalid csr")
    A = synth.random_small(20, 20, 0.3, seed=13)
    ci = A.colidx.copy()
    i = int(np.flatnonzero(np.diff(A.rowptr) >= 2)[0])
    p = A.rowptr[i]
    ci[p], ci[p + 1] = ci[p + 1], ci[p]                         # unsorted row
    with pytest.raises(spc.SpcError) as e:
        spc.csr_to_beta(1, 8, A.rowptr, ci, A.values, A.n_cols)
    assert e.value.code == -3
    ci2 = A.colidx.copy()
    ci2[-1] = 20                                                # out of range
    with pytest.raises(spc.SpcError) as e:
        spc.csr_to_beta(2, 4, A.rowptr, ci2, A.values, A.n_cols)
    assert e.value.code == -4
    rp = A.rowptr.copy()
    rp[5] = rp[6] + 1                                           # decreasing
    with pytest.raises(spc.SpcError) as e:
        spc.csr_to_beta(4, 4, rp, A.colidx, A.values, A.n_cols)
    assert e.value.code == -4


def test_corrupt_view_is_refused_by_plan():
    say("[err] corrupt view")
    A = synth.random_small(40, 40, 0.3, seed=14)
    B = to_beta(A, 1, 8, torch.float64)
    B.block_colidx[0] = 40                                      # block runs past n_cols
    with pytest.raises(spc.SpcError) as e:
        B.plan()
    assert e.value.code == -4
    B2 = to_beta(A, 1, 8, torch.float64)
    B2.values = B2.values[:-1].clone()                          # nnz disagrees with masks
    with pytest.raises(spc.SpcError):
        B2.plan()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_values_not_16_byte_aligned(dtype):
    say(f"[align] {dtype}")
    A = case("fem3").astype(NP[dtype])
    x = synth.dense_vector(A.n_cols, 26, dtype=NP[dtype])
    y_ref, s_ref = oracle.csr_spmv(A, x)
    B = to_beta(A, 2, 4, dtype)
    buf = torch.empty(B.nnz + 1, dtype=dtype, device="cuda")
    buf[1:] = B.values
    B.values = buf[1:]                      # element-aligned, not 16-byte aligned
    assert B.values.data_ptr() % 16 != 0
    y = spc.spmv(B, torch.from_numpy(x).cuda()).cpu().numpy()
    check_rows(y, y_ref, s_ref, TOL[dtype], "misaligned values")


def test_empty_matrix_with_null_masks_pointer():
    # a matrix without blocks may come with no masks array at all
    say("[null masks] all-empty matrix, view without a masks pointer")
    import ctypes
    from paper_1801_01134_amd import _binding as Bd
    A = case("all_empty")
    B = to_beta(A, 1, 8, torch.float64)
    v = B.view()
    v.block_masks = None
    h = ctypes.c_void_p()
    Bd.check(Bd.lib().spc_plan_create(ctypes.byref(v), None, ctypes.byref(h), Bd.stream_ptr()))
    x = torch.ones(A.n_cols, dtype=torch.float64, device="cuda")
    y = torch.full((A.n_rows,), 7.0, dtype=torch.float64, device="cuda")
    Bd.check(Bd.lib().spc_spmv_beta(ctypes.byref(v), h, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), 0, Bd.stream_ptr()))
    assert torch.all(y == 0)
    Bd.lib().spc_plan_destroy(h)


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("chunks", [2, 4, 6, 8])
@pytest.mark.parametrize("grid", [1, 3, 40])
def test_pipelined_equals_one_tile_per_wave(rc, dtype, chunks, grid):
    """Persistent wavefronts that prefetch their next tile (capped at `grid`
    workgroups, so every wavefront walks many tiles) compute the same tiles
    in the same order of operations: identical bits, also with accumulate."""
    r, c = rc
    say(f"[pipe] beta{rc} {dtype} chunks={chunks} grid={grid}")
    for name in ("powerlaw", "dense_rows", "empty_rows", "stencil13"):
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 25).astype(NP[dtype])
        B = to_beta(A, r, c, dtype)
        xd = torch.from_numpy(x).cuda()
        y0 = spc.spmv(B, xd, plan=B.plan(0, 0, 0, chunks))
        P = B.plan(0, 0, 0, chunks, grid + 1)
        y1 = spc.spmv(B, xd, plan=P)
        assert torch.equal(y0, y1), name
        base = torch.from_numpy(synth.dense_vector(A.n_rows, 26).astype(NP[dtype])).cuda()
        ya = base.clone()
        yb = base.clone()
        spc.spmv(B, xd, ya, accumulate=True, plan=B.plan(0, 0, 0, chunks))
        spc.spmv(B, xd, yb, accumulate=True, plan=P)
        assert torch.equal(ya, yb), name
    y_ref, s_ref = oracle.csr_spmv(A, x)
    check_rows(y1.cpu().numpy().astype(np.float64), y_ref, s_ref, TOL[dtype], f"pipe beta{rc}")


def _oracle_check(B, ref, r, c):
    assert B.n_blocks == ref.n_blocks
    assert np.array_equal(B.block_rowptr.cpu().numpy(), ref.block_rowptr)
    assert np.array_equal(B.block_colidx.cpu().numpy(), ref.block_colidx)
    assert np.array_equal(B.block_masks.cpu().numpy()[:ref.n_blocks * r * c // 8], ref.mask_bytes())
    assert np.array_equal(B.values.cpu().numpy().view(np.uint64), ref.values.view(np.uint64))


@pytest.mark.parametrize("offset", [1, 2, 3])
@pytest.mark.parametrize("name", ["powerlaw", "stencil13", "dense_rows", "tiny3x5"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_colidx_not_16_byte_aligned(name, rc, offset):
    """Columns handed over at an address 4, 8 or 12 bytes past a 16-byte
    boundary: conversion and features read them in 16-byte windows from the
    boundary below, and give the same results."""
    r, c = rc
    A = case(name)
    say(f"[colidx+{offset}] {name} beta{rc}")
    big = torch.zeros(A.nnz + 8, dtype=torch.int32, device="cuda")
    big[offset:offset + A.nnz] = torch.from_numpy(A.colidx).cuda()
    ci = big[offset:offset + A.nnz]
    assert ci.data_ptr() % 16 == 4 * offset
    rp = torch.from_numpy(A.rowptr).cuda()
    B = spc.csr_to_beta(r, c, rp, ci, torch.from_numpy(A.values), A.n_cols)
    _oracle_check(B, oracle.csr_to_beta(A, r, c), r, c)
    f1, nb1 = spc.matrix_features(rp, ci, A.n_cols)
    f0, nb0 = spc.matrix_features(rp, torch.from_numpy(A.colidx).cuda(), A.n_cols)
    assert np.array_equal(nb1, nb0) and np.array_equal(f1.view(np.uint32), f0.view(np.uint32))


@pytest.mark.parametrize("name", ["powerlaw", "stencil13", "fem6", "two_per_row"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_block_columns_not_16_byte_aligned(name, rc):
    """A caller's block-column array 4 bytes past a 16-byte boundary: the
    block columns are then stored one by one, with the same result."""
    import ctypes
    from paper_1801_01134_amd import _binding as Bd
    r, c = rc
    A = case(name)
    say(f"[bcol+4] {name} beta{rc}")
    ref = oracle.csr_to_beta(A, r, c)
    rp = torch.from_numpy(A.rowptr).cuda()
    ci = torch.from_numpy(A.colidx).cuda()
    v = torch.from_numpy(A.values).cuda()
    n_int = (A.n_rows + r - 1) // r
    brow = torch.empty(n_int + 1, dtype=torch.int32, device="cuda")
    nb = ctypes.c_int64()
    L, s = Bd.lib(), Bd.stream_ptr()
    Bd.check(L.spc_beta_count(r, c, A.n_rows, A.n_cols, Bd._ptr(rp), Bd._ptr(ci), Bd._ptr(brow),
                              ctypes.byref(nb), s))
    nb = nb.value
    bcol_big = torch.full((nb + 8,), -7, dtype=torch.int32, device="cuda")
    bcol = bcol_big[1:1 + nb]
    assert bcol.data_ptr() % 16 == 4
    masks = torch.empty(Bd.mask_bytes(r, c, nb), dtype=torch.uint8, device="cuda")
    vout = torch.empty_like(v)
    Bd.check(L.spc_csr_to_beta(r, c, Bd._dtype_code(v.dtype), A.n_rows, A.n_cols, Bd._ptr(rp), Bd._ptr(ci),
                               Bd._ptr(v), Bd._ptr(brow), Bd._ptr(bcol), Bd._ptr(masks), Bd._ptr(vout), s))
    torch.cuda.synchronize()
    assert np.array_equal(bcol.cpu().numpy(), ref.block_colidx)
    # nothing written outside the caller's range
    assert int(bcol_big[0]) == -7 and bool((bcol_big[1 + nb:] == -7).all())
    assert np.array_equal(masks.cpu().numpy()[:nb * r * c // 8], ref.mask_bytes())
    assert np.array_equal(vout.cpu().numpy().view(np.uint64), ref.values.view(np.uint64))


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_null_plan_through_the_abi(rc, dtype):
    """spc_spmv_beta and spc_spmm_beta with plan = NULL build the library's
    default plan for the call: same result as that plan passed explicitly,
    within the oracle's bound, with accumulate too."""
    import ctypes
    from paper_1801_01134_amd import _binding as Bd
    r, c = rc
    L, s = Bd.lib(), Bd.stream_ptr()
    for name in ("powerlaw", "empty_rows", "stencil13"):
        say(f"[null plan] {name} beta{rc} {dtype}")
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 71).astype(NP[dtype])
        y_ref, s_ref = oracle.csr_spmv(A, x)
        B = to_beta(A, r, c, dtype)
        v = B.view()
        xd = torch.from_numpy(x).cuda()
        y = torch.full((A.n_rows,), 3.0, dtype=dtype, device="cuda")
        Bd.check(L.spc_spmv_beta(ctypes.byref(v), None, Bd._ptr(xd), Bd._ptr(y), 0, s))
        check_rows(y.cpu().numpy().astype(np.float64), y_ref, s_ref, TOL[dtype], f"null plan beta{rc}")
        assert torch.equal(y, spc.spmv(B, xd, plan=B.default_plan()))
        base = torch.from_numpy(synth.dense_vector(A.n_rows, 72).astype(NP[dtype])).cuda()
        ya = base.clone()
        Bd.check(L.spc_spmv_beta(ctypes.byref(v), None, Bd._ptr(xd), Bd._ptr(ya), 1, s))
        yb = base.clone()
        spc.spmv(B, xd, yb, accumulate=True, plan=B.default_plan())
        assert torch.equal(ya, yb)
        X = torch.from_numpy(synth.dense_block(A.n_cols, 4, 73, dtype=NP[dtype])).cuda()
        Y = torch.empty((A.n_rows, 4), dtype=dtype, device="cuda")
        Bd.check(L.spc_spmm_beta(ctypes.byref(v), None, 4, Bd._ptr(X), 4, Bd._ptr(Y), 4, 0, s))
        assert torch.equal(Y, spc.spmm(B, X, plan=B.default_plan()))


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("chunks", [2, 4, 6, 8])
def test_two_tiles_per_wavefront_same_bits(rc, dtype, chunks):
    """wave_tiles = 2 (two consecutive tiles per wavefront, the second staged
    in registers) runs the same tiles in the same order of operations: the
    same bits as one tile per wavefront, with accumulate too, and odd tile
    counts and long intervals among them."""
    r, c = rc
    say(f"[pair] beta{rc} {dtype} chunks={chunks}")
    for name in ("powerlaw", "dense_rows", "empty_rows", "stencil13", "diagonal", "tiny3x5"):
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 27).astype(NP[dtype])
        B = to_beta(A, r, c, dtype)
        xd = torch.from_numpy(x).cuda()
        y0 = spc.spmv(B, xd, plan=B.plan(0, 0, 0, chunks))
        for order in (0, 1):
            P = B.plan(0, order, 0, chunks, 0, 0, 2)
            assert torch.equal(spc.spmv(B, xd, plan=P), y0), (name, order)
        base = torch.from_numpy(synth.dense_vector(A.n_rows, 28).astype(NP[dtype])).cuda()
        ya, yb = base.clone(), base.clone()
        spc.spmv(B, xd, ya, accumulate=True, plan=B.plan(0, 0, 0, chunks))
        spc.spmv(B, xd, yb, accumulate=True, plan=B.plan(0, 0, 0, chunks, 0, 0, 2))
        assert torch.equal(ya, yb), name
    y_ref, s_ref = oracle.csr_spmv(A, x)
    check_rows(y0.cpu().numpy().astype(np.float64), y_ref, s_ref, TOL[dtype], f"pair beta{rc}")


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("chunks", [2, 4, 6, 8])
def test_block_row_lanes_parity(rc, dtype, chunks):
    """Mode 3 (lane = block row, walking its set bits) on every case against
    the oracle, y = A x and y += A x (rows without entries keep y), capped
    and uncapped launches giving the same bits, and repeated calls
    reproducing them."""
    r, c = rc
    say(f"[brow] beta{rc} {dtype} chunks={chunks}")
    for name in CASES:
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 29, dtype=NP[dtype])
        y_ref, s_ref = oracle.csr_spmv(A, x)
        B = to_beta(A, r, c, dtype)
        xd = torch.from_numpy(x).cuda()
        P = B.plan(0, 0, 3, chunks)
        assert P.info()["tile_bits"] == (64 * chunks - 1) * (16 // NP[dtype]().itemsize)
        y = spc.spmv(B, xd, plan=P)
        check_rows(y.cpu().numpy(), y_ref, s_ref, TOL[dtype], f"brow {name} beta{rc}")
        assert torch.equal(spc.spmv(B, xd, plan=P), y), name
        assert torch.equal(spc.spmv(B, xd, plan=B.plan(0, 1, 3, chunks, 0, 3)), y), name
        y0 = synth.dense_vector(A.n_rows, 30, dtype=NP[dtype])
        ya = spc.spmv(B, xd, torch.from_numpy(y0.copy()).cuda(), accumulate=True, plan=P).cpu().numpy()
        check_rows(ya, y_ref + y0.astype(np.float64), s_ref + np.abs(y0.astype(np.float64)), TOL[dtype],
                   f"brow {name} beta{rc} accumulate")
        empty = A.row_lengths() == 0
        assert np.array_equal(ya[empty], y0[empty])
        if empty.any():
            yh = y.cpu().numpy()
            assert np.all(yh[empty] == 0) and not np.signbit(yh[empty]).any()


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_block_row_lanes_integers_and_nonfinite(rc, dtype):
    """Mode 3: integer-valued inputs give exact sums; an Inf in x reaches
    exactly the rows that store an entry in its column."""
    r, c = rc
    say(f"[brow-int] beta{rc} {dtype}")
    A = synth.powerlaw(1500, 1500, seed=11)
    A.values = np.round(A.values * 16)
    x = np.round(synth.dense_vector(A.n_cols, 24) * 16)
    y_ref, _ = oracle.csr_spmv(A, x)
    B = to_beta(A.astype(NP[dtype]), r, c, dtype)
    for chunks in (2, 8):
        y = spc.spmv(B, torch.from_numpy(x.astype(NP[dtype])).cuda(), plan=B.plan(0, 0, 3, chunks))
        assert np.array_equal(y.cpu().numpy().astype(np.float64), y_ref)
    S = synth.random_small(64, 64, 0.15, seed=12)
    j = 9
    xs = synth.dense_vector(64, 25)
    xs[j] = np.inf
    Bs = to_beta(S.astype(NP[dtype]), r, c, dtype)
    ys = spc.spmv(Bs, torch.from_numpy(xs.astype(NP[dtype])).cuda(), plan=Bs.plan(0, 0, 3, 4)).cpu().numpy()
    has_j = np.array([j in S.colidx[S.rowptr[i]:S.rowptr[i + 1]] for i in range(S.n_rows)])
    assert np.all(np.isfinite(ys[~has_j])) and not np.any(np.isfinite(ys[has_j]))


def test_block_row_lanes_refusals():
    """Mode 3 takes neither two tiles per wavefront nor the pipeline; SpMM
    and CG refuse its plans; mode 5 does not exist."""
    say("[brow-refuse]")
    A = case("stencil13")
    B = to_beta(A, 2, 4, torch.float64)
    for bad in (dict(mode=3, wave_chunks=4, wave_tiles=2), dict(mode=3, wave_chunks=4, pipeline=1),
                dict(mode=5, wave_chunks=4)):
        with pytest.raises(spc.SpcError):
            spc.plan_from(B, bad)
    P = B.plan(0, 0, 3, 4)
    X = torch.from_numpy(synth.dense_block(A.n_cols, 4, 31)).cuda()
    with pytest.raises(spc.SpcError):
        spc.spmm(B, X, plan=P)
    with pytest.raises(spc.SpcError):
        spc.cg(B, X, rel_tol=1e-6, max_iter=5, check_every=5, plan=P)


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_block_row_lanes_tiles_and_unaligned_values(rc, dtype):
    """Mode 3 tiles hold up to the buffer's values and the shape's block cap
    (more blocks than a mode 0 tile where blocks are sparse); with values
    that are not 16-byte aligned the same tiles run as 4032-bit workgroup
    tiles, still matching the oracle."""
    r, c = rc
    say(f"[brow-tiles] beta{rc} {dtype}")
    esz = NP[dtype]().itemsize
    for name in ("stencil16", "uniform", "dense_rows", "diagonal"):
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 32, dtype=NP[dtype])
        y_ref, s_ref = oracle.csr_spmv(A, x)
        B = to_beta(A, r, c, dtype)
        for chunks in (2, 8):
            P3, P0 = B.plan(0, 0, 3, chunks), B.plan(0, 0, 0, chunks)
            vcap = (64 * chunks - 1) * (16 // esz)
            # value-sized tiles are never more numerous than bit-sized ones
            assert P3.info()["n_tiles"] <= P0.info()["n_tiles"], name
            assert P3.info()["tile_bits"] == vcap
            y = spc.spmv(B, torch.from_numpy(x).cuda(), plan=P3).cpu().numpy()
            check_rows(y, y_ref, s_ref, TOL[dtype], f"brow {name} chunks={chunks}")
        buf = torch.empty(B.nnz + 1, dtype=dtype, device="cuda")
        buf[1:] = B.values
        Bu = to_beta(A, r, c, dtype)
        Bu.values = buf[1:]
        assert Bu.values.data_ptr() % 16 != 0
        for chunks in (2, 8):
            y = spc.spmv(Bu, torch.from_numpy(x).cuda(), plan=Bu.plan(0, 0, 3, chunks)).cpu().numpy()
            check_rows(y, y_ref, s_ref, TOL[dtype], f"brow unaligned {name} chunks={chunks}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("chunks", [2, 4, 6, 8])
def test_value_lanes_parity(dtype, chunks):
    """Mode 4 (beta(1,8), one lane per stored value) on every case against
    the oracle: y = A x and y += A x (rows without entries keep y), capped
    launches, repeated calls giving the same bits, the same tiles as mode 3,
    and values that are not 16-byte aligned (4032-bit workgroup tiles)."""
    say(f"[vlane] {dtype} chunks={chunks}")
    for name in CASES:
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 33, dtype=NP[dtype])
        y_ref, s_ref = oracle.csr_spmv(A, x)
        B = to_beta(A, 1, 8, dtype)
        xd = torch.from_numpy(x).cuda()
        P = B.plan(0, 0, 4, chunks)
        assert P.info()["n_tiles"] == B.plan(0, 0, 3, chunks).info()["n_tiles"]
        y = spc.spmv(B, xd, plan=P)
        check_rows(y.cpu().numpy(), y_ref, s_ref, TOL[dtype], f"vlane {name}")
        assert torch.equal(spc.spmv(B, xd, plan=P), y), name
        assert torch.equal(spc.spmv(B, xd, plan=B.plan(0, 1, 4, chunks, 0, 3)), y), name
        y0 = synth.dense_vector(A.n_rows, 34, dtype=NP[dtype])
        ya = spc.spmv(B, xd, torch.from_numpy(y0.copy()).cuda(), accumulate=True, plan=P).cpu().numpy()
        check_rows(ya, y_ref + y0.astype(np.float64), s_ref + np.abs(y0.astype(np.float64)), TOL[dtype],
                   f"vlane {name} accumulate")
        empty = A.row_lengths() == 0
        assert np.array_equal(ya[empty], y0[empty])
        if empty.any():
            yh = y.cpu().numpy()
            assert np.all(yh[empty] == 0) and not np.signbit(yh[empty]).any()
        if name in ("stencil16", "dense_rows", "powerlaw"):
            buf = torch.empty(B.nnz + 1, dtype=dtype, device="cuda")
            buf[1:] = B.values
            Bu = to_beta(A, 1, 8, dtype)
            Bu.values = buf[1:]
            yu = spc.spmv(Bu, xd, plan=Bu.plan(0, 0, 4, chunks)).cpu().numpy()
            check_rows(yu, y_ref, s_ref, TOL[dtype], f"vlane unaligned {name}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_value_lanes_integers_nonfinite_and_shapes(dtype):
    """Mode 4: integer-valued inputs give exact sums; an Inf in x reaches
    exactly the rows that store an entry in its column; shapes other than
    beta(1,8) are refused."""
    say(f"[vlane-int] {dtype}")
    A = synth.powerlaw(1500, 1500, seed=11)
    A.values = np.round(A.values * 16)
    x = np.round(synth.dense_vector(A.n_cols, 24) * 16)
    y_ref, _ = oracle.csr_spmv(A, x)
    B = to_beta(A.astype(NP[dtype]), 1, 8, dtype)
    for chunks in (2, 8):
        y = spc.spmv(B, torch.from_numpy(x.astype(NP[dtype])).cuda(), plan=B.plan(0, 0, 4, chunks))
        assert np.array_equal(y.cpu().numpy().astype(np.float64), y_ref)
    S = synth.random_small(64, 64, 0.15, seed=12)
    j = 9
    xs = synth.dense_vector(64, 25)
    xs[j] = np.inf
    Bs = to_beta(S.astype(NP[dtype]), 1, 8, dtype)
    ys = spc.spmv(Bs, torch.from_numpy(xs.astype(NP[dtype])).cuda(), plan=Bs.plan(0, 0, 4, 4)).cpu().numpy()
    has_j = np.array([j in S.colidx[S.rowptr[i]:S.rowptr[i + 1]] for i in range(S.n_rows)])
    assert np.all(np.isfinite(ys[~has_j])) and not np.any(np.isfinite(ys[has_j]))
    for (r, c) in spc.SHAPES[1:]:
        Bo = to_beta(S.astype(NP[dtype]), r, c, dtype)
        with pytest.raises(spc.SpcError):
            Bo.plan(0, 0, 4, 4)
    with pytest.raises(spc.SpcError):
        spc.plan_from(Bs, dict(mode=4, wave_chunks=4, wave_tiles=2))
