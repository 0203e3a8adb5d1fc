"""Reordering on the device against the oracle: the library's reverse
Cuthill-McKee order equals the oracle's (the order is fully defined), the
device permutation B = P A P^T equals the oracle's bit for bit, and products
through the reordered beta(r,c) matrix with permuted vectors match the CSR
oracle on the original matrix (per-row bound 1e-13 / 2e-6 sum |a x|)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import reorder as R
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _one_sided():
    A = synth.powerlaw(700, 700, seed=31)
    keep = np.repeat(np.arange(A.n_rows), np.diff(A.rowptr)) <= A.colidx   # upper triangle only
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.rowptr))[keep]
    return synth.from_keys_sorted(A.n_rows, A.n_cols, rows, A.colidx[keep], 32)


CASES = {
    "path_scrambled": lambda: synth.grid_scrambled(500, 1, 1, "5pt", seed=1),
    "grid2d_scrambled": lambda: synth.grid_scrambled(30, 40, 1, "9pt", seed=2),
    "grid3d_scrambled": lambda: synth.grid_scrambled(12, 11, 13, "27pt", seed=3),
    "stencil_natural": lambda: synth.stencil27(14),
    "powerlaw": lambda: synth.powerlaw(1500, 1500, seed=4),
    "one_sided": _one_sided,
    "components": lambda: synth.CSR(6, 6, np.array([0, 1, 2, 2, 4, 5, 6]), np.array([1, 0, 4, 5, 3, 3]),
                                    np.arange(1.0, 7.0)),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_rcm_order_equals_oracle(name):
    say(f"[reorder] order {name}")
    A = case(name)
    p = spc.rcm_order(A.rowptr, A.colidx).cpu().numpy()
    assert np.array_equal(p, R.rcm_order(A))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_permute_bit_exact(name, dtype):
    say(f"[reorder] permute {name} {dtype}")
    A = case(name).astype(NP[dtype])
    p = R.rcm_order(A)
    rp, ci, v = spc.csr_permute(A.rowptr, A.colidx, torch.from_numpy(A.values), torch.from_numpy(p))
    rp0, ci0, v0 = R.permute(A, p)
    assert np.array_equal(rp.cpu().numpy(), rp0) and np.array_equal(ci.cpu().numpy(), ci0)
    assert np.array_equal(v.cpu().numpy().view(np.uint8), v0.view(np.uint8))


def test_permute_refuses_a_non_permutation():
    A = case("powerlaw")
    bad = np.arange(A.n_rows, dtype=np.int32)
    bad[5] = 7
    with pytest.raises(spc.SpcError):
        spc.csr_permute(A.rowptr, A.colidx, torch.from_numpy(A.values), torch.from_numpy(bad))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
def test_products_through_the_reordered_matrix(rc, dtype):
    r, c = rc
    for name in ("grid3d_scrambled", "powerlaw", "one_sided"):
        say(f"[reorder] spmv {name} beta{rc} {dtype}")
        A = case(name).astype(NP[dtype])
        x = synth.dense_vector(A.n_cols, 40).astype(NP[dtype])
        y_ref, s_ref = oracle.csr_spmv(A, x)
        perm = spc.rcm_order(A.rowptr, A.colidx)
        rp, ci, v = spc.csr_permute(A.rowptr, A.colidx, torch.from_numpy(A.values), perm)
        B = spc.csr_to_beta(r, c, rp, ci, v, A.n_cols)
        xd = torch.from_numpy(x).cuda()
        xp = spc.permute_vector(xd, perm)
        assert torch.equal(xp.cpu(), torch.from_numpy(x[perm.cpu().numpy()]))
        y = spc.permute_vector(spc.spmv(B, xp), perm, scatter=True).cpu().numpy().astype(np.float64)
        bad = np.flatnonzero(~(np.abs(y - y_ref) <= TOL[dtype] * s_ref))
        assert bad.size == 0, (name, bad[:5])


def test_full_size_scrambled_stencil():
    """The 27-point stencil of a 128^3 grid numbered at random: RCM gives a
    permutation (checked on the host), the blocks regain values, and the
    beta(2,4) product of the reordered matrix matches the oracle on every row
    of the original one."""
    say("[reorder] 128^3 scrambled stencil")
    A = synth.grid_scrambled(128, 128, 128, "27pt", seed=9)
    perm = spc.rcm_order(A.rowptr, A.colidx)
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(A.n_rows))
    rp, ci, v = spc.csr_permute(A.rowptr, A.colidx, torch.from_numpy(A.values), perm)
    B0 = spc.csr_to_beta(2, 4, A.rowptr, A.colidx, torch.from_numpy(A.values), A.n_cols)
    B = spc.csr_to_beta(2, 4, rp, ci, v, A.n_cols)
    assert A.nnz / B.n_blocks > 2.5 * (A.nnz / B0.n_blocks)
    x = synth.dense_vector(A.n_cols, 41)
    y_ref, s_ref = oracle.csr_spmv(A, x)
    xp = spc.permute_vector(torch.from_numpy(x).cuda(), perm)
    y = spc.permute_vector(spc.spmv(B, xp), perm, scatter=True).cpu().numpy()
    bad = np.flatnonzero(~(np.abs(y - y_ref) <= 1e-13 * s_ref))
    assert bad.size == 0
