"""Pins for the reordering oracle (section "Matrix permutation/reordering":
Cuthill-McKee renumbering). The order is checked against hand-computed
cases and against closed forms of the bandwidth it reaches; the symmetric
permutation against its definition (round trip and the product identity)."""
import numpy as np
import pytest

import oracle
from oracle import reorder as R
from paper_1801_01134_amd import synth


def _from_edges(n, edges, diag=True):
    a = np.zeros((n, n))
    for i, j in edges:
        a[i, j] = a[j, i] = 1.0
    if diag:
        a[np.arange(n), np.arange(n)] = 1.0
    return synth.from_dense(a)


def test_hand_computed_order():
    # edges 0-2, 0-4, 2-4, 1-3, 3-4; degrees 0:2 1:1 2:2 3:2 4:3.
    # start = 1 (degree 1); 1 numbers 3; 3 numbers 4; 4 numbers 0 and 2
    # (both degree 2, index order); Cuthill-McKee order 1 3 4 0 2, reversed
    # 2 0 4 3 1
    A = _from_edges(5, [(0, 2), (0, 4), (2, 4), (1, 3), (3, 4)])
    assert R.rcm_order(A).tolist() == [2, 0, 4, 3, 1]


def test_components_and_isolated_vertex():
    # edges 0-1 and 3-4, vertex 2 alone (degree 0): start 2, then 0 (degree 1,
    # lowest index) numbers 1, then 3 numbers 4: order 2 0 1 3 4, reversed
    A = _from_edges(5, [(0, 1), (3, 4)])
    assert R.rcm_order(A).tolist() == [4, 3, 1, 0, 2]


def test_one_sided_pattern_is_symmetrized():
    # only the upper triangle stored: (0,3) and (3,1); the graph is 0-3-1
    a = np.eye(4)
    a[0, 3] = a[3, 1] = 2.0
    A = synth.from_dense(a)
    # degrees 0:1 1:1 2:0 3:2; start 2; then 0 numbers 3, 3 numbers 1:
    # order 2 0 3 1, reversed 1 3 0 2
    assert R.rcm_order(A).tolist() == [1, 3, 0, 2]


@pytest.mark.parametrize("n,seed", [(2, 0), (7, 1), (50, 2), (301, 3)])
def test_scrambled_path_becomes_tridiagonal(n, seed):
    # a path numbered at random: breadth-first from an end walks the path, so
    # the reordered matrix has bandwidth exactly 1
    A = synth.grid_scrambled(n, 1, 1, "5pt", seed=seed)
    p = R.rcm_order(A)
    assert sorted(p.tolist()) == list(range(n))
    rp, ci, _ = R.permute(A, p)
    assert R.bandwidth(rp, ci) == 1


@pytest.mark.parametrize("m", [5, 12, 20])
def test_scrambled_grid_bandwidth(m):
    # 5-point m x m grid: search from a corner (degree 2); the breadth-first
    # levels are the anti-diagonals (at most m points), neighbours lie in
    # adjacent levels, so the bandwidth is below two level widths
    A = synth.grid_scrambled(m, m, 1, "5pt", seed=m)
    p = R.rcm_order(A)
    rp, ci, _ = R.permute(A, p)
    assert R.bandwidth(rp, ci) <= 2 * m
    assert R.bandwidth(A.rowptr, A.colidx) > 2 * m      # the random numbering is far wider


def test_permutation_round_trip_and_product():
    A = synth.grid_scrambled(9, 7, 3, "27pt", seed=4)
    A.values = np.round(A.values * 16)                   # small integers: exact sums
    rng = np.random.default_rng(5)
    p = rng.permutation(A.n_rows)
    rp, ci, v = R.permute(A, p)
    B = synth.CSR(A.n_rows, A.n_cols, rp, ci, v)
    inv = np.empty_like(p)
    inv[p] = np.arange(A.n_rows)
    rp2, ci2, v2 = R.permute(B, inv)
    assert np.array_equal(rp2, A.rowptr) and np.array_equal(ci2, A.colidx) and np.array_equal(v2, A.values)
    # y = A x  <=>  y[p[i]] = (B x')[i], x'[j] = x[p[j]]
    x = np.round(synth.dense_vector(A.n_cols, 6) * 16)
    y, _ = oracle.csr_spmv(A, x)
    yb, _ = oracle.csr_spmv(B, x[p])
    out = np.empty_like(y)
    out[p] = yb
    assert np.array_equal(out, y)
    # rows of B keep sorted, unique columns
    for i in range(B.n_rows):
        c = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_reordering_restores_blocks_of_a_scrambled_stencil():
    # a 3-D stencil numbered at random has about one value per beta(1,8)
    # block; after RCM its rows again hold runs of neighbouring columns
    A = synth.grid_scrambled(10, 10, 10, "27pt", seed=7)
    p = R.rcm_order(A)
    rp, ci, v = R.permute(A, p)
    B = synth.CSR(A.n_rows, A.n_cols, rp, ci, v)
    for (r, c) in ((1, 8), (2, 4), (4, 8)):
        before = A.nnz / oracle.n_blocks(A, r, c)
        after = B.nnz / oracle.n_blocks(B, r, c)
        assert after > 1.5 * before, (r, c, before, after)
