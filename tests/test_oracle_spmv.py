"""Pins for the CSR product oracle: brute force, closed forms, exact cases."""
import numpy as np
import pytest

import oracle
from paper_1801_01134_amd import synth


@pytest.mark.parametrize("shape,density,seed", [((1, 1), 1.0, 0), ((7, 5), 0.4, 1),
                                               ((16, 16), 0.2, 2), ((33, 70), 0.1, 3),
                                               ((64, 9), 0.5, 4), ((5, 40), 0.0, 5)])
def test_spmv_matches_dense_bruteforce_exactly(shape, density, seed):
    A = synth.random_small(*shape, density, seed=seed, integer_values=True)
    dense = np.zeros(shape)
    for i in range(A.n_rows):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            dense[i, A.colidx[p]] = A.values[p]
    x = synth.rng_for(99, seed).integers(-16, 17, size=shape[1]).astype(np.float64)
    y, s = oracle.csr_spmv(A, x)
    # small integers: every partial sum is exact, so equality is bitwise
    assert np.array_equal(y, oracle.dense_matvec(dense, x))
    assert np.array_equal(s, oracle.dense_matvec(np.abs(dense), np.abs(x)))


def test_identity_permutation_and_empty_rows():
    n = 50
    x = synth.dense_vector(n, 7)
    I = synth.from_dense(np.eye(n))
    assert np.array_equal(oracle.csr_spmv(I, x)[0], x)
    perm = synth.rng_for(5).permutation(n)
    Pm = np.zeros((n, n))
    Pm[np.arange(n), perm] = 1.0
    assert np.array_equal(oracle.csr_spmv(synth.from_dense(Pm), x)[0], x[perm])
    Z = np.zeros((n, n))
    Z[3, 4] = 2.0
    y = oracle.csr_spmv(synth.from_dense(Z), x)[0]
    assert y[3] == 2.0 * x[4] and np.count_nonzero(y) == 1


def test_spmm_columns_equal_spmv():
    A = synth.band_plus_uniform(512, seed=3)
    X = synth.dense_block(A.n_cols, 5, 1)
    Y, S = oracle.csr_spmm(A, X)
    for q in range(5):
        y, s = oracle.csr_spmv(A, X[:, q])
        assert np.array_equal(Y[:, q], y) and np.array_equal(S[:, q], s)


def test_stencil_row_sums_closed_form():
    # off-diagonals -1 and diagonal 26 + shift: A * ones = shift + (26 - (len-1))
    m = 12
    A = synth.stencil27(m, diag=26.1, offdiag=-1.0)
    y, _ = oracle.csr_spmv(A, np.ones(A.n_cols))
    lens = A.row_lengths()
    assert np.allclose(y, 26.1 - (lens - 1), rtol=0, atol=1e-12)
    assert A.nnz == synth.stencil27_nnz(m)
