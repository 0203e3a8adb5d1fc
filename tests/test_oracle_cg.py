"""Pins for the CG oracle: manufactured solutions, finite termination on a
matrix with few distinct eigenvalues, and a dense direct solve."""
import numpy as np

from oracle import cg as CG
from paper_1801_01134_amd import synth


def test_manufactured_solution_spd_stencil():
    A = synth.stencil27(8, diag=26.1, offdiag=-1.0)
    xs = synth.dense_block(A.n_cols, 3, 11)
    import oracle
    B, _ = oracle.csr_spmm(A, xs)
    X, it, hist = CG.cg(A, B, tol=1e-10)
    assert (it > 0).all()
    assert np.max(np.abs(X - xs)) < 1e-8
    assert np.all(CG.true_residual(A, X, B) <= 1e-9 * np.linalg.norm(B, axis=0))


def test_terminates_in_m_steps_for_m_distinct_eigenvalues():
    eig = np.repeat([1.0, 3.0, 10.0, 40.0], 25)  # 4 distinct values
    A = synth.from_dense(np.diag(eig))
    b = synth.dense_vector(eig.size, 12)
    X, it, hist = CG.cg(A, b, tol=1e-12)
    assert 0 < it[0] <= 4


def test_dense_spd_against_direct_solve():
    rng = synth.rng_for(13)
    M = rng.normal(size=(30, 30))
    Ad = M @ M.T + 30 * np.eye(30)
    A = synth.from_dense(Ad)
    b = rng.normal(size=30)
    X, it, _ = CG.cg(A, b, tol=1e-13)
    assert np.allclose(X[:, 0], np.linalg.solve(Ad, b), rtol=1e-10, atol=1e-12)
