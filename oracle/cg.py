"""FP64 conjugate gradients for k independent right-hand sides sharing one
matrix. TEST INFRASTRUCTURE ONLY. The paper motivates fast SpMV by Krylov
solvers such as CG, where one matrix is applied many times (Introduction);
this is the plain Hestenes-Stiefel recurrence, one column at a time in
lockstep, with columns frozen once their residual meets the tolerance.
"""
from __future__ import annotations

import numpy as np

from . import csr_spmm


def cg(csr, B, tol: float = 1e-8, maxit: int = 10_000):
    """Solve A X = B column by column from X0 = 0.

    Column q stops when ||r_q|| <= tol * ||b_q||. Returns X, the iteration at
    which each column converged (-1 if never), and the per-iteration residual
    norms (k columns)."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    k = B.shape[1]
    X = np.zeros_like(B)
    R = B.copy()
    P = R.copy()
    rr = np.sum(R * R, axis=0)
    bnorm = np.sqrt(np.sum(B * B, axis=0))
    done = np.sqrt(rr) <= tol * bnorm
    it_done = np.where(done, 0, -1)
    hist = [np.sqrt(rr)]
    for it in range(1, maxit + 1):
        if done.all():
            break
        Q, _ = csr_spmm(csr, P)
        pq = np.sum(P * Q, axis=0)
        alpha = np.where(done, 0.0, rr / np.where(done, 1.0, pq))
        X += alpha * P
        R -= alpha * Q
        rr_new = np.sum(R * R, axis=0)
        beta = np.where(done, 0.0, rr_new / np.where(done, 1.0, rr))
        P = R + beta * P
        rr = np.where(done, rr, rr_new)
        hist.append(np.sqrt(rr))
        newly = (~done) & (np.sqrt(rr) <= tol * bnorm)
        it_done[newly] = it
        done |= newly
    return X, it_done, np.array(hist)


def true_residual(csr, X, B):
    """||B - A X|| per column, recomputed from scratch with the CSR oracle."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
        X = np.asarray(X)[:, None]
    AX, _ = csr_spmm(csr, X)
    return np.sqrt(np.sum((B - AX) ** 2, axis=0))
