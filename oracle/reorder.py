"""Oracle of the reordering step (section "Matrix permutation/reordering":
a Cuthill-McKee breadth-first renumbering puts connected rows and columns
next to each other, so blocks hold more values). TEST INFRASTRUCTURE ONLY.

The order is defined exactly, so that any implementation following the same
definition gives the same permutation:

  G      the graph of the pattern of A + A^T without the diagonal (square A);
         deg(v) = number of distinct neighbours of v.
  start  among the vertices not yet numbered, the one of smallest degree
         (smallest index on ties).
  BFS    from the start vertex: take vertices off the queue in order; each
         appends its neighbours not yet numbered, sorted by (degree, index),
         to the order and to the queue. When the queue empties with vertices
         left (another connected component), pick a new start as above.
  RCM    the order reversed: perm[new] = old.

The reordered matrix is B = P A P^T with B[i][j] = A[perm[i]][perm[j]]; for
y = A x this gives y[perm[i]] = (B x')[i] with x'[j] = x[perm[j]].
"""
from __future__ import annotations

from collections import deque

import numpy as np


def neighbours(csr) -> list[list[int]]:
    """Distinct neighbours of every vertex in A + A^T, diagonal dropped."""
    n = csr.n_rows
    if csr.n_cols != n:
        raise ValueError("reordering needs a square matrix")
    nb = [set() for _ in range(n)]
    for i in range(n):
        for p in range(int(csr.rowptr[i]), int(csr.rowptr[i + 1])):
            j = int(csr.colidx[p])
            if j != i:
                nb[i].add(j)
                nb[j].add(i)
    return [sorted(s) for s in nb]


def rcm_order(csr) -> np.ndarray:
    """perm[new] = old, by the definition in the module docstring."""
    nb = neighbours(csr)
    n = len(nb)
    deg = [len(s) for s in nb]
    numbered = [False] * n
    order: list[int] = []
    while len(order) < n:
        start = min((v for v in range(n) if not numbered[v]), key=lambda v: (deg[v], v))
        numbered[start] = True
        order.append(start)
        q = deque([start])
        while q:
            v = q.popleft()
            for w in sorted((w for w in nb[v] if not numbered[w]), key=lambda w: (deg[w], w)):
                numbered[w] = True
                order.append(w)
                q.append(w)
    return np.array(order[::-1], dtype=np.int64)


def permute(csr, perm):
    """B = P A P^T as (rowptr, colidx, values): row i of B is row perm[i] of A
    with every column j renamed inv[j] (inv the inverse permutation), columns
    sorted; values are moved bit for bit."""
    perm = np.asarray(perm, dtype=np.int64)
    n = csr.n_rows
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        lo, hi = int(csr.rowptr[perm[i]]), int(csr.rowptr[perm[i] + 1])
        c = inv[csr.colidx[lo:hi].astype(np.int64)]
        o = np.argsort(c, kind="stable")
        cols.append(c[o])
        vals.append(np.asarray(csr.values)[lo:hi][o])
        rowptr[i + 1] = rowptr[i] + (hi - lo)
    colidx = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    values = np.concatenate(vals) if vals else np.zeros(0, np.asarray(csr.values).dtype)
    return rowptr, colidx.astype(np.int32), values


def bandwidth(rowptr, colidx) -> int:
    """max |i - j| over the stored entries."""
    bw = 0
    for i in range(len(rowptr) - 1):
        for p in range(int(rowptr[i]), int(rowptr[i + 1])):
            bw = max(bw, abs(int(colidx[p]) - i))
    return bw
