"""CPU oracle for the mask-block SpMV method (Bramas & Kus, arXiv 1801.01134).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the GPU
library (``paper_1801_01134_amd``) and imports nothing from it; the two meet
only through the seeded input generators in ``paper_1801_01134_amd.synth``,
which the callers use to draw inputs and then hand to both sides.

Everything here is plain and slow on purpose: the definitions are written out
in double precision, in the order the paper gives them.

* ``csr_spmv`` / ``csr_spmm``: y = A x over CSR, the plain definition the
  mask-block kernels must reproduce (Background, "Sparse Matrix Vector
  Product"; Algorithm 1's input/output), plus s_i = sum_j |a_ij x_j| for the
  per-row error bound.
* ``beta_count`` / ``csr_to_beta`` / ``beta_to_csr``: the beta(r,c) storage
  (Design, "Block-based storage without zero padding", Eq. (1)) under the
  greedy leftmost-cover reading of where blocks start.
* ``vexpand`` / ``expand_to_dense``: what the beta arrays mean, block by
  block, with the vexpand placement rule from the Vectorization section
  (tiny inputs).
* ``occupancy`` and friends: Eqs. (1)-(4).
* ``features``, ``fit_interpolation``, ``select_interpolation``, ``regret``:
  the record-based kernel selection ("Performance polynomial interpolation").
* ``mlp``: the FP64 reference of the learned selector (forward, backward, Adam).
* ``cg``: FP64 conjugate gradients used to check the multi-RHS solver.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

SHAPES = ((1, 8), (2, 4), (2, 8), (4, 4), (4, 8), (8, 4))


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, OpenMP)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.oracle_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_csr_spmv.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        L.oracle_csr_spmm.argtypes = [i64, vp, vp, vp, i32, vp, i64, vp, i64, vp]
        L.oracle_beta_count.argtypes = [i32, i32, i64, vp, vp, vp]
        L.oracle_beta_fill.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp]
        L.oracle_beta_decode.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp]
        L.oracle_beta_decode.restype = i32
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the C oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_parts(csr):
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(csr.colidx, dtype=np.int32)
    return rp, ci


# --------------------------------------------------------------------------
# y = A x (Background: CSR; Algorithm 1 input/output)
# --------------------------------------------------------------------------
def csr_spmv(csr, x) -> tuple[np.ndarray, np.ndarray]:
    """Returns (y, s): y_i = sum_j a_ij x_j and s_i = sum_j |a_ij x_j| in FP64.

    Inputs of lower precision are upcast exactly before any arithmetic."""
    rp, ci = _csr_parts(csr)
    v = np.ascontiguousarray(csr.values, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(csr.n_rows, dtype=np.float64)
    s = np.empty(csr.n_rows, dtype=np.float64)
    lib().oracle_csr_spmv(csr.n_rows, _p(rp), _p(ci), _p(v), _p(xx), _p(y), _p(s))
    return y, s


def csr_spmm(csr, X) -> tuple[np.ndarray, np.ndarray]:
    """Y = A X for a row-major block X (n_cols x k); returns (Y, S) in FP64."""
    rp, ci = _csr_parts(csr)
    v = np.ascontiguousarray(csr.values, dtype=np.float64)
    XX = np.ascontiguousarray(X, dtype=np.float64)
    k = XX.shape[1]
    Y = np.empty((csr.n_rows, k), dtype=np.float64)
    S = np.empty((csr.n_rows, k), dtype=np.float64)
    lib().oracle_csr_spmm(csr.n_rows, _p(rp), _p(ci), _p(v), k, _p(XX), k, _p(Y), k, _p(S))
    return Y, S


def dense_matvec(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Brute-force dense product, one scalar at a time (tiny inputs only)."""
    n, m = a.shape
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        acc = 0.0
        for j in range(m):
            if a[i, j] != 0.0:
                acc += float(a[i, j]) * float(x[j])
        y[i] = acc
    return y


# --------------------------------------------------------------------------
# beta(r,c) storage (Design: block-based storage without zero padding)
# --------------------------------------------------------------------------
class BetaRef:
    """The four beta(r,c) arrays as the oracle builds them.

    block_rowptr int64[ceil(n_rows/r)+1]  prefix pointers into the blocks
    block_colidx int32[n_blocks]          column of each block's left edge
    masks        uint32[n_blocks]         bit i*c+k <-> (row i, column k) of the block
    values       packed values, block order, row-major inside a block
    perm         int64[nnz]               CSR position of each packed value
    """

    def __init__(self, r, c, n_rows, n_cols, block_rowptr, block_colidx, masks, values, perm):
        self.r, self.c = int(r), int(c)
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.block_rowptr = block_rowptr
        self.block_colidx = block_colidx
        self.masks = masks
        self.values = values
        self.perm = perm

    @property
    def n_blocks(self) -> int:
        return int(self.block_rowptr[-1])

    @property
    def nnz(self) -> int:
        return int(self.values.size)

    def mask_bytes(self) -> np.ndarray:
        """Masks as the byte stream of ceil(r*c/8)-byte little-endian words."""
        w = (self.r * self.c) // 8
        m = self.masks.astype("<u4").view(np.uint8).reshape(-1, 4)
        return np.ascontiguousarray(m[:, :w]).reshape(-1)


def beta_count(csr, r: int, c: int) -> np.ndarray:
    """Blocks per row interval under the greedy leftmost cover (int64)."""
    rp, ci = _csr_parts(csr)
    n_int = (csr.n_rows + r - 1) // r
    counts = np.empty(n_int, dtype=np.int64)
    lib().oracle_beta_count(r, c, csr.n_rows, _p(rp), _p(ci), _p(counts))
    return counts


def n_blocks(csr, r: int, c: int) -> int:
    return int(beta_count(csr, r, c).sum())


def csr_to_beta(csr, r: int, c: int) -> BetaRef:
    """CSR -> beta(r,c). Packed values keep their type and bits (a permutation)."""
    if r * c not in (8, 16, 32) or r > 8:
        raise ValueError("unsupported block shape")
    rp, ci = _csr_parts(csr)
    counts = beta_count(csr, r, c)
    brp = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=brp[1:])
    nb = int(brp[-1])
    bcol = np.empty(nb, dtype=np.int32)
    masks = np.empty(nb, dtype=np.uint32)
    perm = np.empty(csr.nnz, dtype=np.int64)
    lib().oracle_beta_fill(r, c, csr.n_rows, _p(rp), _p(ci), _p(brp), _p(bcol), _p(masks), _p(perm))
    values = np.ascontiguousarray(csr.values)[perm]
    return BetaRef(r, c, csr.n_rows, csr.n_cols, brp, bcol, masks, values, perm)


def beta_to_csr(beta: BetaRef):
    """beta(r,c) -> CSR (rowptr, colidx, values) with values moved bit for bit."""
    brp = np.ascontiguousarray(beta.block_rowptr, dtype=np.int64)
    bcol = np.ascontiguousarray(beta.block_colidx, dtype=np.int32)
    masks = np.ascontiguousarray(beta.masks, dtype=np.uint32)
    nnz = int(sum(int(m).bit_count() for m in masks)) if masks.size < 4096 else \
        int(np.unpackbits(masks.view(np.uint8)).sum())
    rowptr = np.zeros(beta.n_rows + 1, dtype=np.int32)
    colidx = np.empty(nnz, dtype=np.int32)
    src = np.empty(nnz, dtype=np.int64)
    rc = lib().oracle_beta_decode(beta.r, beta.c, beta.n_rows, _p(brp), _p(bcol), _p(masks),
                                  _p(rowptr), _p(colidx), _p(src))
    if rc != 0:
        raise ValueError(f"malformed beta matrix (code {rc})")
    return rowptr, colidx, np.ascontiguousarray(beta.values)[src]


# --------------------------------------------------------------------------
# The format's meaning, block by block (tiny inputs)
# --------------------------------------------------------------------------
def vexpand(mask: int, packed, width: int):
    """The vexpandpd rule (Vectorization section): lane k takes the next packed
    value when bit k of the mask is set, else 0; bit 0 is the leftmost lane."""
    out, idx = [], 0
    for k in range(width):
        if (mask >> k) & 1:
            out.append(packed[idx])
            idx += 1
        else:
            out.append(0.0)
    return out, idx


def expand_to_dense(beta: BetaRef) -> np.ndarray:
    """The dense matrix a beta(r,c) matrix stands for.

    Each block is an r x c tile whose upper-left corner is (interval * r,
    block column). Its packed values are expanded by the vexpand rule over
    the block's r*c mask bits taken row after row (values are row-major
    inside a block, and bit i*c + k is row i, column k), so the tile's entry
    (i, k) is the next packed value when that bit is set and 0 otherwise.
    Tiles of one interval never overlap, so they are written, not added."""
    r, c = beta.r, beta.c
    out = np.zeros((beta.n_rows, beta.n_cols + c), dtype=np.float64)
    vpos = 0
    for t in range(len(beta.block_rowptr) - 1):
        for b in range(int(beta.block_rowptr[t]), int(beta.block_rowptr[t + 1])):
            tile, used = vexpand(int(beta.masks[b]), beta.values[vpos:vpos + r * c], r * c)
            vpos += used
            col = int(beta.block_colidx[b])
            for i in range(r):
                if t * r + i < beta.n_rows:
                    out[t * r + i, col:col + c] = tile[i * c:(i + 1) * c]
    if vpos != beta.values.size:
        raise ValueError("mask bits do not account for every packed value")
    return out[:, :beta.n_cols]


def min_cover_bruteforce(cols: list[int], c: int) -> int:
    """Fewest width-c windows covering a set of integers, by exhaustive search
    over window starts taken from the set (tiny sets only)."""
    cols = sorted(set(cols))
    if not cols:
        return 0
    from itertools import combinations
    for k in range(1, len(cols) + 1):
        for starts in combinations(cols, k):
            if all(any(s <= v < s + c for s in starts) for v in cols):
                return k
    return len(cols)


# --------------------------------------------------------------------------
# Eqs. (1)-(4): memory occupancy
# --------------------------------------------------------------------------
def occupancy(r: int, c: int, nnz: int, n_rows: int, n_blocks_: int, s_float: int,
              s_int: int = 4) -> dict:
    """Eq. (1), with the row-pointer term taken exactly as (ceil(N/r)+1) ints."""
    o_values = nnz * s_float
    o_rowptr = ((n_rows + r - 1) // r + 1) * s_int
    o_colidx = n_blocks_ * s_int
    o_masks = n_blocks_ * r * c // 8
    return {"values": o_values, "block_rowptr": o_rowptr, "block_colidx": o_colidx,
            "block_masks": o_masks, "total": o_values + o_rowptr + o_colidx + o_masks}


def occupancy_eq2(r: int, c: int, nnz: int, n_rows: int, avg: float, s_float: int,
                  s_int: int = 4) -> float:
    """Eq. (2): the total after substituting N_blocks = NNZ / Avg(r,c)."""
    return nnz * s_float + n_rows * s_int / r + nnz * (8 * s_int + r * c) / (8 * avg)


def occupancy_csr(nnz: int, n_rows: int, s_float: int, s_int: int = 4) -> int:
    """Eq. (3) with the exact N_rows + 1 row pointers."""
    return nnz * s_float + (n_rows + 1) * s_int + nnz * s_int


def breakeven_avg(r: int, c: int, s_int: int = 4) -> float:
    """Eq. (4): beta(r,c) index bytes beat CSR's when Avg(r,c) exceeds this."""
    return 1.0 + (r * c) / (8.0 * s_int)


from . import select as select  # noqa: E402  (re-export submodules)
from . import mlp as mlp  # noqa: E402
from . import cg as cg  # noqa: E402
from . import reorder as reorder  # noqa: E402
