"""Seeded synthetic inputs: sparse matrices in CSR form and dense vectors.

This module only draws inputs. It holds none of the mask-block method's
arithmetic, and both the library tests and the CPU oracle take their inputs
from here. Every generator returns plain numpy arrays:

    rowptr  int32[n_rows + 1]
    colidx  int32[nnz]        (ascending and unique inside each row)
    values  float64[nnz]

The shapes mimic the kinds of matrices the paper measures (SuiteSparse sets of
its Tables 1 and 2: stencil-like, FEM block structure, banded, power-law and
uniformly random rows); the paper's own matrices are not used.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
BASE_SEED = 1801


def splitmix64(state: int) -> int:
    """One SplitMix64 output for the given 64-bit state (Steele et al. 2014)."""
    z = (state + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def derive_seed(*parts: int) -> int:
    """Fold integers into one 64-bit seed with SplitMix64."""
    s = BASE_SEED
    for p in parts:
        s = splitmix64((s ^ (int(p) & MASK64)) & MASK64)
    return s


def rng_for(*parts: int) -> np.random.Generator:
    return np.random.default_rng(derive_seed(*parts))


class CSR:
    """A CSR matrix as plain arrays; `values` is float64 unless cast."""

    __slots__ = ("n_rows", "n_cols", "rowptr", "colidx", "values")

    def __init__(self, n_rows, n_cols, rowptr, colidx, values):
        self.n_rows = int(n_rows)
        self.n_cols = int(n_cols)
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self.colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        self.values = np.ascontiguousarray(values)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def astype(self, dtype) -> "CSR":
        return CSR(self.n_rows, self.n_cols, self.rowptr, self.colidx,
                   self.values.astype(dtype))

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)


def from_keys_sorted(n_rows: int, n_cols: int, rows, cols, seed: int) -> CSR:
    """CSR of the given (row, col) pairs (deduplicated and sorted), values U[-1, 1]."""
    return _from_keys(n_rows, n_cols, np.asarray(rows), np.asarray(cols), rng_for(10, n_rows, seed))


def _from_keys(n_rows: int, n_cols: int, rows: np.ndarray, cols: np.ndarray,
               rng: np.random.Generator, low=-1.0, high=1.0) -> CSR:
    """Deduplicate (row, col) pairs, sort them row-major and draw values."""
    keys = rows.astype(np.int64) * n_cols + cols.astype(np.int64)
    keys = np.unique(keys)
    r = (keys // n_cols).astype(np.int64)
    c = (keys % n_cols).astype(np.int32)
    counts = np.bincount(r, minlength=n_rows)
    rowptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    vals = rng.uniform(low, high, size=c.size)
    return CSR(n_rows, n_cols, rowptr, c, vals)


def dense_vector(n: int, *seed_parts: int, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1], seeded."""
    return rng_for(0x58, *seed_parts).uniform(-1.0, 1.0, size=n).astype(dtype)


def dense_block(n: int, k: int, *seed_parts: int, dtype=np.float64) -> np.ndarray:
    """Row-major n x k block of right-hand sides, U[-1, 1]."""
    return rng_for(0x59, *seed_parts).uniform(-1.0, 1.0, size=(n, k)).astype(dtype)


# --------------------------------------------------------------------------
# Band + uniform rows: n square, per row `band` distinct columns inside
# [i - half, i + half) and `uni` distinct uniform columns disjoint from them.
# --------------------------------------------------------------------------
def band_plus_uniform(n: int = 4096, band: int = 8, uni: int = 8, half: int = 16,
                      seed: int = 0) -> CSR:
    rng = rng_for(1, seed)
    rows = np.empty(n * (band + uni), dtype=np.int64)
    cols = np.empty_like(rows)
    k = 0
    for i in range(n):
        lo, hi = max(0, i - half), min(n, i + half)
        bcols = rng.choice(np.arange(lo, hi), size=min(band, hi - lo), replace=False)
        chosen = set(int(v) for v in bcols)
        ucols = []
        while len(ucols) < uni:
            for v in rng.integers(0, n, size=2 * uni):
                v = int(v)
                if v not in chosen:
                    chosen.add(v)
                    ucols.append(v)
                    if len(ucols) == uni:
                        break
        allc = np.array(sorted(chosen), dtype=np.int64)
        rows[k:k + allc.size] = i
        cols[k:k + allc.size] = allc
        k += allc.size
    return _from_keys(n, n, rows[:k], cols[:k], rng)


# --------------------------------------------------------------------------
# 27-point stencil on an m^3 grid in natural order idx = i + m (j + m k),
# truncated at the boundary. Off-diagonals are U[-1, 1] (or a constant).
# --------------------------------------------------------------------------
def stencil27(m: int, diag: float = 27.0, offdiag: float | None = None,
              seed: int = 0) -> CSR:
    n = m * m * m
    rng = rng_for(2, m, seed)
    ii = np.arange(m, dtype=np.int32)
    # Offsets in ascending column order: dz major, then dy, then dx.
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    # Row lengths: product of per-axis neighbour counts.
    cnt1 = np.full(m, 3, dtype=np.int64)
    cnt1[0] -= 1
    cnt1[-1] -= 1
    if m == 1:
        cnt1[:] = 1
    rl = (cnt1[None, None, :] * cnt1[None, :, None] * cnt1[:, None, None]).reshape(-1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(rl, out=rowptr[1:])
    nnz = int(rowptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    colidx = np.empty(nnz, dtype=np.int32)
    is_diag = np.zeros(nnz, dtype=bool)
    # Fill plane by plane (k) to bound temporary memory.
    plane = m * m
    jj, xx = np.meshgrid(ii, ii, indexing="ij")  # jj: y index, xx: x index
    jj = jj.reshape(-1)
    xx = xx.reshape(-1)
    for k in range(m):
        base = k * plane
        rows = base + np.arange(plane, dtype=np.int64)
        start = rowptr[base:base + plane].copy()
        for (dz, dy, dx) in offs:
            kz, jy, ix = k + dz, jj + dy, xx + dx
            if kz < 0 or kz >= m:
                continue
            ok = (jy >= 0) & (jy < m) & (ix >= 0) & (ix < m)
            pos = start[ok]
            colidx[pos] = (ix[ok] + m * (jy[ok] + m * kz)).astype(np.int32)
            if dz == 0 and dy == 0 and dx == 0:
                is_diag[pos] = True
            start[ok] += 1
        assert np.array_equal(start, rowptr[base + 1:base + plane + 1])
        del rows
    if offdiag is None:
        values = rng.uniform(-1.0, 1.0, size=nnz)
    else:
        values = np.full(nnz, float(offdiag))
    values[is_diag] = diag
    return CSR(n, n, rowptr, colidx, values)


def stencil27_nnz(m: int) -> int:
    return (3 * m - 2) ** 3


# --------------------------------------------------------------------------
# Uniform random rows: Poisson(lam) distinct uniform columns per row.
# --------------------------------------------------------------------------
def uniform_random(n_rows: int, n_cols: int, lam: float, seed: int = 0) -> CSR:
    rng = rng_for(3, n_rows, n_cols, seed)
    lens = np.minimum(rng.poisson(lam, size=n_rows), n_cols)
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), lens)
    cols = rng.integers(0, n_cols, size=rows.size)
    return _from_keys(n_rows, n_cols, rows, cols, rng)


# --------------------------------------------------------------------------
# Banded: every column within `width/2` of the diagonal kept with prob density.
# --------------------------------------------------------------------------
def banded(n: int, width: int, density: float, seed: int = 0) -> CSR:
    rng = rng_for(4, n, width, seed)
    half = max(1, width // 2)
    offs = np.arange(-half, half + 1, dtype=np.int64)
    chunks_r, chunks_c = [], []
    step = max(1, (1 << 24) // offs.size)
    for s in range(0, n, step):
        r = np.arange(s, min(n, s + step), dtype=np.int64)
        c = r[:, None] + offs[None, :]
        keep = (c >= 0) & (c < n) & (rng.random(c.shape) < density)
        keep[:, half] = True  # the diagonal is always present
        rr = np.broadcast_to(r[:, None], c.shape)[keep]
        chunks_r.append(rr)
        chunks_c.append(c[keep])
    return _from_keys(n, n, np.concatenate(chunks_r), np.concatenate(chunks_c), rng)


# --------------------------------------------------------------------------
# Power-law rows: Zipf(a) lengths clipped to [1, max_len]; columns come in
# runs of geometric length starting at uniform positions.
# --------------------------------------------------------------------------
def powerlaw(n_rows: int, n_cols: int, a: float = 1.5, max_len: int = 2000,
             mean_run: float = 4.0, seed: int = 0) -> CSR:
    rng = rng_for(5, n_rows, n_cols, seed)
    lens = rng.zipf(a, size=n_rows)
    bad = lens > max_len
    while bad.any():
        lens[bad] = rng.zipf(a, size=int(bad.sum()))
        bad = lens > max_len
    lens = np.minimum(lens, n_cols).astype(np.int64)
    total = int(lens.sum())
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), lens)
    # Position inside the row, and the run each entry belongs to.
    pos = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(lens) - lens, lens)
    # Every row opens a run; later positions open a new one with probability
    # 1/mean_run, so run lengths are geometric with that mean.
    is_start = (pos == 0) | (rng.random(total) < (1.0 / mean_run))
    run_id = np.cumsum(is_start) - 1
    run_first = np.flatnonzero(is_start)
    run_start_col = rng.integers(0, n_cols, size=run_first.size)
    offset = np.arange(total, dtype=np.int64) - run_first[run_id]
    cols = (run_start_col[run_id] + offset) % n_cols
    return _from_keys(n_rows, n_cols, rows, cols, rng)


# --------------------------------------------------------------------------
# FEM-like: dense b x b blocks on a block pattern near the diagonal.
# --------------------------------------------------------------------------
def fem_blocks(n_block_rows: int, b: int, blocks_per_row: float, spread: int,
               seed: int = 0) -> CSR:
    rng = rng_for(6, n_block_rows, b, seed)
    nb = n_block_rows
    k = np.maximum(1, rng.poisson(blocks_per_row, size=nb))
    brow = np.repeat(np.arange(nb, dtype=np.int64), k)
    first = np.zeros(brow.size, dtype=bool)
    first[np.cumsum(k) - k] = True
    delta = rng.integers(-spread, spread + 1, size=brow.size)
    delta[first] = 0  # diagonal block
    bcol = np.clip(brow + delta, 0, nb - 1)
    bkeys = np.unique(brow * nb + bcol)
    br, bc = bkeys // nb, bkeys % nb
    ii, jj = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")
    rows = (br[:, None] * b + ii.reshape(1, -1)).reshape(-1)
    cols = (bc[:, None] * b + jj.reshape(1, -1)).reshape(-1)
    n = nb * b
    return _from_keys(n, n, rows, cols, rng)


# --------------------------------------------------------------------------
# Mixed: Poisson(lam_u) uniform columns per row plus Poisson(lam_b) aligned
# 3x3 dense blocks per 3-row block row.
# --------------------------------------------------------------------------
def uniform_plus_3x3(n: int, lam_u: float = 16.8, lam_b: float = 2.4,
                     seed: int = 0) -> CSR:
    rng = rng_for(7, n, seed)
    lens = rng.poisson(lam_u, size=n)
    r1 = np.repeat(np.arange(n, dtype=np.int64), lens)
    c1 = rng.integers(0, n, size=r1.size)
    nbr = (n + 2) // 3
    kb = rng.poisson(lam_b, size=nbr)
    br = np.repeat(np.arange(nbr, dtype=np.int64), kb)
    bc = rng.integers(0, nbr, size=br.size)
    ii, jj = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    r2 = (br[:, None] * 3 + ii.reshape(1, -1)).reshape(-1)
    c2 = (bc[:, None] * 3 + jj.reshape(1, -1)).reshape(-1)
    ok = (r2 < n) & (c2 < n)
    rows = np.concatenate([r1, r2[ok]])
    cols = np.concatenate([c1, c2[ok]])
    return _from_keys(n, n, rows, cols, rng)


def dense(n_rows: int, n_cols: int, seed: int = 0) -> CSR:
    rng = rng_for(8, n_rows, n_cols, seed)
    rowptr = np.arange(n_rows + 1, dtype=np.int64) * n_cols
    colidx = np.tile(np.arange(n_cols, dtype=np.int32), n_rows)
    return CSR(n_rows, n_cols, rowptr, colidx, rng.uniform(-1, 1, size=n_rows * n_cols))


def from_dense(a: np.ndarray) -> CSR:
    """CSR of the stored (nonzero) entries of a small dense array."""
    a = np.asarray(a)
    r, c = np.nonzero(a)
    counts = np.bincount(r, minlength=a.shape[0])
    rowptr = np.zeros(a.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(a.shape[0], a.shape[1], rowptr, c.astype(np.int32), a[r, c].astype(np.float64))


def random_small(n_rows: int, n_cols: int, density: float, seed: int = 0,
                 integer_values: bool = False) -> CSR:
    """Tiny matrices for brute-force checks; optional small-integer values."""
    rng = rng_for(9, n_rows, n_cols, seed)
    mask = rng.random((n_rows, n_cols)) < density
    r, c = np.nonzero(mask)
    counts = np.bincount(r, minlength=n_rows)
    rowptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if integer_values:
        vals = rng.integers(-8, 9, size=r.size).astype(np.float64)
    else:
        vals = rng.uniform(-1, 1, size=r.size)
    return CSR(n_rows, n_cols, rowptr, c.astype(np.int32), vals)


# --------------------------------------------------------------------------
# Selector training families (four kinds, 25% each) and the batched mix.
# --------------------------------------------------------------------------
FAMILIES = ("powerlaw", "fem", "banded", "uniform")


def selector_matrix(index: int, min_rows: int = 50_000, max_rows: int = 4_000_000) -> tuple[str, CSR]:
    """Matrix `index` of the selector training/test population."""
    rng = rng_for(30, index)
    fam = FAMILIES[index % 4]
    n = int(np.exp(rng.uniform(np.log(min_rows), np.log(max_rows))))
    s = int(rng.integers(0, 2**31))
    if fam == "powerlaw":
        return fam, powerlaw(n, n, 1.5, 2000, mean_run=float(rng.uniform(1.0, 8.0)), seed=s)
    if fam == "fem":
        b = int(rng.choice([3, 6]))
        return fam, fem_blocks(max(1, n // b), b, float(rng.uniform(3, 12)),
                               int(np.exp(rng.uniform(0, np.log(2000)))), seed=s)
    if fam == "banded":
        w = int(np.exp(rng.uniform(np.log(8), np.log(512))))
        return fam, banded(n, w, float(rng.uniform(0.05, 1.0)), seed=s)
    return fam, uniform_random(n, n, float(rng.uniform(2, 40)), seed=s)


LARGE_NNZ_CAP = 1 << 28


def large_matrix(index: int, min_rows: int = 1_000_000, max_rows: int = 4_000_000) -> tuple[str, CSR]:
    """Matrix `index` of the large population: the four selector families
    with rows log-uniform in [min_rows, max_rows]. Where a family's draw
    would exceed LARGE_NNZ_CAP entries, the parameter that sets the entries
    per row (the band width, the blocks per block row, the mean row length)
    is lowered to meet it."""
    rng = rng_for(31, index)
    fam = FAMILIES[index % 4]
    n = int(np.exp(rng.uniform(np.log(min_rows), np.log(max_rows))))
    s = int(rng.integers(0, 2**31))
    per_row = LARGE_NNZ_CAP / n
    if fam == "powerlaw":  # mean row length about 34: under the cap for n <= 4M
        return fam, powerlaw(n, n, 1.5, 2000, mean_run=float(rng.uniform(1.0, 8.0)), seed=s)
    if fam == "fem":
        b = int(rng.choice([3, 6]))
        k = min(float(rng.uniform(3, 12)), per_row / b)
        return fam, fem_blocks(max(1, n // b), b, k, int(np.exp(rng.uniform(0, np.log(2000)))), seed=s)
    if fam == "banded":
        d = float(rng.uniform(0.05, 1.0))
        w = min(int(np.exp(rng.uniform(np.log(8), np.log(512)))), max(8, int(per_row / d)))
        return fam, banded(n, w, d, seed=s)
    return fam, uniform_random(n, n, min(float(rng.uniform(2, 40)), per_row), seed=s)


# --------------------------------------------------------------------------
# Structured grid operators: 2-D 5/9-point and 3-D 7/27-point stencils in
# natural order idx = x + mx (y + my z), truncated at the boundary, with an
# optional random dropout of off-diagonal entries.
# --------------------------------------------------------------------------
STENCILS = {
    "5pt": [(0, dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if abs(dy) + abs(dx) <= 1],
    "9pt": [(0, dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
    "7pt": [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if abs(dz) + abs(dy) + abs(dx) <= 1],
    "27pt": [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
}


def grid_stencil(mx: int, my: int, mz: int, kind: str, keep: float = 1.0, seed: int = 0) -> CSR:
    n = mx * my * mz
    rng = rng_for(8, mx, my, mz, seed)
    offs = sorted(STENCILS[kind], key=lambda o: o[0] * mx * my + o[1] * mx + o[2])
    idx = np.arange(n, dtype=np.int64)
    x = idx % mx
    y = (idx // mx) % my
    z = idx // (mx * my)
    valid = []
    counts = np.zeros(n, dtype=np.int64)
    for (dz, dy, dx) in offs:
        ok = (x + dx >= 0) & (x + dx < mx) & (y + dy >= 0) & (y + dy < my) & (z + dz >= 0) & (z + dz < mz)
        if keep < 1.0 and (dz, dy, dx) != (0, 0, 0):
            ok &= rng.random(n) < keep
        valid.append(ok)
        counts += ok
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    colidx = np.empty(nnz, dtype=np.int32)
    start = rowptr[:-1].copy()
    for (dz, dy, dx), ok in zip(offs, valid):
        pos = start[ok]
        colidx[pos] = (idx[ok] + dz * mx * my + dy * mx + dx).astype(np.int32)
        start[ok] += 1
    return CSR(n, n, rowptr, colidx, rng.uniform(-1.0, 1.0, size=nnz))


def grid_scrambled(mx: int, my: int, mz: int, kind: str, seed: int = 0) -> CSR:
    """The grid operator of grid_stencil(mx, my, mz, kind) with its points
    numbered in a seeded random order instead of the natural one: point p
    carries the label lab[p], and every stencil pair (p, q) is the entry
    (lab[p], lab[q]). Values U[-1, 1]."""
    n = mx * my * mz
    rng = rng_for(11, mx, my, mz, seed)
    lab = rng.permutation(n).astype(np.int64)
    idx = np.arange(n, dtype=np.int64)
    x = idx % mx
    y = (idx // mx) % my
    z = idx // (mx * my)
    rows, cols = [], []
    for (dz, dy, dx) in STENCILS[kind]:
        ok = (x + dx >= 0) & (x + dx < mx) & (y + dy >= 0) & (y + dy < my) & (z + dz >= 0) & (z + dz < mz)
        p = idx[ok]
        rows.append(lab[p])
        cols.append(lab[p + dz * mx * my + dy * mx + dx])
    return _from_keys(n, n, np.concatenate(rows), np.concatenate(cols), rng)


def structured_matrix(index: int, min_rows: int = 50_000, max_rows: int = 4_000_000) -> tuple[str, CSR]:
    """Matrix `index` of the structured (grid operator) population."""
    rng = rng_for(50, index)
    kind = ("5pt", "9pt", "7pt", "27pt")[index % 4]
    n = float(np.exp(rng.uniform(np.log(min_rows), np.log(max_rows))))
    keep = 1.0 if rng.random() < 0.5 else float(rng.uniform(0.5, 1.0))
    if kind in ("5pt", "9pt"):
        mx = max(2, int(round(np.sqrt(n * rng.uniform(0.25, 4.0)))))
        my = max(2, int(round(n / mx)))
        mz = 1
    else:
        mx = max(2, int(round((n * rng.uniform(0.25, 4.0)) ** (1.0 / 3.0))))
        my = max(2, int(round(np.sqrt(n / mx * rng.uniform(0.5, 2.0)))))
        mz = max(2, int(round(n / (mx * my))))
    return f"stencil{kind}", grid_stencil(mx, my, mz, kind, keep, seed=int(rng.integers(0, 2**31)))


def batched_matrix(index: int, min_rows: int = 10_000, max_rows: int = 500_000) -> CSR:
    rng = rng_for(40, index)
    n = int(np.exp(rng.uniform(np.log(min_rows), np.log(max_rows))))
    return uniform_plus_3x3(n, 16.8, 2.4, seed=int(rng.integers(0, 2**31)))
