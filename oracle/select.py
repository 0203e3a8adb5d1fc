"""Oracle for kernel selection: matrix features, the polynomial-interpolation
selector and the regret of a choice (section "Performance prediction and
optimal kernel selection", subsection "Performance polynomial interpolation",
and Table 3's speed difference). TEST INFRASTRUCTURE ONLY.

Feature vector (16 entries, FP64 here; the GPU computes them in FP32):

  0  log2(n_rows)                 8-13  Avg(r,c) = NNZ / N_blocks(r,c) for the six
  1  log2(n_cols)                       shapes (1,8) (2,4) (2,8) (4,4) (4,8) (8,4),
  2  log2(nnz + 1)                      0 when there are no blocks
  3  mean nnz per row             14    share of beta(1,8) blocks holding one value
  4  std / mean of nnz per row    15    mean over non-empty rows of
  5  log2(1 + max nnz per row)          log2((last col - first col + 1) / nnz_row)
  6  share of empty rows
  7  mean |j - i| / max(n_rows, n_cols) over the stored entries

Entries 8-13 are the quantity the paper computes "without conversion" to
feed its per-kernel interpolation; the rest are cheap statistics of the row
pointer and column arrays, the multi-input direction the conclusion names.
"""
from __future__ import annotations

import numpy as np

from . import SHAPES, beta_count, csr_to_beta

N_FEATURES = 16


def features(csr) -> np.ndarray:
    f = np.zeros(N_FEATURES, dtype=np.float64)
    n, m, nnz = csr.n_rows, csr.n_cols, csr.nnz
    lens = np.diff(csr.rowptr.astype(np.int64)).astype(np.float64)
    f[0] = np.log2(n)
    f[1] = np.log2(m)
    f[2] = np.log2(nnz + 1.0)
    mean = nnz / n
    f[3] = mean
    f[4] = (np.sqrt(np.mean((lens - mean) ** 2)) / mean) if mean > 0 else 0.0
    f[5] = np.log2(1.0 + lens.max())
    f[6] = float(np.count_nonzero(lens == 0)) / n
    if nnz:
        rows = np.repeat(np.arange(n, dtype=np.int64), lens.astype(np.int64))
        f[7] = float(np.mean(np.abs(csr.colidx.astype(np.int64) - rows))) / max(n, m)
    for k, (r, c) in enumerate(SHAPES):
        nb = int(beta_count(csr, r, c).sum())
        f[8 + k] = nnz / nb if nb else 0.0
    if nnz:
        b = csr_to_beta(csr, 1, 8)
        pc = np.array([int(v).bit_count() for v in b.masks]) if b.masks.size < 1 << 16 else \
            np.unpackbits(b.masks.view(np.uint8).reshape(-1, 4), axis=1).sum(axis=1)
        f[14] = float(np.count_nonzero(pc == 1)) / b.masks.size
        ne = lens > 0
        first = csr.colidx[csr.rowptr[:-1][ne]].astype(np.float64)
        last = csr.colidx[csr.rowptr[1:][ne] - 1].astype(np.float64)
        f[15] = float(np.mean(np.log2((last - first + 1.0) / lens[ne])))
    return f


class Interpolation:
    """Per-kernel polynomial of speed against Avg(r,c), fitted by least squares
    on recorded runs; a new matrix gets each kernel's predicted speed from its
    own Avg (clamped to the fitted range) and the fastest prediction wins."""

    def __init__(self, coeffs, lo, hi, degree):
        self.coeffs = coeffs  # list of numpy polyfit coefficient arrays (highest first)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.degree = degree

    def predict(self, avg) -> np.ndarray:
        avg = np.clip(np.asarray(avg, dtype=np.float64), self.lo, self.hi)
        return np.array([np.polyval(self.coeffs[k], avg[k]) for k in range(len(self.coeffs))])

    def select(self, avg) -> int:
        p = self.predict(avg)
        return int(np.argmax(p))  # argmax returns the lowest index on ties


def fit_interpolation(avgs: np.ndarray, speeds: np.ndarray, degree: int = 3) -> Interpolation:
    """avgs, speeds: [n_matrices, 6]. Degree drops when records are few."""
    avgs = np.asarray(avgs, dtype=np.float64)
    speeds = np.asarray(speeds, dtype=np.float64)
    coeffs, lo, hi = [], [], []
    for k in range(avgs.shape[1]):
        a, s = avgs[:, k], speeds[:, k]
        d = int(min(degree, max(0, len(np.unique(a)) - 1)))
        coeffs.append(np.polyfit(a, s, d))
        lo.append(a.min())
        hi.append(a.max())
    return Interpolation(coeffs, lo, hi, degree)


class Interpolation2D:
    """Per-kernel polynomial of speed against two inputs (section "Parallel
    performance estimation": the average values per block and the amount of
    parallel hardware, here u = log2 of the share of compute units used):
    sum over i <= da, j <= du of c[i, j] Avg^i u^j, fitted by least squares.
    A query's Avg and u are clamped to the fitted ranges; the fastest
    prediction wins (lowest index on ties)."""

    def __init__(self, coeffs, lo, hi, ulo, uhi):
        self.coeffs = coeffs          # list of 2-D arrays c[i, j]
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.ulo, self.uhi = float(ulo), float(uhi)

    def predict(self, avg, share) -> np.ndarray:
        a = np.clip(np.asarray(avg, dtype=np.float64), self.lo, self.hi)
        u = min(max(np.log2(share), self.ulo), self.uhi)
        out = []
        for k, c in enumerate(self.coeffs):
            out.append(sum(c[i, j] * a[k] ** i * u ** j for i in range(c.shape[0]) for j in range(c.shape[1])))
        return np.array(out)

    def select(self, avg, share) -> int:
        return int(np.argmax(self.predict(avg, share)))


def fit_interpolation_2d(avgs, log2_shares, speeds, deg_avg: int = 3, deg_share: int = 2) -> Interpolation2D:
    """avgs, speeds: [n, 6]; log2_shares: [n]. Degrees drop when the records
    hold fewer distinct values than a degree needs, and then (share degree
    first) while there are more coefficients than records."""
    avgs = np.asarray(avgs, dtype=np.float64)
    speeds = np.asarray(speeds, dtype=np.float64)
    u = np.asarray(log2_shares, dtype=np.float64)
    n = avgs.shape[0]
    du0 = min(deg_share, len(np.unique(u)) - 1)
    coeffs, lo, hi = [], [], []
    for k in range(avgs.shape[1]):
        a, s = avgs[:, k], speeds[:, k]
        da, du = min(deg_avg, max(0, len(np.unique(a)) - 1)), du0
        while (da + 1) * (du + 1) > n:
            if du > 0:
                du -= 1
            else:
                da -= 1
        V = np.stack([a ** i * u ** j for i in range(da + 1) for j in range(du + 1)], axis=1)
        c, *_ = np.linalg.lstsq(V, s, rcond=None)
        coeffs.append(c.reshape(da + 1, du + 1))
        lo.append(a.min())
        hi.append(a.max())
    return Interpolation2D(coeffs, lo, hi, u.min(), u.max())


def regret(times_row, chosen: int) -> float:
    """t_selected / t_best - 1 (the time form of Table 3's speed difference)."""
    t = np.asarray(times_row, dtype=np.float64)
    return float(t[chosen] / t.min() - 1.0)


def best_kernel(times_row) -> int:
    return int(np.argmin(np.asarray(times_row, dtype=np.float64)))


def fill_ratio(avg: float, r: int, c: int) -> float:
    """Share of the r*c slots of a block that hold a value (Table 1's percent)."""
    return float(avg) / (r * c)
