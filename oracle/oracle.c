/*
 * CPU oracle for the mask-block sparse matrix-vector product (Bramas & Kus,
 * "Computing the sparse matrix vector product using block-based kernels
 * without zero padding on processors with AVX-512 instructions").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library links or calls this file;
 * only the tests, the smoke check and the benchmark's CPU baseline do. It is
 * deliberately plain: no blocking, no vector code, one obvious loop per
 * definition, everything in double precision.
 *
 * Contents
 *   oracle_csr_spmv   y = A x over CSR (Background, CSR paragraph: row i holds
 *                     entries rowptr[i] .. rowptr[i+1]-1), plus s_i = sum |a_ij x_j|.
 *   oracle_csr_spmm   Y = A X for k right-hand sides, same definition per column.
 *   oracle_beta_count number of r x c blocks per row interval under the greedy
 *                     leftmost cover (reading of the storage section: blocks are
 *                     row-aligned, start at any column).
 *   oracle_beta_fill  the four arrays of the beta(r,c) format: values in block
 *                     order and row-major inside a block (storage section),
 *                     block_colidx, block_rowptr (prefix pointers), masks with
 *                     bit i*c+k for (row i, column k) of the block.
 *   oracle_beta_decode beta(r,c) back to CSR (inverse of the above).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops that follow (the CPU baseline times one and
 * all host threads); n < 1 leaves the setting alone. */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* y_i = sum_j a_ij x_j, summed left to right in column order, and
 * s_i = sum_j |a_ij x_j|. Rows are independent, so they are spread over
 * threads without changing any row's summation order. */
void oracle_csr_spmv(int64_t n_rows, const int32_t *rowptr, const int32_t *colidx,
                     const double *values, const double *x, double *y, double *s) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n_rows; ++i) {
        double acc = 0.0, aacc = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double t = values[p] * x[colidx[p]];
            acc += t;
            aacc += fabs(t);
        }
        y[i] = acc;
        if (s) s[i] = aacc;
    }
}

/* Y[i][q] = sum_j a_ij X[j][q] for q < k; X and Y row-major with leading
 * dimensions ldx, ldy. S (optional) gets sum_j |a_ij X[j][q]|. */
void oracle_csr_spmm(int64_t n_rows, const int32_t *rowptr, const int32_t *colidx,
                     const double *values, int k, const double *X, int64_t ldx,
                     double *Y, int64_t ldy, double *S) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n_rows; ++i) {
        for (int q = 0; q < k; ++q) {
            double acc = 0.0, aacc = 0.0;
            for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                double t = values[p] * X[(int64_t)colidx[p] * ldx + q];
                acc += t;
                aacc += fabs(t);
            }
            Y[i * ldy + q] = acc;
            if (S) S[i * ldy + q] = aacc;
        }
    }
}

/* Greedy leftmost cover of one row interval: the rows t*r .. t*r+r-1 (clipped
 * to n_rows). Let U be the sorted union of their column indices. Repeatedly
 * open a block at s = min U, covering columns s .. s+c-1, and drop those
 * columns from U. Returns the number of blocks; when the output pointers are
 * given, also writes each block's column start, its mask and, for each stored
 * value in block order (row-major inside the block, ascending columns in a
 * row), the CSR position it comes from. */
static int64_t cover_interval(int r, int c, int64_t n_rows, int64_t t,
                              const int32_t *rowptr, const int32_t *colidx,
                              int32_t *bcol, uint32_t *bmask, int64_t *src_out) {
    int64_t row0 = t * r;
    int nr = (int)((row0 + r <= n_rows) ? r : (n_rows - row0));
    int32_t head[8], end[8];
    for (int i = 0; i < nr; ++i) {
        head[i] = rowptr[row0 + i];
        end[i] = rowptr[row0 + i + 1];
    }
    int64_t nb = 0;
    for (;;) {
        /* s = smallest column not yet covered among the interval's rows */
        int64_t s = -1;
        for (int i = 0; i < nr; ++i)
            if (head[i] < end[i] && (s < 0 || colidx[head[i]] < s)) s = colidx[head[i]];
        if (s < 0) break;
        uint32_t mask = 0;
        for (int i = 0; i < nr; ++i) {
            while (head[i] < end[i] && colidx[head[i]] < s + c) {
                int k = (int)(colidx[head[i]] - s);
                mask |= 1u << (i * c + k);
                if (src_out) *src_out++ = head[i];
                head[i]++;
            }
        }
        if (bcol) bcol[nb] = (int32_t)s;
        if (bmask) bmask[nb] = mask;
        nb++;
    }
    return nb;
}

/* counts[t] = blocks of interval t, for t < ceil(n_rows / r). */
void oracle_beta_count(int r, int c, int64_t n_rows, const int32_t *rowptr,
                       const int32_t *colidx, int64_t *counts) {
    int64_t n_int = (n_rows + r - 1) / r, t;
#pragma omp parallel for schedule(dynamic, 1024)
    for (t = 0; t < n_int; ++t)
        counts[t] = cover_interval(r, c, n_rows, t, rowptr, colidx, NULL, NULL, NULL);
}

/* Fills the beta(r,c) index arrays given block_rowptr (prefix sums of the
 * counts). The values of interval t occupy the same range as the CSR values
 * of its rows, rowptr[t*r] .. rowptr[min(t*r+r, n_rows)], only reordered:
 * perm[p] is the CSR position of the value stored at p, so the packed values
 * are values[perm] bit for bit, whatever the value type. Masks are returned
 * widened to 32 bits (bit i*c + k <-> row i, column k of the block). */
void oracle_beta_fill(int r, int c, int64_t n_rows, const int32_t *rowptr,
                      const int32_t *colidx, const int64_t *block_rowptr,
                      int32_t *block_colidx, uint32_t *block_masks, int64_t *perm) {
    int64_t n_int = (n_rows + r - 1) / r, t;
#pragma omp parallel for schedule(dynamic, 1024)
    for (t = 0; t < n_int; ++t) {
        int64_t b0 = block_rowptr[t];
        cover_interval(r, c, n_rows, t, rowptr, colidx, block_colidx + b0,
                       block_masks + b0, perm + rowptr[t * r]);
    }
}

/* beta(r,c) -> CSR. Walks Algorithm 1's loop structure: intervals, then the
 * blocks of the interval, keeping a running value cursor advanced by the
 * popcount of each mask; each set bit i*c+k is entry (t*r+i, col+k). The
 * per-row entries are emitted in ascending column order, which is the block
 * order because blocks of one interval never overlap and ascend. src_out[w]
 * is the packed-value position of CSR entry w (values_csr = packed[src_out]). */
int oracle_beta_decode(int r, int c, int64_t n_rows, const int64_t *block_rowptr,
                       const int32_t *block_colidx, const uint32_t *block_masks,
                       int32_t *rowptr_out, int32_t *colidx_out, int64_t *src_out) {
    int64_t n_int = (n_rows + r - 1) / r;
    int64_t cursor = 0, w = 0;
    rowptr_out[0] = 0;
    for (int64_t t = 0; t < n_int; ++t) {
        /* value index of block b's first value inside this interval */
        int64_t nb = block_rowptr[t + 1] - block_rowptr[t];
        int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (nb ? nb : 1));
        if (!start) return -1;
        int64_t cur = cursor;
        for (int64_t b = 0; b < nb; ++b) {
            start[b] = cur;
            cur += __builtin_popcount(block_masks[block_rowptr[t] + b]);
        }
        for (int i = 0; i < r; ++i) {
            int64_t row = t * r + i;
            for (int64_t b = 0; b < nb; ++b) {
                uint32_t m = block_masks[block_rowptr[t] + b];
                /* values of rows above i inside this block come first */
                int64_t v = start[b] + __builtin_popcount(i > 0 ? (m & ((1u << (i * c)) - 1u)) : 0u);
                for (int k = 0; k < c; ++k) {
                    if (m & (1u << (i * c + k))) {
                        if (row >= n_rows) { free(start); return -2; }
                        colidx_out[w] = block_colidx[block_rowptr[t] + b] + k;
                        src_out[w] = v++;
                        w++;
                    }
                }
            }
            if (row < n_rows) rowptr_out[row + 1] = (int32_t)w;
        }
        cursor = cur;
        free(start);
    }
    return 0;
}
