/*
 * spc5hip.h -- C ABI of the gfx950 (MI355X) library for the mask-block sparse
 * matrix-vector product of Bramas & Kus, "Computing the sparse matrix vector
 * product using block-based kernels without zero padding on processors with
 * AVX-512 instructions" (PeerJ Computer Science, 2018).
 *
 * Storage format beta(r,c) (Design, "Block-based storage without zero
 * padding", Eq. (1)): the matrix is cut into row intervals of r consecutive
 * rows; each interval is covered by r x c blocks that start at row t*r and at
 * any column. Per block the format keeps its left column and an r*c-bit mask;
 * the values are packed in block order, row-major inside a block, with no
 * padding. Supported shapes: (1,8) (2,4) (2,8) (4,4) (4,8) (8,4).
 *
 * Conventions for every entry point
 *   - Return value: SPC_OK (0) or a negative spc_status. No C++ exception
 *     crosses the ABI. spc_status_string() names a code; spc_last_error()
 *     gives the detail of the most recent failure in the calling thread.
 *   - Pointers are device pointers unless marked "host". They are owned by
 *     the caller and never freed or retained by the library, except that a
 *     plan (spc_plan, spc_batch) keeps the view it was built from: the caller
 *     keeps those arrays alive and unchanged while the plan is used.
 *   - Work is enqueued on the given HIP stream (NULL = default stream) and
 *     returns before it completes, unless the entry point says it
 *     synchronizes. Argument checks happen on the host before any launch.
 *   - Library-owned objects (plans, batches, selectors) are created by
 *     *_create and released by *_destroy.
 *   - Index types: int32 row pointers and column indices, as the paper's
 *     kernel uses (S_integer = 4 in Eq. (4)); int64 sizes and value offsets.
 */
#ifndef SPC5HIP_H
#define SPC5HIP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spc_status;
#define SPC_OK                       0
#define SPC_ERR_INVALID_ARG         -1  /* null pointer, negative size, bad flag, misaligned array */
#define SPC_ERR_UNSUPPORTED_SHAPE   -2  /* (r,c) is not one of the six shapes */
#define SPC_ERR_CSR_UNSORTED_OR_DUP -3  /* a CSR row has decreasing or repeated columns */
#define SPC_ERR_INDEX_RANGE         -4  /* column outside [0, n_cols) or row pointers not monotone */
#define SPC_ERR_OVERFLOW            -5  /* a count does not fit the int32 index type */
#define SPC_ERR_HIP                 -6  /* a HIP runtime call failed (detail in spc_last_error) */
#define SPC_ERR_NO_MODEL            -7  /* selector has no trained network; use interpolation */
#define SPC_ERR_CAPACITY            -8  /* a size exceeds a documented library limit */

typedef enum { SPC_F32 = 0, SPC_F64 = 1 } spc_dtype;

/* Shape indices used by the selector, in the paper's order of the six
 * optimized kernels (Design, "Optimized kernel implementation"). */
#define SPC_N_SHAPES 6
/* 0 = (1,8), 1 = (2,4), 2 = (2,8), 3 = (4,4), 4 = (4,8), 5 = (8,4) */

/* A beta(r,c) matrix as the caller's device arrays (a view; never freed).
 *   block_rowptr int32[ceil(n_rows/r) + 1]  prefix pointers: the blocks of
 *                interval t are block_rowptr[t] .. block_rowptr[t+1]-1
 *                (Algorithm 1 indexes it this way)
 *   block_colidx int32[n_blocks]  left column of each block (any column;
 *                a block may reach past n_cols, those bits are zero)
 *   block_masks  n_blocks masks of r*c bits stored as ceil(r*c/8)-byte
 *                little-endian words: bit i*c + k set <=> the block holds
 *                the entry (row t*r + i, column colidx + k). Bit 0 is the
 *                leftmost column, as in the vexpand example of the
 *                Vectorization section. The array must be 8-byte aligned and
 *                readable for spc_mask_bytes(r, c, n_blocks) bytes.
 *   values       nnz entries of dtype, block order, row-major in a block */
typedef struct spc_beta_view {
    int32_t r, c;
    int32_t dtype;          /* spc_dtype */
    int32_t reserved;
    int64_t n_rows, n_cols, nnz, n_blocks;
    const int32_t *block_rowptr;
    const int32_t *block_colidx;
    const void    *block_masks;
    const void    *values;
} spc_beta_view;

const char *spc_status_string(spc_status s);
const char *spc_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t spc_version(void);

/* Shape index 0..5 of (r,c), or SPC_ERR_UNSUPPORTED_SHAPE. */
spc_status spc_shape_index(int32_t r, int32_t c);

/* Bytes the masks array of n_blocks blocks must span: n_blocks*r*c/8
 * rounded up to a multiple of 8, plus 512 bytes that the kernels may read
 * (but never use) when they fetch a tile's mask words in one go. Returns -1
 * for an unsupported shape. */
int64_t spc_mask_bytes(int32_t r, int32_t c, int64_t n_blocks);

/* ---------------------------------------------------------------------------
 * Conversion CSR -> beta(r,c), on the device, in two calls so that the
 * caller can size the output arrays (storage section; the paper gives only
 * the format, so blocks are placed by the greedy leftmost cover: in each
 * interval the next block starts at the smallest column not yet covered,
 * which uses the fewest blocks).
 *
 * spc_beta_count: checks the CSR arrays (rowptr int32[n_rows+1] monotone from
 *   0, colidx int32[rowptr[n_rows]] strictly increasing inside each row and
 *   inside [0, n_cols)), counts the blocks of every interval and writes
 *   block_rowptr_out int32[ceil(n_rows/r)+1] as prefix pointers. Stores the
 *   block total in *n_blocks_out (host). Synchronizes the stream. Errors:
 *   SPC_ERR_CSR_UNSORTED_OR_DUP, SPC_ERR_INDEX_RANGE, SPC_ERR_OVERFLOW (more
 *   than 2^31-1 blocks), SPC_ERR_UNSUPPORTED_SHAPE, SPC_ERR_INVALID_ARG.
 *   n_rows == 0 writes block_rowptr_out[0] = 0 and returns 0 blocks.
 *
 * spc_csr_to_beta: fills block_colidx_out[n_blocks], block_masks_out
 *   (spc_mask_bytes bytes, padding zeroed) and values_out[nnz] (values are
 *   moved bit for bit; for r = 1 they keep the CSR order, as the paper notes)
 *   from the same CSR arrays and the block_rowptr of spc_beta_count.
 *   Asynchronous. */
spc_status spc_beta_count(int32_t r, int32_t c, int64_t n_rows, int64_t n_cols,
                          const int32_t *rowptr, const int32_t *colidx,
                          int32_t *block_rowptr_out, int64_t *n_blocks_out,
                          hipStream_t stream);
spc_status spc_csr_to_beta(int32_t r, int32_t c, int32_t dtype, int64_t n_rows, int64_t n_cols,
                           const int32_t *rowptr, const int32_t *colidx, const void *values,
                           const int32_t *block_rowptr, int32_t *block_colidx_out,
                           void *block_masks_out, void *values_out, hipStream_t stream);

/* beta(r,c) -> CSR on the device: rowptr_out int32[n_rows+1],
 * colidx_out int32[nnz], values_out[nnz] (bitwise). Synchronizes. */
spc_status spc_beta_to_csr(const spc_beta_view *A, int32_t *rowptr_out, int32_t *colidx_out,
                           void *values_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Reordering before conversion (section "Matrix permutation/reordering": a
 * Cuthill-McKee breadth-first renumbering puts coupled rows and columns side
 * by side, so that r x c blocks hold more values). For a square matrix.
 *
 * spc_rcm_order: reverse Cuthill-McKee order of the pattern of A + A^T
 *   (diagonal ignored) into perm_out (device int32[n], perm[new] = old).
 *   The order is fully defined: deg(v) = distinct neighbours of v; the
 *   search starts at the unnumbered vertex of smallest degree (smallest
 *   index on ties); each vertex taken off the queue numbers its unnumbered
 *   neighbours in (degree, index) order; an exhausted queue with vertices
 *   left restarts from a new start vertex; the final order is reversed. The
 *   walk runs on the host (the pattern is copied there once). rowptr int32
 *   [n+1], colidx int32[nnz] (device; rows need not be sorted). Errors:
 *   SPC_ERR_INDEX_RANGE (bad row pointers or columns), SPC_ERR_OVERFLOW.
 *   Synchronizes.
 * spc_csr_permute: B = P A P^T on the device: B[i][j] = A[perm[i]][perm[j]],
 *   rows of B with sorted columns, values (dtype) moved bit for bit.
 *   rowptr_out int32[n+1], colidx_out int32[nnz], values_out[nnz] (caller
 *   allocated). SPC_ERR_INDEX_RANGE if perm is not a permutation of 0..n-1.
 *   Synchronizes.
 * spc_permute_vector: scatter = 0: out[i] = in[perm[i]] (x' = P x);
 *   scatter = 1: out[perm[i]] = in[i] (y = P^T y'). So y = A x is
 *   spc_permute_vector(scatter 1) of B (spc_permute_vector(scatter 0) of x).
 *   in and out must not overlap. Asynchronous. */
spc_status spc_rcm_order(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                         int32_t *perm_out, hipStream_t stream);
spc_status spc_csr_permute(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                           int32_t dtype, const void *values, const int32_t *perm,
                           int32_t *rowptr_out, int32_t *colidx_out, void *values_out,
                           hipStream_t stream);
spc_status spc_permute_vector(int64_t n, int32_t dtype, const int32_t *perm, const void *in, void *out,
                              int32_t scatter, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Plans: the row-interval partition the kernels run on (Design,
 * "Parallelization": consecutive intervals grouped so that groups hold about
 * the same number of blocks and no interval is split). A tile is one such
 * group, processed by one workgroup; an interval with more blocks than a
 * tile holds becomes a tile of its own. Creating a plan reads block_rowptr
 * and the masks once and synchronizes the stream.
 *   tile_bits  mode 1: mask bits a tile may hold (blocks * r * c); 0 = 2048;
 *              one of 1024, 2048, 3072, 4032. Mode 0 sizes its tiles from
 *              wave_chunks instead: (64 * wave_chunks - 1) * (16 / value size)
 *              bits, so one wavefront's 16-byte loads cover a tile's values
 *   tile_order SPC_ORDER_XCD (0, the default): workgroup g runs on XCD
 *              g mod 8, so the launch renumbers tiles to give each of the 8
 *              XCDs one contiguous range of them (the x entries a range
 *              gathers then stay in that XCD's L2); SPC_ORDER_HW (1): tiles
 *              in the hardware's round-robin order (neighbouring tiles on
 *              different XCDs). Persistent (pipelined) launches ignore it.
 *   mode       0 = one wavefront per tile, four independent tiles per
 *              workgroup: all of a tile's streams are requested at once
 *              (values with 16-byte loads), x is gathered one lane per value;
 *              1 = one workgroup per tile, one lane per mask bit loads,
 *              gathers and multiplies (the direct form of the vexpand step);
 *              2 = "test" tiles (Algorithm 2, for beta(1,8) and beta(2,4)
 *              only, else SPC_ERR_UNSUPPORTED_SHAPE): one wavefront per tile
 *              as in mode 0, but a block holding a single value takes one
 *              lane and no expansion (its column from its bit's position),
 *              and only blocks with several values are expanded, one lane
 *              per mask bit of a compacted list. A tile holds up to
 *              248 blocks (fewer with 2 chunks, or 4 chunks and FP64 for
 *              beta(2,4)), at most 64 of them with several values, and no
 *              more values than mode 0's tile (planning reads the masks once);
 *              3 = block-row lanes: one wavefront per tile, lane =
 *              (block, block row): the lane walks that block row's set bits
 *              in turn, one x gather per stored value, and its sum is the
 *              block row's partial (mode 0 spends a lane per mask bit,
 *              stored or not). Tiles are sized by values: up to
 *              (64 * wave_chunks - 1) * (16 / value size) values and at most
 *              a per-shape block count (64 mask words, 4032 mask bits, and
 *              partials that fit the tile's LDS buffer); planning reads the
 *              masks once;
 *              4 = value lanes (beta(1,8) only, else
 *              SPC_ERR_UNSUPPORTED_SHAPE): mode 3's tiles; each block's
 *              columns are written to LDS at its values' ranks, then one
 *              lane per stored value gathers x and multiplies, and a row's
 *              products (contiguous, one row per block) are added. FP32:
 *              each product is rounded to float, the sums are in double.
 *              Modes 3 and 4 with values that are not 16-byte aligned run
 *              their tiles as 4032-bit workgroup tiles
 * params == NULL selects spc_plan_default_params(A); all zeros select mode 0
 * with 4 chunks per lane. */
typedef struct spc_plan spc_plan;
#define SPC_ORDER_XCD 0   /* tile_order: each XCD walks one contiguous range of tiles (default) */
#define SPC_ORDER_HW  1   /* tile_order: the hardware's round-robin of workgroups over the XCDs */
typedef struct spc_plan_params {
    int32_t tile_bits;
    int32_t tile_order;     /* SPC_ORDER_XCD (0) or SPC_ORDER_HW (1) */
    int32_t mode;           /* 0 = wavefront tiles (default), 1 = workgroup tiles, 2 = test tiles,
                               3 = block-row lanes, 4 = value lanes (beta(1,8)); see the plan
                               notes above */
    int32_t wave_chunks;    /* modes 0, 2, 3 and 4: 16-byte value chunks per lane, 2, 4, 6 or 8;
                               0 = 4 */
    int32_t pipeline;       /* mode 0: 0 = one wavefront per tile; 1 = persistent wavefronts (as
                               many workgroups as fit on the device) that load their next tile
                               while working on the current one; N > 1 = the same with at most N
                               workgroups */
    int32_t cu_groups;      /* modes 0, 2, 3 and 4, launches that are not persistent and SpMM: 0 = as many
                               workgroups per compute unit as fit; 2..8 = at most that many (the
                               launch reserves LDS to hold the others off). Fewer resident
                               wavefronts can keep more of the gathered rows of X in cache. */
    int32_t wave_tiles;     /* mode 0, not pipelined, single-vector products: 0 or 1 = one tile per
                               wavefront; 2 = two consecutive tiles per wavefront, the second one's
                               values held in registers while the first is worked on, so that both
                               tiles' loads are in flight together (same results, bit for bit) */
    int32_t spmm_path;      /* SpMM kernel: SPC_SPMM_AUTO (0), SPC_SPMM_BITS (1) or SPC_SPMM_ROWS (2);
                               see spc_spmm_beta */
} spc_plan_params;
#define SPC_SPMM_AUTO 0   /* spmm_path: the row path for rows of 64 bytes or more, else mask-bit lanes */
#define SPC_SPMM_BITS 1   /* spmm_path: lanes on mask bits, column groups taken in turn */
#define SPC_SPMM_ROWS 2   /* spmm_path: values sorted by row, lanes on rows and column groups */

spc_status spc_plan_create(const spc_beta_view *A, const spc_plan_params *params,
                           spc_plan **plan_out, hipStream_t stream);
/* The library's default parameters for a matrix, from its sizes alone (no
 * device access): mode 0, XCD order, no cap, and 8 chunks per lane from 16M
 * entries up, 4 from 1M, else 2 (larger tiles cost fewer per-tile steps,
 * smaller ones give small matrices enough wavefronts). They are not tuned:
 * spc_autotune picks among measured candidates. */
spc_status spc_plan_default_params(const spc_beta_view *A, spc_plan_params *params_out);
spc_status spc_plan_destroy(spc_plan *plan);
/* n_tiles, tiles taking the long-interval path, tile_bits actually used. */
spc_status spc_plan_info(const spc_plan *plan, int64_t *n_tiles, int64_t *n_long,
                         int32_t *tile_bits);

/* ---------------------------------------------------------------------------
 * y = A x (accumulate = 0) or y += A x (accumulate = 1; Algorithm 1 adds the
 * row sums into y). x: n_cols entries, y: n_rows entries, both of A's dtype.
 * Only stored entries touch y (an Inf or NaN in x under an unset mask bit
 * does not reach y). Rows with no entries get +0 when accumulate = 0.
 * Precision: FP64 forms every product and sum in double precision. FP32
 * forms each product, and the sum of the (at most c = 8) products of one
 * block row of one block, in single precision; those block-row sums are
 * added in double precision and the row is rounded to float once (plan
 * mode 4: products in single precision, every sum in double). The order
 * of additions is fixed by the plan, so repeated calls give identical bits.
 * plan: from spc_plan_create on this same A; or NULL, in which case the call
 * builds a plan with spc_plan_default_params(A), runs the product and
 * releases the plan: it then reads block_rowptr to the host and
 * synchronizes the stream (a convenience for one-off products; callers that
 * repeat products keep a plan). Asynchronous when plan is not NULL. */
spc_status spc_spmv_beta(const spc_beta_view *A, const spc_plan *plan, const void *x, void *y,
                         int32_t accumulate, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Y = A X (accumulate = 0) or Y += A X for k right-hand sides, 1 <= k <= 16.
 * X: n_cols x k and Y: n_rows x k, row-major with leading dimensions
 * ldx, ldy >= k (the k values of one row are contiguous), A's dtype. Each
 * Y entry is the plain definition sum_j a_ij X[j][q], summed in double
 * precision (FP32: products in FP32, sums in double). plan must be a mode-0
 * plan of A (wavefront tiles); values must be 16-byte aligned and X smaller
 * than 3.75 GiB. "Grouped" below means: k is a multiple of 16 / (value
 * size) and X, Y and their leading dimensions keep every such group of
 * columns 16-byte aligned. Two kernels, chosen by the plan's spmm_path:
 *   mask-bit lanes (SPC_SPMM_BITS): a tile's values stay on the lanes of
 *     their mask bits and the columns are taken in turn (one at a time, or
 *     one group at a time when grouped, with the same bits);
 *   row path (SPC_SPMM_ROWS, grouped only, else SPC_ERR_INVALID_ARG): a
 *     tile's values are sorted by row in LDS, then a row's 16-byte column
 *     groups go to lanes of their own, which walk the row's values in
 *     column order; each Y row is written whole, once.
 *   SPC_SPMM_AUTO takes the row path when grouped with rows of at least 64
 *   bytes (FP64 k >= 8, FP32 k = 16), else mask-bit lanes.
 * The two paths add in different orders (results within the same bound;
 * each path repeats its bits). k = 1 with unit leading dimensions runs the
 * single-vector kernel. plan NULL: as for spc_spmv_beta (a default plan is
 * built and released by the call, which then synchronizes). Asynchronous
 * when plan is not NULL. */
spc_status spc_spmm_beta(const spc_beta_view *A, const spc_plan *plan, int32_t k, const void *X,
                         int64_t ldx, void *Y, int64_t ldy, int32_t accumulate, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Conjugate gradients on k independent systems A X = B (A square and
 * symmetric positive definite, the caller's responsibility), started from
 * X = 0. Each iteration costs one spc_spmm_beta with k columns plus
 * column-wise dot products and updates; all scalars stay on the device.
 * Column q stops changing once ||r_q|| <= rel_tol * ||b_q|| (r the
 * recurrence residual). The host reads the stop flags every check_every
 * iterations and returns when all columns stopped or max_iter is reached.
 * use_graph = 1 captures one iteration in a HIP graph and replays it
 * (needs a non-NULL stream; with a NULL stream the iteration is launched
 * directly). workspace: device memory of spc_cg_workspace_bytes(n, k,
 * dtype) bytes, owned by the caller. On return (host arrays of k entries):
 * iters_out[q] = iteration at which column q met the tolerance (-1 if it did
 * not), rel_res_out[q] = ||r_q|| / ||b_q|| of the recurrence; total_iters_out
 * = iterations run. Synchronizes. */
int64_t spc_cg_workspace_bytes(int64_t n, int32_t k, int32_t dtype);
spc_status spc_cg_solve(const spc_beta_view *A, const spc_plan *plan, int32_t k, const void *B,
                        int64_t ldb, void *X, int64_t ldx, double rel_tol, int32_t max_iter,
                        int32_t check_every, int32_t use_graph, void *workspace,
                        int64_t workspace_bytes, int32_t *iters_out, double *rel_res_out,
                        int32_t *total_iters_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Timing records and autotuning (the record-based strategy of the paper's
 * contributions list: choices are made from timings of earlier runs).
 *
 * spc_time_spmv: average device time of one y = A x launch under `plan`,
 *   over `reps` launches after `warmup` launches, measured with HIP events
 *   on `stream` (microseconds, host *us_out). Synchronizes.
 *
 * spc_autotune: builds a plan for every candidate parameter set (mode 0
 *   with 2, 4, 6 and 8 chunks per lane, one wavefront per tile or
 *   pipelined, and with 4, 6 and 8 chunks also capped at 2 and 4 resident
 *   workgroups per compute unit; mode 1 with 1024, 2048, 3072 and 4032 tile
 *   bits; each in both tile orders where the grid order applies; mode 3
 *   with 2, 4, 6 and 8 chunks; for beta(1,8) also mode 4 with 2, 4, 6 and
 *   8 chunks; for beta(1,8) and beta(2,4) also mode 2 with 2, 4, 6 and 8
 *   chunks), times it
 *   with spc_time_spmv and returns the fastest set in *best and its time in
 *   *best_us. If records is not NULL, up to max_records timings are written
 *   there (host memory) and *n_records says how many. x and y are scratch
 *   vectors of A's dtype (n_cols and n_rows entries); y is overwritten.
 *   Synchronizes. */
typedef struct spc_tune_record {
    spc_plan_params params;
    float us;
    int32_t n_tiles;
} spc_tune_record;

spc_status spc_time_spmv(const spc_beta_view *A, const spc_plan *plan, const void *x, void *y,
                         int32_t warmup, int32_t reps, float *us_out, hipStream_t stream);
spc_status spc_autotune(const spc_beta_view *A, const void *x, void *y, int32_t reps,
                        spc_plan_params *best, float *best_us, spc_tune_record *records,
                        int32_t max_records, int32_t *n_records, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched products: y_i = A_i x_i (or y_i += A_i x_i) for `count` matrices
 * of uneven sizes and any of the six shapes. Each matrix is partitioned as
 * spc_plan_create would (whole intervals, about equal blocks per tile,
 * section "Parallelization") with its own parameters: mode 0 (wavefront
 * tiles), mode 3 (block-row lanes), for beta(1,8) mode 4 (value lanes), or
 * for beta(1,8) and beta(2,4) mode 2 (the test tiles of Algorithm 2), and
 * its own wave_chunks. Matrices of one (mode, shape,
 * chunk count) form a group; a product is one launch per group, of a kernel
 * built for that group, over the tiles of all its matrices.
 *
 * spc_batch_create: views (host array of count views, all of one dtype,
 *   values 16-byte aligned, x of each under 3.75 GiB, count < 2^29);
 *   params (host) with n_params = 0 (params unused: each matrix takes
 *   spc_plan_default_params), 1 (params[0] for every matrix) or count
 *   (params[i] for matrix i). Each set used must have mode 0, 2, 3 or 4
 *   (2 only for the one-byte-mask shapes, 4 only for beta(1,8)), pipeline 0
 *   and wave_tiles 0 or 1; its
 *   tile_order and cu_groups are not used. The batch keeps the views: their
 *   arrays must stay alive and unchanged. Synchronizes.
 * spc_batch_set_vectors: xs, ys = host arrays of count device pointers (x_i
 *   with n_cols_i entries, y_i with n_rows_i entries). Copies them to the
 *   batch's device table with a synchronous copy; do not call it while a
 *   batched launch of this batch is still running.
 * spc_spmv_batched: grid_blocks = 0 launches one wavefront per tile;
 *   grid_blocks > 0 caps each launch at that many workgroups, which loop
 *   over their group's tiles (persistent). use_graph = 1 captures the
 *   launches once in a HIP graph (needs a non-NULL stream; recaptured when
 *   accumulate or grid_blocks change) and replays it. Asynchronous.
 * spc_batch_set_kernel(batch, 1) runs the whole list instead as ONE launch
 *   of a kernel that switches on each tile's shape (its LDS is the largest
 *   shape's); it needs every matrix in mode 0 with one chunk count
 *   (SPC_ERR_INVALID_ARG otherwise); 0 restores the grouped launches.
 * spc_batch_info: tile and long-interval counts, the shape index shared by
 *   all matrices (-1 when shapes differ) and the number of groups. */
typedef struct spc_batch spc_batch;
spc_status spc_batch_create(int32_t count, const spc_beta_view *views, const spc_plan_params *params,
                            int32_t n_params, spc_batch **out, hipStream_t stream);
spc_status spc_batch_destroy(spc_batch *batch);
spc_status spc_batch_info(const spc_batch *batch, int64_t *n_tiles, int64_t *n_long, int32_t *single_shape,
                          int32_t *n_groups);
spc_status spc_batch_set_kernel(spc_batch *batch, int32_t general);
spc_status spc_batch_set_vectors(spc_batch *batch, const void *const *xs, void *const *ys);
spc_status spc_spmv_batched(spc_batch *batch, int32_t accumulate, int32_t grid_blocks, int32_t use_graph,
                            hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Matrix features for kernel selection, from the CSR structure alone (section
 * "Performance prediction and optimal kernel selection": the block counts
 * that drive the per-kernel prediction are obtained without converting).
 * rowptr int32[n_rows+1] (monotone from 0 to nnz) and colidx int32[nnz]
 * (strictly increasing in each row, inside [0, n_cols)) are device arrays.
 * features_out (host, 16 floats):
 *    0 log2(n_rows)       1 log2(n_cols)       2 log2(nnz + 1)
 *    3 mean entries per row                    4 std / mean of row lengths
 *    5 log2(1 + longest row)                   6 share of empty rows
 *    7 mean |j - i| over entries / max(n_rows, n_cols)
 *    8..13 Avg(r,c) = nnz / N_b(r,c) for the six shapes (0 if no block)
 *   14 share of beta(1,8) blocks that hold one value
 *   15 mean over non-empty rows of log2((last col - first col + 1) / length)
 * N_b(r,c) is the block count of the greedy leftmost cover, i.e. exactly
 * the n_blocks spc_beta_count returns. n_blocks_out (host, 6 entries, may be
 * NULL) receives them. Counts and sums are exact integers except entry 15
 * (double); the 16 entries are rounded to float once at the end.
 * Errors: SPC_ERR_INVALID_ARG (n_rows or n_cols < 1), SPC_ERR_INDEX_RANGE,
 * SPC_ERR_CSR_UNSORTED_OR_DUP, SPC_ERR_OVERFLOW. Synchronizes the stream. */
#define SPC_N_FEATURES 16
spc_status spc_matrix_features(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rowptr,
                               const int32_t *colidx, float *features_out, int64_t *n_blocks_out,
                               hipStream_t stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): spc_matrix_features without any
 * allocation. Same arguments, checks, results (bit for bit) and
 * synchronization. Its kernels work in a fixed 1 MiB device array that the
 * library holds on each GPU it runs on until the process ends, so it takes
 * at most spc_matrix_features_noalloc_max_rows() rows (about 19 million);
 * more return SPC_ERR_CAPACITY before any device work. Every call on one GPU
 * uses that GPU's array: calls that overlap on one GPU (other host threads
 * or other streams) race and must be serialized by the caller. The array
 * keeps the last call's contents; each call clears the part it relies on. */
spc_status spc_matrix_features_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rowptr,
                                       const int32_t *colidx, float *features_out, int64_t *n_blocks_out,
                                       hipStream_t stream);
int64_t spc_matrix_features_noalloc_max_rows(void);

/* ---------------------------------------------------------------------------
 * Kernel classes. The selectors choose among SPC_N_CLASSES kernels: classes
 * 0..5 are the six block shapes in SPC_SHAPE order, each run by its own
 * kernels (plan modes 0, 1 and 3); class 6 is the beta(1,8) "test" kernel and
 * class 7 the beta(2,4) "test" kernel (plan mode 2; Algorithm 2, and the
 * "test" rows of Table 3). A selector fitted on n_classes = 6 records
 * chooses among the shapes only. The Avg(r,c) of class k is feature
 * 8 + spc_class_shape(k).
 * ------------------------------------------------------------------------- */
#define SPC_N_CLASSES 8
#define SPC_CLASS_TEST_B1X8 6
#define SPC_CLASS_TEST_B2X4 7
/* Shape index (0..5) of class k (0..7), or -1 for any other k. */
int32_t spc_class_shape(int32_t k);
/* Plan mode the class runs in: 2 for the test classes, else -1 (the
 * shape's own modes 0, 1 and 3; the autotuner or the default plan chooses). */
int32_t spc_class_mode(int32_t k);

/* ---------------------------------------------------------------------------
 * Learned kernel selector: a 16 -> 64 -> 64 -> K ReLU network in FP32 whose
 * forward, backward and Adam steps run in this library's kernels, with
 * K = n_out = 6 (the shapes) or 8 (the kernel classes above). The paper
 * selects kernels from recorded speeds with one polynomial per kernel
 * (section "Performance polynomial interpolation") and names selection from
 * several matrix properties as future work (Conclusions); the network is
 * that extension. Definitions:
 *   x^   = (x - mu) / sd                 (per feature; training statistics)
 *   h1   = relu(W1 x^ + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3
 *   tau  = log2(t / min_k t_k)           (time relative to the best kernel)
 *   loss = mean over the batch and the K outputs of (o - tau)^2
 *   choice = argmin_k o_k (lowest index on ties)
 *   Adam: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected, constant lr.
 * params: SPC_MLP_PARAMS(K) floats, in this order, row-major [out][in]:
 *   W1[64][16], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].
 * X: n x 16 feature rows (float, row-major); times, tau: n x K.
 * n_out other than 6 or 8 is SPC_ERR_INVALID_ARG.
 * All arrays are device memory unless marked host. */
#define SPC_MLP_N_IN 16
#define SPC_MLP_N_HIDDEN 64
#define SPC_MLP_N_OUT 6
#define SPC_MLP_MAX_OUT 8
#define SPC_MLP_PARAMS(k) (SPC_MLP_N_HIDDEN * (SPC_MLP_N_IN + 1) + SPC_MLP_N_HIDDEN * (SPC_MLP_N_HIDDEN + 1) + \
                           (k) * (SPC_MLP_N_HIDDEN + 1))
#define SPC_MLP_N_PARAMS 5638 /* SPC_MLP_PARAMS(6); SPC_MLP_PARAMS(8) = 5768 */
#define SPC_MLP_MAX_BATCH 64

/* mu, sd (16 each): mean and population standard deviation of the columns
 * of X (sd < 1e-12 is replaced by 1). Asynchronous. */
spc_status spc_mlp_standardizer(const float *X, int32_t n, float *mu_out, float *sd_out, hipStream_t stream);
/* tau = log2(t / row minimum) for n rows of n_out positive times.
 * Asynchronous. */
spc_status spc_mlp_targets(const float *times, int32_t n, int32_t n_out, float *tau_out, hipStream_t stream);
/* Loss and gradient (SPC_MLP_PARAMS(n_out) floats) of one batch: rows
 * (host, batch entries in [0, n)) pick the batch from X and tau;
 * 1 <= batch <= 64. loss_out: one device float. Synchronizes. */
spc_status spc_mlp_loss_grad(const float *params, const float *mu, const float *sd, const float *X,
                             const float *tau, int32_t n, int32_t n_out, const int32_t *rows, int32_t batch,
                             float *grad_out, float *loss_out, hipStream_t stream);
/* n_steps Adam steps, step s on the rows order[s*batch .. s*batch+batch-1]
 * (host array, entries in [0, n)). params, adam_m, adam_v (each
 * SPC_MLP_PARAMS(n_out) floats) are updated in place; step0 = Adam steps
 * already taken (bias correction continues from there). losses_out[s] =
 * loss of step s before its update. One workgroup runs all steps in one
 * launch. Synchronizes. */
spc_status spc_mlp_train(float *params, float *adam_m, float *adam_v, int32_t step0, float lr,
                         const float *mu, const float *sd, const float *X, const float *tau, int32_t n,
                         int32_t n_out, const int32_t *order, int32_t n_steps, int32_t batch, float *losses_out,
                         hipStream_t stream);
/* Scores (n x n_out, may be NULL) and choices (n, may be NULL) for n
 * feature rows. Asynchronous. */
spc_status spc_mlp_infer(const float *params, const float *mu, const float *sd, const float *X, int32_t n,
                         int32_t n_out, float *scores_out, int32_t *choice_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Selector object (library-owned). Interpolation: per kernel class, a
 * least-squares polynomial of speed against Avg(r,c) over n records (avg,
 * speed: host n x n_classes doubles, n_classes 6 or 8, speed in GFlop/s),
 * degree lowered to (distinct Avg values - 1) when records are few; a
 * query's Avg (feature 8 + spc_class_shape(k)) is clamped to the fitted
 * range and the highest predicted speed wins (lowest index on ties).
 * MLP: spc_selector_set_mlp copies a trained network with n_out outputs
 * (host arrays) to the current device; the smallest score wins.
 * spc_select_kernel: features = host float[16] (spc_matrix_features);
 * method SPC_SEL_INTERP or SPC_SEL_MLP; *class_out = the chosen class, in
 * 0..n-1 for a model of n classes; scores_out (host float[SPC_N_CLASSES],
 * may be NULL; the first n entries are written) = predicted GFlop/s
 * (interpolation) or predicted log2 time ratios (MLP). SPC_ERR_NO_MODEL
 * when the method has no model, so the caller can fall back to the other
 * one. Synchronizes (MLP). */
#define SPC_SEL_INTERP 0
#define SPC_SEL_MLP 1
typedef struct spc_selector spc_selector;
spc_status spc_selector_create(spc_selector **out);
spc_status spc_selector_destroy(spc_selector *sel);
spc_status spc_selector_fit_interp(spc_selector *sel, int32_t n, int32_t n_classes, const double *avg,
                                   const double *speed, int32_t degree);
/* Coefficients (host SPC_N_CLASSES x 4 doubles, lowest power first, zero
 * above the degree) and fitted Avg ranges (host SPC_N_CLASSES doubles each,
 * may be NULL) of the first *n_classes_out rows. */
spc_status spc_selector_interp_coeffs(const spc_selector *sel, double *coeffs_out, double *lo_out,
                                      double *hi_out, int32_t *n_classes_out);
/* Number of classes the method's model chooses among (0 without a model). */
int32_t spc_selector_n_classes(const spc_selector *sel, int32_t method);
spc_status spc_selector_set_mlp(spc_selector *sel, int32_t n_out, const float *params, const float *mu,
                                const float *sd);
spc_status spc_select_kernel(spc_selector *sel, const float *features, int32_t method, int32_t *class_out,
                             float *scores_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Parallel performance estimation (section "Parallel performance
 * estimation": a non-linear regression of performance on two inputs, the
 * average values per block and the number of threads). On the GPU the
 * second input is the share of the compute units a product runs on.
 *
 * spc_stream_create_cu: a stream whose kernels run on n_cus of the current
 *   device's compute units (1 <= n_cus <= spc_device_cu_count(); on a
 *   256-unit device a multiple of 8, the same number on each of its 8 XCDs),
 *   spread evenly over the XCDs; the stream has the default priority.
 *   Release it with spc_stream_destroy.
 * spc_selector_fit_interp2d: per shape, least squares of speed (GFlop/s,
 *   host n x 6) on the tensor polynomial sum_{i<=deg_avg, j<=deg_share}
 *   c_ij Avg^i u^j, with u = log2_share[k] (host n) the log2 of the share
 *   record k ran on (0 = all units). deg_avg <= 3, deg_share <= 2; degrees
 *   drop when the records hold fewer distinct values, or fewer records than
 *   coefficients (the share degree first).
 * spc_selector_interp2d_coeffs: c_ij (host 6 x 4 x 3 doubles, [shape][i][j],
 *   zero above the degrees), the fitted Avg range per shape (host 6 each,
 *   may be NULL) and the fitted u range (host 2, may be NULL).
 * spc_select_kernel_at: the shape of highest predicted speed for a feature
 *   vector (host float[16]) at a share in (0, 1]; Avg and u are clamped to
 *   the fitted ranges; scores_out (host float[6], may be NULL) = predicted
 *   GFlop/s. SPC_ERR_NO_MODEL without a 2-D fit. */
spc_status spc_stream_create_cu(int32_t n_cus, hipStream_t *stream_out);
spc_status spc_stream_destroy(hipStream_t stream);
int32_t spc_device_cu_count(void);
spc_status spc_selector_fit_interp2d(spc_selector *sel, int32_t n, const double *avg, const double *log2_share,
                                     const double *speed, int32_t deg_avg, int32_t deg_share);
spc_status spc_selector_interp2d_coeffs(const spc_selector *sel, double *coeffs_out, double *lo_out,
                                        double *hi_out, double *share_range_out);
spc_status spc_select_kernel_at(spc_selector *sel, const float *features, double cu_share, int32_t *shape_out,
                                float *scores_out);

#ifdef __cplusplus
}
#endif
#endif /* SPC5HIP_H */
