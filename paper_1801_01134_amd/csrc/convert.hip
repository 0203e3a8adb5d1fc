// CSR <-> beta(r,c) conversion on the device.
//
// The paper defines the format (Design, "Block-based storage without zero
// padding") but not how blocks are placed; here every interval of r rows is
// covered greedily from the left: the next block opens at the smallest
// column not yet covered. One thread walks one interval with r row cursors
// (an r-way merge of sorted column lists), first to count blocks, then, once
// the counts are scanned into block_rowptr, to write the blocks. The values
// of interval t keep the CSR range of its rows and are only reordered, so no
// value offsets have to be scanned: with r = 1 the values array is the CSR
// one, as the paper points out.
#include "common.hpp"
#include "cursor.hpp"

namespace spc {
namespace {

constexpr int kConvThreads = 256;

enum : int { kErrNone = 0, kErrRange = 1, kErrOrder = 2 };

// Row pointers must start at 0, never decrease and (when total >= 0) end at
// total. Run before anything reads through them.
__global__ void k_check_ptr(const int32_t *__restrict__ p, int64_t n, int64_t total, int *err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (i == 0) bad = p[0] != 0;
        else bad = p[i] < p[i - 1];
        if (i == n && total >= 0) bad = bad || p[n] != total;
        if (bad) atomicOr(err, 1 << kErrRange);
    }
}

// Checks the rows of one interval and counts its blocks. Each entry is read
// once, through the row's cursor, by the merge that places it in a block;
// the range and order checks are made on the way.
template <int R, int C>
__global__ __launch_bounds__(kConvThreads) void k_count(int64_t n_rows, int64_t n_cols,
                                                        const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx, int64_t nnz,
                                                        int32_t *__restrict__ counts, int *err) {
    const int64_t n_int = (n_rows + R - 1) / R;
    // whole wavefronts run the loop (the resource is per wavefront)
    const int64_t n_iter = (n_int + 63) & ~(int64_t)63;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_iter;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t_first = t - (threadIdx.x & 63);
        int64_t rel;
        const auto cr = dev::col_rsrc(colidx, nnz, rowptr[t_first * R], &rel);
        if (t >= n_int) continue;
        const int64_t row0 = t * R;
        const int nr = (int)min<int64_t>(R, n_rows - row0);
        dev::ColCursor cur[R];
        int32_t prev[R];
        int bad = kErrNone;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            int64_t a = 0, e = 0;
            if (i < nr) {
                a = rowptr[row0 + i];
                e = rowptr[row0 + i + 1];
                if (e < a || a < 0) {
                    bad = kErrRange;
                    e = a;
                }
            }
            cur[i].init(cr, (int32_t)(a + rel), (int32_t)(e + rel));
            prev[i] = INT32_MIN;
        }
        int32_t nb = 0;
        for (;;) {
            int64_t s = INT64_MAX;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (cur[i].live()) s = min(s, (int64_t)cur[i].cur());
            if (s == INT64_MAX) break;
            const int64_t lim = s + C;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                while (cur[i].live() && (int64_t)cur[i].cur() < lim) {
                    // columns strictly increasing inside [0, n_cols)
                    const int32_t v = cur[i].cur();
                    if (v < 0 || v >= n_cols) bad = bad ? bad : kErrRange;
                    else if (v <= prev[i]) bad = bad ? bad : kErrOrder;
                    prev[i] = v;
                    cur[i].next(cr);
                }
            }
            ++nb;
        }
        if (bad) {
            atomicOr(err, 1 << bad);
            nb = 0;
        }
        counts[t] = nb;
    }
}

__global__ void k_narrow(const int64_t *__restrict__ in, int64_t n, int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

template <int MB>
struct MaskWord;
template <> struct MaskWord<1> { using T = uint8_t; };
template <> struct MaskWord<2> { using T = uint16_t; };
template <> struct MaskWord<4> { using T = uint32_t; };

// A lane's run of consecutive outputs out[q0], out[q0 + 1], ... of type T:
// stored N at a time (one store of N elements per N-aligned group; out
// aligned to N * sizeof(T) bytes), the partial groups at the run's two ends
// one by one. The runs of a wavefront's 64 lanes lie far apart, so this
// cuts the memory transactions of its stores by N.
template <class T, int N>
struct Run {
    struct alignas(N * sizeof(T)) Pack {
        T v[N];
    };
    int64_t q0, q;
    T b[N];  // shift register: the latest element last (static indices only)
    __device__ __forceinline__ void init(int64_t start) { q0 = q = start; }
    __device__ __forceinline__ void put(T *__restrict__ out, T v) {
        if ((q & ~(int64_t)(N - 1)) < q0) {
            out[q] = v;  // the run's first group is partial
        } else {
#pragma unroll
            for (int j = 0; j + 1 < N; ++j) b[j] = b[j + 1];
            b[N - 1] = v;
            if ((q & (N - 1)) == N - 1) {
                Pack w;
#pragma unroll
                for (int j = 0; j < N; ++j) w.v[j] = b[j];
                *reinterpret_cast<Pack *>(out + (q - (N - 1))) = w;
            }
        }
        ++q;
    }
    // the last, partial group: its m elements are the last m of the register
    __device__ __forceinline__ void flush(T *__restrict__ out) {
        const int m = (int)(q & (N - 1));
        if (m != 0 && (q & ~(int64_t)(N - 1)) >= q0) {
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (j >= N - m) out[q - N + j] = b[j];
        }
    }
};

// Writes the blocks of one interval (column start and mask) and, for each
// position of the block-ordered values array (block order, row-major inside
// a block), the CSR entry whose value goes there. The values stay inside the
// CSR range of the interval's rows, so the move is a local permutation, done
// afterwards by k_permute (coalesced writes). A4: bcol is 16-byte aligned
// (its run is stored four at a time). The masks array is 8-byte aligned.
template <int R, int C, bool A4>
__global__ __launch_bounds__(kConvThreads) void k_fill(int64_t n_rows, const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ colidx, int64_t nnz,
                                                       const int32_t *__restrict__ brow,
                                                       int32_t *__restrict__ bcol, uint8_t *__restrict__ masks,
                                                       int32_t *__restrict__ src) {
    using Sh = Shape<R, C>;
    using MW = typename MaskWord<Sh::MB>::T;
    const int64_t n_int = (n_rows + R - 1) / R;
    const int64_t n_iter = (n_int + 63) & ~(int64_t)63;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_iter;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t_first = t - (threadIdx.x & 63);
        int64_t rel;
        const auto cr = dev::col_rsrc(colidx, nnz, rowptr[t_first * R], &rel);
        if (t >= n_int) continue;
        const int64_t row0 = t * R;
        const int nr = (int)min<int64_t>(R, n_rows - row0);
        dev::ColCursor cur[R];
#pragma unroll
        for (int i = 0; i < R; ++i)
            cur[i].init(cr, i < nr ? (int32_t)(rowptr[row0 + i] + rel) : 0,
                        i < nr ? (int32_t)(rowptr[row0 + i + 1] + rel) : 0);
        int64_t b = brow[t];
        // masks go up to four at a time (at most 8 bytes: the array is 8-byte aligned)
        constexpr int NM = sizeof(MW) == 4 ? 2 : 4;
        Run<int32_t, 4> vrun, brun;
        Run<MW, NM> mrun;
        vrun.init(rowptr[row0]);
        brun.init(b);
        mrun.init(b);
        for (;;) {
            int64_t s = INT64_MAX;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (cur[i].live()) s = min(s, (int64_t)cur[i].cur());
            if (s == INT64_MAX) break;
            const int64_t lim = s + C;
            uint32_t m = 0;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                while (cur[i].live() && (int64_t)cur[i].cur() < lim) {
                    const int32_t v = cur[i].cur();
                    m |= 1u << (i * C + (int)(v - s));
                    if (R > 1) vrun.put(src, (int32_t)((int64_t)cur[i].p - rel));
                    cur[i].next(cr);
                }
            }
            if (A4) brun.put(bcol, (int32_t)s);
            else bcol[b] = (int32_t)s;
            mrun.put(reinterpret_cast<MW *>(masks), (MW)m);
            ++b;
        }
        if (R > 1) vrun.flush(src);
        if (A4) brun.flush(bcol);
        mrun.flush(reinterpret_cast<MW *>(masks));
    }
}

// vout[o] = vals[src[o]], bit for bit (VT: unsigned integer of the value width).
template <class VT>
__global__ __launch_bounds__(kConvThreads) void k_permute(int64_t nnz, const int32_t *__restrict__ src,
                                                          const VT *__restrict__ vals, VT *__restrict__ vout) {
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nnz; o += (int64_t)gridDim.x * blockDim.x)
        vout[o] = vals[src[o]];
}

__global__ void k_zero_bytes(uint8_t *p, int64_t from, int64_t to) {
    int64_t i = from + threadIdx.x;
    if (i < to) p[i] = 0;
}

// ---- beta(r,c) -> CSR -------------------------------------------------------

// Per interval: entries of each of its rows, and the interval's value total.
template <int R, int C>
__global__ __launch_bounds__(kConvThreads) void k_decode_count(int64_t n_rows, const int32_t *__restrict__ brow,
                                                               const uint8_t *__restrict__ masks,
                                                               int32_t *__restrict__ row_cnt,
                                                               int64_t *__restrict__ int_cnt) {
    using Sh = Shape<R, C>;
    using MW = typename MaskWord<Sh::MB>::T;
    const int64_t n_int = (n_rows + R - 1) / R;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_int;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t rc[R];
        for (int i = 0; i < R; ++i) rc[i] = 0;
        int64_t tot = 0;
        for (int32_t b = brow[t]; b < brow[t + 1]; ++b) {
            uint32_t m = reinterpret_cast<const MW *>(masks)[b];
            tot += __popc(m);
            for (int i = 0; i < R; ++i) rc[i] += __popc((m >> (i * C)) & Sh::CMASK);
        }
        int_cnt[t] = tot;
        for (int i = 0; i < R; ++i)
            if (t * R + i < n_rows) row_cnt[t * R + i] = rc[i];
    }
}

template <int R, int C, class VT>
__global__ __launch_bounds__(kConvThreads) void k_decode_fill(int64_t n_rows, const int32_t *__restrict__ brow,
                                                              const int32_t *__restrict__ bcol,
                                                              const uint8_t *__restrict__ masks,
                                                              const VT *__restrict__ vals,
                                                              const int64_t *__restrict__ int_off,
                                                              const int64_t *__restrict__ row_off,
                                                              int32_t *__restrict__ col_out,
                                                              VT *__restrict__ val_out) {
    using Sh = Shape<R, C>;
    using MW = typename MaskWord<Sh::MB>::T;
    const int64_t n_int = (n_rows + R - 1) / R;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_int;
         t += (int64_t)gridDim.x * blockDim.x) {
        for (int i = 0; i < R; ++i) {
            const int64_t row = t * R + i;
            if (row >= n_rows) break;
            int64_t w = row_off[row];
            int64_t v = int_off[t];
            for (int32_t b = brow[t]; b < brow[t + 1]; ++b) {
                uint32_t m = reinterpret_cast<const MW *>(masks)[b];
                uint32_t sub = (m >> (i * C)) & Sh::CMASK;
                int64_t p = v + __popc(i ? (m & ((1u << (i * C)) - 1u)) : 0u);
                for (int k = 0; k < C; ++k) {
                    if ((sub >> k) & 1u) {
                        col_out[w] = bcol[b] + k;
                        val_out[w] = vals[p++];
                        ++w;
                    }
                }
                v += __popc(m);
            }
        }
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t g = div_up(n > 0 ? n : 1, kConvThreads);
    return (unsigned)(g > 65535 * 16 ? 65535 * 16 : g);
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_beta_count(int32_t r, int32_t c, int64_t n_rows, int64_t n_cols,
                                     const int32_t *rowptr, const int32_t *colidx,
                                     int32_t *block_rowptr_out, int64_t *n_blocks_out,
                                     hipStream_t stream) {
    const int s = shape_of(r, c);
    SPC_REQUIRE(s >= 0, SPC_ERR_UNSUPPORTED_SHAPE, "block shape (%d,%d) is not supported", r, c);
    SPC_REQUIRE(n_rows >= 0 && n_cols >= 0, SPC_ERR_INVALID_ARG, "negative matrix size");
    SPC_REQUIRE(n_rows < (int64_t(1) << 31) && n_cols < (int64_t(1) << 31), SPC_ERR_OVERFLOW,
                "matrix dimensions exceed the int32 index range");
    SPC_REQUIRE(block_rowptr_out && n_blocks_out, SPC_ERR_INVALID_ARG, "null output");
    SPC_REQUIRE(n_rows == 0 || (rowptr && colidx), SPC_ERR_INVALID_ARG, "null CSR array");
    const int64_t n_int = div_up(n_rows, r);
    DevBuf counts, scanned, temp, err;
    SPC_HIP(counts.alloc(sizeof(int32_t) * (n_int + 1)));
    SPC_HIP(scanned.alloc(sizeof(int64_t) * (n_int + 1)));
    SPC_HIP(temp.alloc(sizeof(int64_t) * scan_temp_elems(n_int)));
    SPC_HIP(err.alloc(sizeof(int)));
    SPC_HIP(hipMemsetAsync(err.p, 0, sizeof(int), stream));
    int herr = 0;
    int32_t nnz = 0;
    if (n_rows > 0) {
        hipLaunchKernelGGL(k_check_ptr, dim3(grid_for(n_rows + 1)), dim3(kConvThreads), 0, stream, rowptr,
                           n_rows, int64_t(-1), err.as<int>());
        SPC_HIP(hipGetLastError());
        SPC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipMemcpyAsync(&nnz, rowptr + n_rows, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipStreamSynchronize(stream));
        SPC_REQUIRE(herr == 0, SPC_ERR_INDEX_RANGE, "CSR row pointers do not start at 0 or decrease");
    }
    if (n_int > 0) {
        with_shape(s, [&](auto sh) {
            using Sh = decltype(sh);
            hipLaunchKernelGGL((k_count<Sh::R, Sh::C>), dim3(grid_for(n_int)), dim3(kConvThreads), 0,
                               stream, n_rows, n_cols, rowptr, colidx, (int64_t)nnz, counts.as<int32_t>(),
                               err.as<int>());
            return 0;
        });
        SPC_HIP(hipGetLastError());
    }
    spc_status st = scan_counts_i64(counts.as<int32_t>(), n_int, scanned.as<int64_t>(),
                                    temp.as<int64_t>(), stream);
    if (st != SPC_OK) return st;
    int64_t total = 0;
    SPC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipMemcpyAsync(&total, scanned.as<int64_t>() + n_int, sizeof(int64_t),
                           hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(!(herr & (1 << kErrRange)), SPC_ERR_INDEX_RANGE,
                "CSR row pointers not monotone or a column outside [0, n_cols)");
    SPC_REQUIRE(!(herr & (1 << kErrOrder)), SPC_ERR_CSR_UNSORTED_OR_DUP,
                "CSR row with unsorted or repeated column indices");
    SPC_REQUIRE(total < (int64_t(1) << 31), SPC_ERR_OVERFLOW,
                "%lld blocks exceed the int32 block index range", (long long)total);
    hipLaunchKernelGGL(k_narrow, dim3(grid_for(n_int + 1)), dim3(kConvThreads), 0, stream,
                       scanned.as<int64_t>(), n_int + 1, block_rowptr_out);
    SPC_HIP(hipGetLastError());
    SPC_HIP(hipStreamSynchronize(stream));
    *n_blocks_out = total;
    return SPC_OK;
}

extern "C" spc_status spc_csr_to_beta(int32_t r, int32_t c, int32_t dtype, int64_t n_rows, int64_t n_cols,
                                      const int32_t *rowptr, const int32_t *colidx, const void *values,
                                      const int32_t *block_rowptr, int32_t *block_colidx_out,
                                      void *block_masks_out, void *values_out, hipStream_t stream) {
    const int s = shape_of(r, c);
    SPC_REQUIRE(s >= 0, SPC_ERR_UNSUPPORTED_SHAPE, "block shape (%d,%d) is not supported", r, c);
    SPC_REQUIRE(dtype == SPC_F32 || dtype == SPC_F64, SPC_ERR_INVALID_ARG, "bad dtype %d", dtype);
    SPC_REQUIRE(n_rows >= 0 && n_cols >= 0, SPC_ERR_INVALID_ARG, "negative matrix size");
    (void)n_cols;
    const int64_t n_int = div_up(n_rows, r);
    if (n_int == 0) return SPC_OK;
    SPC_REQUIRE(rowptr && colidx && block_rowptr, SPC_ERR_INVALID_ARG, "null input array");
    SPC_REQUIRE(block_colidx_out && block_masks_out && values_out && values, SPC_ERR_INVALID_ARG,
                "null output array");
    SPC_REQUIRE((reinterpret_cast<uintptr_t>(block_masks_out) & 7u) == 0, SPC_ERR_INVALID_ARG,
                "block_masks_out must be 8-byte aligned");
    // block total, for zeroing the mask padding, and the entry count
    int32_t nb = 0, nnz = 0;
    SPC_HIP(hipMemcpyAsync(&nb, block_rowptr + n_int, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipMemcpyAsync(&nnz, rowptr + n_rows, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(nnz >= 0, SPC_ERR_INDEX_RANGE, "negative entry count in the row pointers");
    const int64_t used = (int64_t)nb * (r * c / 8), padded = spc_mask_bytes(r, c, nb);
    if (padded > used)
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(1024), 0, stream,
                           static_cast<uint8_t *>(block_masks_out), used, padded);
    // source entry of each value position (r > 1; with r = 1 the values keep
    // the CSR order)
    DevBuf srcmap;
    if (r > 1 && nnz > 0) SPC_HIP(srcmap.alloc(sizeof(int32_t) * (size_t)nnz));
    const bool a4 = (reinterpret_cast<uintptr_t>(block_colidx_out) & 15u) == 0;
    with_shape(s, [&](auto sh) {
        using Sh = decltype(sh);
        if (a4)
            hipLaunchKernelGGL((k_fill<Sh::R, Sh::C, true>), dim3(grid_for(n_int)), dim3(kConvThreads), 0, stream,
                               n_rows, rowptr, colidx, (int64_t)nnz, block_rowptr, block_colidx_out,
                               static_cast<uint8_t *>(block_masks_out), srcmap.as<int32_t>());
        else
            hipLaunchKernelGGL((k_fill<Sh::R, Sh::C, false>), dim3(grid_for(n_int)), dim3(kConvThreads), 0,
                               stream, n_rows, rowptr, colidx, (int64_t)nnz, block_rowptr, block_colidx_out,
                               static_cast<uint8_t *>(block_masks_out), srcmap.as<int32_t>());
        return 0;
    });
    SPC_HIP(hipGetLastError());
    const size_t es = dtype == SPC_F64 ? 8 : 4;
    if (nnz > 0) {
        if (r == 1) {
            SPC_HIP(hipMemcpyAsync(values_out, values, es * (size_t)nnz, hipMemcpyDeviceToDevice, stream));
        } else if (dtype == SPC_F64) {
            hipLaunchKernelGGL(k_permute<uint64_t>, dim3(grid_for(nnz)), dim3(kConvThreads), 0, stream,
                               (int64_t)nnz, srcmap.as<int32_t>(), static_cast<const uint64_t *>(values),
                               static_cast<uint64_t *>(values_out));
        } else {
            hipLaunchKernelGGL(k_permute<uint32_t>, dim3(grid_for(nnz)), dim3(kConvThreads), 0, stream,
                               (int64_t)nnz, srcmap.as<int32_t>(), static_cast<const uint32_t *>(values),
                               static_cast<uint32_t *>(values_out));
        }
        SPC_HIP(hipGetLastError());
    }
    // the source map is released on return: finish with it first
    if (r > 1 && nnz > 0) SPC_HIP(hipStreamSynchronize(stream));
    return SPC_OK;
}

extern "C" spc_status spc_beta_to_csr(const spc_beta_view *A, int32_t *rowptr_out, int32_t *colidx_out,
                                      void *values_out, hipStream_t stream) {
    spc_status st = check_view(A);
    if (st != SPC_OK) return st;
    SPC_REQUIRE(rowptr_out, SPC_ERR_INVALID_ARG, "null rowptr_out");
    SPC_REQUIRE(A->nnz == 0 || (colidx_out && values_out), SPC_ERR_INVALID_ARG, "null output");
    const int s = shape_of(A->r, A->c);
    const int64_t n = A->n_rows, n_int = div_up(n, A->r);
    DevBuf row_cnt, int_cnt, row_off, int_off, temp;
    SPC_HIP(row_cnt.alloc(sizeof(int32_t) * (n + 1)));
    SPC_HIP(int_cnt.alloc(sizeof(int64_t) * (n_int + 1)));
    SPC_HIP(row_off.alloc(sizeof(int64_t) * (n + 1)));
    SPC_HIP(int_off.alloc(sizeof(int64_t) * (n_int + 1)));
    SPC_HIP(temp.alloc(sizeof(int64_t) * scan_temp_elems(n > n_int ? n : n_int)));
    DevBuf err;
    SPC_HIP(err.alloc(sizeof(int)));
    SPC_HIP(hipMemsetAsync(err.p, 0, sizeof(int), stream));
    if (n_int > 0) {
        int herr = 0;
        hipLaunchKernelGGL(k_check_ptr, dim3(grid_for(n_int + 1)), dim3(kConvThreads), 0, stream,
                           A->block_rowptr, n_int, A->n_blocks, err.as<int>());
        SPC_HIP(hipGetLastError());
        SPC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipStreamSynchronize(stream));
        SPC_REQUIRE(herr == 0, SPC_ERR_INDEX_RANGE,
                    "block_rowptr does not run monotonically from 0 to n_blocks");
    }
    if (n_int > 0) {
        with_shape(s, [&](auto sh) {
            using Sh = decltype(sh);
            hipLaunchKernelGGL((k_decode_count<Sh::R, Sh::C>), dim3(grid_for(n_int)), dim3(kConvThreads), 0,
                               stream, n, A->block_rowptr, static_cast<const uint8_t *>(A->block_masks),
                               row_cnt.as<int32_t>(), int_cnt.as<int64_t>());
            return 0;
        });
        SPC_HIP(hipGetLastError());
    }
    if ((st = scan_counts_i64(row_cnt.as<int32_t>(), n, row_off.as<int64_t>(), temp.as<int64_t>(), stream)))
        return st;
    if ((st = scan_counts64_i64(int_cnt.as<int64_t>(), n_int, int_off.as<int64_t>(), temp.as<int64_t>(),
                                stream)))
        return st;
    int64_t total = 0, itotal = 0;
    SPC_HIP(hipMemcpyAsync(&total, row_off.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipMemcpyAsync(&itotal, int_off.as<int64_t>() + n_int, sizeof(int64_t), hipMemcpyDeviceToHost,
                           stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(total == A->nnz && itotal == A->nnz, SPC_ERR_INVALID_ARG,
                "mask bits count %lld entries (%lld in rows past n_rows) but the view says nnz = %lld",
                (long long)itotal, (long long)(itotal - total), (long long)A->nnz);
    hipLaunchKernelGGL(k_narrow, dim3(grid_for(n + 1)), dim3(kConvThreads), 0, stream, row_off.as<int64_t>(),
                       n + 1, rowptr_out);
    if (n_int > 0) {
        with_shape(s, [&](auto sh) {
            using Sh = decltype(sh);
            if (A->dtype == SPC_F64)
                hipLaunchKernelGGL((k_decode_fill<Sh::R, Sh::C, uint64_t>), dim3(grid_for(n_int)),
                                   dim3(kConvThreads), 0, stream, n, A->block_rowptr, A->block_colidx,
                                   static_cast<const uint8_t *>(A->block_masks),
                                   static_cast<const uint64_t *>(A->values), int_off.as<int64_t>(),
                                   row_off.as<int64_t>(), colidx_out, static_cast<uint64_t *>(values_out));
            else
                hipLaunchKernelGGL((k_decode_fill<Sh::R, Sh::C, uint32_t>), dim3(grid_for(n_int)),
                                   dim3(kConvThreads), 0, stream, n, A->block_rowptr, A->block_colidx,
                                   static_cast<const uint8_t *>(A->block_masks),
                                   static_cast<const uint32_t *>(A->values), int_off.as<int64_t>(),
                                   row_off.as<int64_t>(), colidx_out, static_cast<uint32_t *>(values_out));
            return 0;
        });
    }
    SPC_HIP(hipGetLastError());
    SPC_HIP(hipStreamSynchronize(stream));
    return SPC_OK;
}
