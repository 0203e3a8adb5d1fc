// Matrix features for kernel selection, computed from the CSR structure
// without building any beta(r,c) array (section "Performance prediction and
// optimal kernel selection": the per-kernel block counts are obtained
// without conversion, so the prediction stays cheap).
//
// One thread takes a group of 8 consecutive rows. For every shape it runs the
// greedy leftmost cover of the group's intervals (r = 8: the group; r = 4:
// its two halves; r = 2: its four pairs; r = 1: each row): the next block
// starts at the smallest column not yet covered and spans c columns, which is
// the cover the conversion builds, so the counts equal the converted N_b.
// The same pass checks the CSR and takes the row statistics. Per-block
// partial sums are combined by one block in a fixed order, so the result
// does not depend on scheduling.
#include <climits>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "cursor.hpp"

// Scratch of the entry point that allocates nothing: the per-block partials,
// the total and the error flag of one call. Every GPU holds its own copy for
// the life of the process; host code reaches it only through the address
// hipGetSymbolAddress gives on that device (the name itself is a host-side
// stand-in, not a device address).
static constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) int64_t scratch[kScratchBytes / 8];

namespace spc {
namespace {

constexpr int kFT = 256;     // threads per block
constexpr int kGroup = 8;    // rows per thread (the tallest shape)

enum : int { kErrNone = 0, kErrRange = 1, kErrOrder = 2 };

// Partial sums of one block (all integers exact; the log term in double).
struct FeatSums {
    int64_t nb[SPC_N_SHAPES];  // greedy block counts per shape
    int64_t single18;          // beta(1,8) blocks holding one value
    int64_t empty_rows;
    int64_t sum_len2;          // sum of squared row lengths
    int64_t sum_dist;          // sum over entries of |j - i|
    int64_t max_len;
    int64_t nonempty_rows;
    double sum_log_span;       // sum over non-empty rows of log2(span / length)
    double pad;
};
constexpr int kSumWords = sizeof(FeatSums) / 8;
static_assert(sizeof(FeatSums) == 14 * 8, "FeatSums layout");

// Greedy cover of NR consecutive rows (first row F of the group) with blocks
// c columns wide. lo/hi: the rows' ranges in colidx (hi == lo for rows that
// do not exist or were refused); rel turns an entry index into a position in
// the wavefront's column resource cr.
template <int NR, int F, int C>
__device__ __forceinline__ int64_t cover(__amdgpu_buffer_rsrc_t cr, int64_t rel, const int (&lo)[kGroup],
                                         const int (&hi)[kGroup]) {
    dev::ColCursor cur[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) cur[r].init(cr, (int32_t)(lo[F + r] + rel), (int32_t)(hi[F + r] + rel));
    int64_t count = 0;
    int64_t end = INT64_MIN;  // first column not covered by the last block
    while (true) {
        int64_t s = INT64_MAX;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            while (cur[r].live() && (int64_t)cur[r].cur() < end) cur[r].next(cr);
            if (cur[r].live()) s = min(s, (int64_t)cur[r].cur());
        }
        if (s == INT64_MAX) break;
        ++count;
        end = s + C;
    }
    return count;
}

template <int NR, int C, int G>
__device__ __forceinline__ int64_t cover_all(__amdgpu_buffer_rsrc_t cr, int64_t rel, const int (&lo)[kGroup],
                                             const int (&hi)[kGroup]) {
    if constexpr (G * NR >= kGroup) {
        return 0;
    } else {
        return cover<NR, G * NR, C>(cr, rel, lo, hi) + cover_all<NR, C, G + 1>(cr, rel, lo, hi);
    }
}

__device__ void block_reduce(FeatSums &v, FeatSums *sm, int64_t *out_words) {
    int64_t *w = reinterpret_cast<int64_t *>(&v);
    int64_t *s = reinterpret_cast<int64_t *>(sm);
#pragma unroll
    for (int k = 0; k < kSumWords; ++k) s[threadIdx.x * kSumWords + k] = w[k];
    __syncthreads();
    for (int st = kFT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            FeatSums &a = sm[threadIdx.x];
            const FeatSums &b = sm[threadIdx.x + st];
#pragma unroll
            for (int q = 0; q < SPC_N_SHAPES; ++q) a.nb[q] += b.nb[q];
            a.single18 += b.single18;
            a.empty_rows += b.empty_rows;
            a.sum_len2 += b.sum_len2;
            a.sum_dist += b.sum_dist;
            a.max_len = a.max_len > b.max_len ? a.max_len : b.max_len;
            a.nonempty_rows += b.nonempty_rows;
            a.sum_log_span += b.sum_log_span;
        }
        __syncthreads();
    }
    if (threadIdx.x < kSumWords) out_words[threadIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(kFT) void k_features(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                                  const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, int64_t *part,
                                                  int *err) {
    __shared__ FeatSums sm[kFT];
    FeatSums v = {};
    const int64_t n_groups = (n_rows + kGroup - 1) / kGroup;
    const int64_t g = (int64_t)blockIdx.x * kFT + threadIdx.x;
    const int64_t g_first = g - (threadIdx.x & 63);   // the wavefront's first group
    if (g_first < n_groups) {
        // the wavefront's column resource starts at its first row's entries
        // (clamped into the array, as the row pointers are not checked yet)
        int64_t first = rowptr[g_first * kGroup];
        first = first < 0 ? 0 : first > nnz ? nnz : first;
        int64_t rel;
        const auto cr = dev::col_rsrc(col, nnz, first, &rel);
        if (g < n_groups) {
            int lo[kGroup], hi[kGroup];
            int bad = kErrNone;
#pragma unroll
            for (int r = 0; r < kGroup; ++r) {
                const int64_t i = g * kGroup + r;
                lo[r] = hi[r] = 0;
                if (i >= n_rows) continue;
                const int64_t a = rowptr[i], b = rowptr[i + 1];
                if (a < 0 || b < a || b > nnz || (i == 0 && a != 0) || (i == n_rows - 1 && b != nnz)) {
                    bad |= kErrRange;
                    continue;
                }
                // one pass over the row: the CSR check, the row statistics
                // and its beta(1,8) cover with the values of each block
                const int len = (int)(b - a);
                dev::ColCursor c;
                c.init(cr, (int32_t)(a + rel), (int32_t)(b + rel));
                int64_t prev = -1, dist = 0, first_col = 0, last_col = 0;
                int64_t end18 = INT64_MIN;
                int n_in = 0;
                bool row_ok = true;
                for (int64_t k = 0; c.live(); ++k) {
                    const int64_t j = c.cur();
                    if (j < 0 || j >= n_cols) {
                        bad |= kErrRange;
                        row_ok = false;
                        break;
                    }
                    if (j <= prev) {
                        bad |= kErrOrder;
                        row_ok = false;
                        break;
                    }
                    if (k == 0) first_col = j;
                    last_col = j;
                    prev = j;
                    dist += j > i ? j - i : i - j;
                    if (j >= end18) {
                        if (n_in == 1) ++v.single18;
                        ++v.nb[0];
                        end18 = j + 8;
                        n_in = 1;
                    } else {
                        ++n_in;
                    }
                    c.next(cr);
                }
                if (!row_ok) continue;
                if (n_in == 1) ++v.single18;
                lo[r] = (int)a;
                hi[r] = (int)b;
                v.sum_len2 += (int64_t)len * len;
                v.sum_dist += dist;
                v.max_len = len > v.max_len ? len : v.max_len;
                if (len == 0) {
                    ++v.empty_rows;
                } else {
                    ++v.nonempty_rows;
                    const double span = (double)(last_col - first_col + 1);
                    v.sum_log_span += log2(span / (double)len);
                }
            }
            if (bad) {
                atomicOr(err, bad);
            } else {
                v.nb[1] = cover_all<2, 4, 0>(cr, rel, lo, hi);
                v.nb[2] = cover_all<2, 8, 0>(cr, rel, lo, hi);
                v.nb[3] = cover_all<4, 4, 0>(cr, rel, lo, hi);
                v.nb[4] = cover_all<4, 8, 0>(cr, rel, lo, hi);
                v.nb[5] = cover_all<8, 4, 0>(cr, rel, lo, hi);
            }
        }
    }
    block_reduce(v, sm, part + (int64_t)blockIdx.x * kSumWords);
}

// Sum of the per-block partials in one block, fixed order.
__global__ __launch_bounds__(kFT) void k_features_total(const int64_t *part, int64_t n_part, int64_t *out) {
    __shared__ FeatSums sm[kFT];
    FeatSums v = {};
    for (int64_t b = threadIdx.x; b < n_part; b += kFT) {
        const FeatSums &p = *reinterpret_cast<const FeatSums *>(part + b * kSumWords);
#pragma unroll
        for (int q = 0; q < SPC_N_SHAPES; ++q) v.nb[q] += p.nb[q];
        v.single18 += p.single18;
        v.empty_rows += p.empty_rows;
        v.sum_len2 += p.sum_len2;
        v.sum_dist += p.sum_dist;
        v.max_len = v.max_len > p.max_len ? v.max_len : p.max_len;
        v.nonempty_rows += p.nonempty_rows;
        v.sum_log_span += p.sum_log_span;
    }
    block_reduce(v, sm, out);
}

__global__ void k_zero_int(int *p) { *p = 0; }

// Partial blocks whose sums (plus the total and the flag) fit the scratch.
constexpr int64_t kScratchBlocks = (int64_t)((kScratchBytes - 256) / sizeof(FeatSums)) - 1;

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};   // per device ordinal

spc_status scratch_on_current_device(void **out) {
    int dev = 0;
    SPC_HIP(hipGetDevice(&dev));
    SPC_REQUIRE(dev >= 0 && dev < 64, SPC_ERR_CAPACITY, "device ordinal %d beyond 63", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SPC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SPC_REQUIRE(p != nullptr, SPC_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPC_OK;
}

spc_status check_feature_args(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rowptr,
                              const int32_t *colidx, const float *features_out) {
    SPC_REQUIRE(n_rows >= 1 && n_cols >= 1 && nnz >= 0, SPC_ERR_INVALID_ARG,
                "features need n_rows >= 1, n_cols >= 1 and nnz >= 0");
    SPC_REQUIRE(n_rows < (int64_t(1) << 31) && n_cols < (int64_t(1) << 31) && nnz < (int64_t(1) << 31),
                SPC_ERR_OVERFLOW, "sizes exceed the int32 index range");
    SPC_REQUIRE(rowptr && (colidx || nnz == 0) && features_out, SPC_ERR_INVALID_ARG, "null argument");
    return SPC_OK;
}

// Launches both feature kernels into `buf` (n_blk + 1 FeatSums, then the
// error flag), reads the total back, checks the flag and forms the 16
// features. Synchronizes the stream.
spc_status features_into(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rowptr,
                         const int32_t *colidx, int64_t n_blk, char *buf, float *features_out,
                         int64_t *n_blocks_out, hipStream_t stream) {
    const size_t part_bytes = (size_t)(n_blk + 1) * sizeof(FeatSums);
    int64_t *part = reinterpret_cast<int64_t *>(buf);
    int64_t *total = part + n_blk * kSumWords;
    int *err = reinterpret_cast<int *>(buf + part_bytes);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, stream, err);
    hipLaunchKernelGGL(k_features, dim3((unsigned)n_blk), dim3(kFT), 0, stream, n_rows, n_cols, nnz, rowptr,
                       colidx ? colidx : reinterpret_cast<const int32_t *>(rowptr), part, err);
    hipLaunchKernelGGL(k_features_total, dim3(1), dim3(kFT), 0, stream, part, n_blk, total);
    SPC_HIP(hipGetLastError());
    FeatSums t;
    int herr = 0;
    SPC_HIP(hipMemcpyAsync(&t, total, sizeof(t), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(!(herr & kErrRange), SPC_ERR_INDEX_RANGE,
                "CSR row pointers not monotone from 0 to nnz, or a column outside [0, n_cols)");
    SPC_REQUIRE(!(herr & kErrOrder), SPC_ERR_CSR_UNSORTED_OR_DUP, "a CSR row has unsorted or repeated columns");

    const double n = (double)n_rows, m = (double)n_cols, z = (double)nnz;
    double f[16] = {};
    f[0] = std::log2(n);
    f[1] = std::log2(m);
    f[2] = std::log2(z + 1.0);
    const double mean = z / n;
    f[3] = mean;
    if (nnz > 0) {
        // n^2 * variance = n * sum(len^2) - nnz^2, exact in 128-bit integers
        const __int128 v2 = (__int128)n_rows * t.sum_len2 - (__int128)nnz * nnz;
        f[4] = std::sqrt((double)v2) / n / mean;
    }
    f[5] = std::log2(1.0 + (double)t.max_len);
    f[6] = (double)t.empty_rows / n;
    if (nnz > 0) f[7] = (double)t.sum_dist / z / (n > m ? n : m);
    for (int s = 0; s < SPC_N_SHAPES; ++s) f[8 + s] = t.nb[s] ? z / (double)t.nb[s] : 0.0;
    if (nnz > 0) {
        f[14] = t.nb[0] ? (double)t.single18 / (double)t.nb[0] : 0.0;
        f[15] = t.nonempty_rows ? t.sum_log_span / (double)t.nonempty_rows : 0.0;
    }
    for (int k = 0; k < 16; ++k) features_out[k] = (float)f[k];
    if (n_blocks_out)
        for (int s = 0; s < SPC_N_SHAPES; ++s) n_blocks_out[s] = t.nb[s];
    return SPC_OK;
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_matrix_features(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rowptr,
                                          const int32_t *colidx, float *features_out,
                                          int64_t *n_blocks_out, hipStream_t stream) {
    spc_status st = check_feature_args(n_rows, n_cols, nnz, rowptr, colidx, features_out);
    if (st != SPC_OK) return st;
    const int64_t n_blk = div_up(div_up(n_rows, kGroup), kFT);
    DevBuf buf;
    SPC_HIP(buf.alloc((size_t)(n_blk + 1) * sizeof(FeatSums) + 256));
    return features_into(n_rows, n_cols, nnz, rowptr, colidx, n_blk, buf.as<char>(), features_out, n_blocks_out,
                         stream);
}

extern "C" int64_t spc_matrix_features_noalloc_max_rows(void) { return kScratchBlocks * kFT * kGroup; }

extern "C" spc_status spc_matrix_features_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                                  const int32_t *rowptr, const int32_t *colidx,
                                                  float *features_out, int64_t *n_blocks_out,
                                                  hipStream_t stream) {
    spc_status st = check_feature_args(n_rows, n_cols, nnz, rowptr, colidx, features_out);
    if (st != SPC_OK) return st;
    const int64_t n_blk = div_up(div_up(n_rows, kGroup), kFT);
    SPC_REQUIRE(n_blk <= kScratchBlocks, SPC_ERR_CAPACITY,
                "spc_matrix_features_noalloc takes at most %lld rows (its fixed scratch holds %lld partial "
                "blocks); got %lld",
                (long long)spc_matrix_features_noalloc_max_rows(), (long long)kScratchBlocks, (long long)n_rows);
    void *p = nullptr;
    if ((st = scratch_on_current_device(&p)) != SPC_OK) return st;
    return features_into(n_rows, n_cols, nnz, rowptr, colidx, n_blk, static_cast<char *>(p), features_out,
                         n_blocks_out, stream);
}
