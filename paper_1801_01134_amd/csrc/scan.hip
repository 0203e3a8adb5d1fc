// Device exclusive prefix sums of per-item counts (used by conversion,
// decoding and planning). Three passes: per-chunk totals, a single-workgroup
// scan of the totals, then per-chunk scans offset by the chunk's base.
#include "common.hpp"

namespace spc {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int kScanChunk = kScanThreads * kScanPerThread;  // 2048 items

__device__ inline int64_t block_excl_scan(int64_t v, int64_t *smem, int64_t *total) {
    // Wave-level inclusive scan with shuffles, then across the 4 waves via LDS.
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t s = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(s, d, 64);
        if (lane >= d) s += o;
    }
    if (lane == 63) smem[wid] = s;
    __syncthreads();
    int64_t wbase = 0, all = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) wbase += smem[w];
        all += smem[w];
    }
    __syncthreads();
    *total = all;
    return wbase + s - v;
}

template <class CT>
__global__ __launch_bounds__(kScanThreads) void k_chunk_totals(const CT *in, int64_t n, int64_t *tot) {
    __shared__ int64_t sm[4];
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t v = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanPerThread + k;
        if (i < n) v += (int64_t)in[i];
    }
    int64_t total;
    (void)block_excl_scan(v, sm, &total);
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int64_t *tot, int64_t m) {
    __shared__ int64_t sm[4];
    int64_t carry = 0;
    for (int64_t base = 0; base < m; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < m ? tot[i] : 0;
        int64_t total;
        int64_t e = block_excl_scan(v, sm, &total);
        if (i < m) tot[i] = carry + e;
        carry += total;
    }
}

template <class CT>
__global__ __launch_bounds__(kScanThreads) void k_chunk_scan(const CT *in, int64_t n, const int64_t *tot,
                                                             int64_t *out) {
    __shared__ int64_t sm[4];
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t loc[kScanPerThread];
    int64_t v = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanPerThread + k;
        loc[k] = i < n ? (int64_t)in[i] : 0;
        v += loc[k];
    }
    int64_t total;
    int64_t e = block_excl_scan(v, sm, &total) + tot[blockIdx.x];
    for (int k = 0; k < kScanPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanPerThread + k;
        if (i < n) out[i] = e;
        e += loc[k];
        if (i == n - 1) out[n] = e;
    }
}

template <class CT>
spc_status scan_impl(const CT *counts, int64_t n, int64_t *out, int64_t *temp, hipStream_t stream) {
    if (n <= 0) {
        SPC_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), stream));
        return SPC_OK;
    }
    int64_t m = div_up(n, kScanChunk);
    hipLaunchKernelGGL(k_chunk_totals<CT>, dim3((unsigned)m), dim3(kScanThreads), 0, stream, counts, n, temp);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, stream, temp, m);
    hipLaunchKernelGGL(k_chunk_scan<CT>, dim3((unsigned)m), dim3(kScanThreads), 0, stream, counts, n, temp, out);
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

}  // namespace

int64_t scan_temp_elems(int64_t n) { return div_up(n > 0 ? n : 1, kScanChunk); }

spc_status scan_counts_i64(const int32_t *counts, int64_t n, int64_t *out, int64_t *temp,
                           hipStream_t stream) {
    return scan_impl<int32_t>(counts, n, out, temp, stream);
}

spc_status scan_counts64_i64(const int64_t *counts, int64_t n, int64_t *out, int64_t *temp,
                             hipStream_t stream) {
    return scan_impl<int64_t>(counts, n, out, temp, stream);
}

}  // namespace spc
