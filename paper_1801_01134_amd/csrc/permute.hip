// Symmetric permutation of a CSR matrix, B = P A P^T, and of vectors, on the
// device (the second half of the reordering step of section "Matrix
// permutation/reordering"; the order comes from spc_rcm_order or the caller).
//
// perm[new] = old. Row i of B is row perm[i] of A with each column j renamed
// inv[j] (inv[perm[i]] = i) and the row's columns sorted; values are moved
// bit for bit. One thread builds one row of B: it copies the renamed entries
// and sorts them in place (insertion sort for short rows, a Shell sort with
// the gaps 1, 4, 13, 40, ... for longer ones).
#include "common.hpp"

namespace spc {
namespace {

constexpr int kPT = 256;

__global__ __launch_bounds__(kPT) void k_inverse(const int32_t *__restrict__ perm, int64_t n,
                                                 int32_t *__restrict__ inv, int *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm[i];
    if (o < 0 || o >= n) {
        atomicOr(err, 1);
        return;
    }
    // a repeated entry leaves some slot unclaimed and another claimed twice
    if (atomicExch(&inv[o], (int32_t)i) != -1) atomicOr(err, 2);
}

__global__ __launch_bounds__(kPT) void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kPT) void k_perm_lengths(const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ perm, int64_t n,
                                                      int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i < n) len[i] = rowptr[perm[i] + 1] - rowptr[perm[i]];
}

__global__ __launch_bounds__(kPT) void k_offsets_to_i32(const int64_t *__restrict__ off, int64_t n,
                                                        int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i <= n) out[i] = (int32_t)off[i];
}

template <class V>
__device__ __forceinline__ void sort_row(int32_t *c, V *v, int len) {
    if (len <= 32) {
        for (int a = 1; a < len; ++a) {
            const int32_t ck = c[a];
            const V vk = v[a];
            int b = a - 1;
            while (b >= 0 && c[b] > ck) {
                c[b + 1] = c[b];
                v[b + 1] = v[b];
                --b;
            }
            c[b + 1] = ck;
            v[b + 1] = vk;
        }
        return;
    }
    int gap = 1;
    while (gap < len / 3) gap = 3 * gap + 1;
    for (; gap >= 1; gap /= 3) {
        for (int a = gap; a < len; ++a) {
            const int32_t ck = c[a];
            const V vk = v[a];
            int b = a - gap;
            while (b >= 0 && c[b] > ck) {
                c[b + gap] = c[b];
                v[b + gap] = v[b];
                b -= gap;
            }
            c[b + gap] = ck;
            v[b + gap] = vk;
        }
    }
}

template <class V>
__global__ __launch_bounds__(kPT) void k_perm_rows(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                                   const V *__restrict__ vals, const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ inv, int64_t n,
                                                   const int32_t *__restrict__ rowptr_out, int32_t *__restrict__ col_out,
                                                   V *__restrict__ val_out) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm[i];
    const int32_t s = rowptr[o], len = rowptr[o + 1] - s;
    const int32_t d = rowptr_out[i];
    for (int k = 0; k < len; ++k) {
        col_out[d + k] = inv[colidx[s + k]];
        val_out[d + k] = vals[s + k];
    }
    sort_row(col_out + d, val_out + d, len);
}

template <class V>
__global__ __launch_bounds__(kPT) void k_perm_vector(const int32_t *__restrict__ perm, int64_t n, const V *__restrict__ in,
                                                     V *__restrict__ out, int scatter) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= n) return;
    if (scatter) out[perm[i]] = in[i];
    else out[i] = in[perm[i]];
}

unsigned blocks(int64_t n) { return (unsigned)div_up(n > 0 ? n : 1, kPT); }

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_csr_permute(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                                      int32_t dtype, const void *values, const int32_t *perm,
                                      int32_t *rowptr_out, int32_t *colidx_out, void *values_out,
                                      hipStream_t stream) {
    SPC_REQUIRE(n >= 0 && nnz >= 0, SPC_ERR_INVALID_ARG, "negative size");
    SPC_REQUIRE(n < (int64_t(1) << 31) && nnz < (int64_t(1) << 31), SPC_ERR_OVERFLOW,
                "sizes exceed the int32 index range");
    SPC_REQUIRE(dtype == SPC_F32 || dtype == SPC_F64, SPC_ERR_INVALID_ARG, "bad dtype %d", dtype);
    SPC_REQUIRE(rowptr && rowptr_out, SPC_ERR_INVALID_ARG, "null row pointers");
    if (n == 0) {
        SPC_HIP(hipMemsetAsync(rowptr_out, 0, sizeof(int32_t), stream));
        return SPC_OK;
    }
    SPC_REQUIRE(perm, SPC_ERR_INVALID_ARG, "null perm");
    SPC_REQUIRE(nnz == 0 || (colidx && values && colidx_out && values_out), SPC_ERR_INVALID_ARG, "null argument");
    DevBuf inv, err, len, off, temp;
    SPC_HIP(inv.alloc(sizeof(int32_t) * n));
    SPC_HIP(err.alloc(sizeof(int)));
    SPC_HIP(len.alloc(sizeof(int32_t) * n));
    SPC_HIP(off.alloc(sizeof(int64_t) * (n + 1)));
    SPC_HIP(temp.alloc(sizeof(int64_t) * scan_temp_elems(n)));
    SPC_HIP(hipMemsetAsync(err.p, 0, sizeof(int), stream));
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n)), dim3(kPT), 0, stream, inv.as<int32_t>(), n, -1);
    hipLaunchKernelGGL(k_inverse, dim3(blocks(n)), dim3(kPT), 0, stream, perm, n, inv.as<int32_t>(), err.as<int>());
    int herr = 0;
    SPC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(herr == 0, SPC_ERR_INDEX_RANGE, "perm is not a permutation of 0..n-1");
    hipLaunchKernelGGL(k_perm_lengths, dim3(blocks(n)), dim3(kPT), 0, stream, rowptr, perm, n, len.as<int32_t>());
    spc_status st = scan_counts_i64(len.as<int32_t>(), n, off.as<int64_t>(), temp.as<int64_t>(), stream);
    if (st != SPC_OK) return st;
    hipLaunchKernelGGL(k_offsets_to_i32, dim3(blocks(n + 1)), dim3(kPT), 0, stream, off.as<int64_t>(), n,
                       rowptr_out);
    if (nnz > 0) {
        if (dtype == SPC_F64)
            hipLaunchKernelGGL(k_perm_rows<uint64_t>, dim3(blocks(n)), dim3(kPT), 0, stream, rowptr, colidx,
                               static_cast<const uint64_t *>(values), perm, inv.as<int32_t>(), n, rowptr_out,
                               colidx_out, static_cast<uint64_t *>(values_out));
        else
            hipLaunchKernelGGL(k_perm_rows<uint32_t>, dim3(blocks(n)), dim3(kPT), 0, stream, rowptr, colidx,
                               static_cast<const uint32_t *>(values), perm, inv.as<int32_t>(), n, rowptr_out,
                               colidx_out, static_cast<uint32_t *>(values_out));
    }
    SPC_HIP(hipGetLastError());
    // the scratch buffers are freed on return: wait for the kernels that read them
    SPC_HIP(hipStreamSynchronize(stream));
    return SPC_OK;
}

extern "C" spc_status spc_permute_vector(int64_t n, int32_t dtype, const int32_t *perm, const void *in, void *out,
                                         int32_t scatter, hipStream_t stream) {
    SPC_REQUIRE(n >= 0, SPC_ERR_INVALID_ARG, "negative size");
    SPC_REQUIRE(dtype == SPC_F32 || dtype == SPC_F64, SPC_ERR_INVALID_ARG, "bad dtype %d", dtype);
    SPC_REQUIRE(scatter == 0 || scatter == 1, SPC_ERR_INVALID_ARG, "scatter must be 0 or 1");
    if (n == 0) return SPC_OK;
    SPC_REQUIRE(perm && in && out && in != out, SPC_ERR_INVALID_ARG, "null or aliased argument");
    if (dtype == SPC_F64)
        hipLaunchKernelGGL(k_perm_vector<uint64_t>, dim3(blocks(n)), dim3(kPT), 0, stream, perm, n,
                           static_cast<const uint64_t *>(in), static_cast<uint64_t *>(out), scatter);
    else
        hipLaunchKernelGGL(k_perm_vector<uint32_t>, dim3(blocks(n)), dim3(kPT), 0, stream, perm, n,
                           static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out), scatter);
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}
