// Column cursors for walks along CSR rows (conversion, features).
#pragma once

#include "wave_common.hpp"

namespace spc {
namespace dev {

// The resource a wavefront uses for the rows of its entries starting at
// entry `first` of colidx: it starts at the 16-byte boundary at or below that
// entry and runs to the end of the array (at most 4 GB); *rel is added to an
// entry index to get its position in the resource. The few bytes read below
// colidx[first] share its 16-byte block.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_rsrc(const int32_t *colidx, int64_t nnz, int64_t first,
                                                           int64_t *rel) {
    const int64_t shift = (int64_t)((reinterpret_cast<uintptr_t>(colidx) & 15u) >> 2);
    const int64_t b4 = (first + shift) & ~(int64_t)3;
    const int32_t *base = colidx - shift + b4;
    const int64_t bytes = (nnz + shift - b4) * 4;
    *rel = shift - b4;
    return rsrc(base, (uint32_t)(bytes < 0 ? 0 : bytes > 0xfffffff0ll ? 0xfffffff0ll : bytes));
}

// A cursor over the sorted columns of one CSR row, positions [p, end) of
// the wavefront's column resource (col_rsrc). The columns are read 16 bytes
// at a time, with the following 16 bytes already in flight, so a walk along
// the row waits on memory about once per four entries instead of once per
// entry. Windows reaching past the array return zeros.
struct ColCursor {
    using I4 = __attribute__((ext_vector_type(4))) int;
    int32_t p, end;
    I4 w, wn;  // the windows at (p & ~3) and the next four entries

    __device__ __forceinline__ static I4 load(__amdgpu_buffer_rsrc_t r, int32_t q) {
        return __builtin_bit_cast(I4, __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)q * 4u, 0, 0));
    }
    __device__ __forceinline__ void init(__amdgpu_buffer_rsrc_t r, int32_t p0, int32_t e) {
        p = p0;
        end = e;
        const int32_t b = p0 & ~3;
        w = load(r, b);
        wn = load(r, b + 4);
    }
    __device__ __forceinline__ bool live() const { return p < end; }
    // the current column (meaningful while live())
    __device__ __forceinline__ int32_t cur() const {
        const int k = p & 3;
        return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
    }
    __device__ __forceinline__ void next(__amdgpu_buffer_rsrc_t r) {
        ++p;
        if ((p & 3) == 0) {
            w = wn;
            wn = load(r, p + 4);
        }
    }
};

}  // namespace dev
}  // namespace spc
