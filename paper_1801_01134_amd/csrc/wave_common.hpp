// Device helpers shared by the wavefront kernels (SpMV, SpMM, batched).
#pragma once

#include "common.hpp"

namespace spc {
namespace dev {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Bit l set iff lane l's predicate holds (lanes of the wavefront's exec mask).
__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot((int)p); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ unsigned lane_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// s_waitcnt with one counter at zero and the others left alone (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8). The builtin
// lets the compiler's own wait insertion see the wait; the empty asm keeps
// memory accesses from moving across it.
// Loads with an LDS destination are not tracked by the compiler: data they
// bring is read only after wait_vm_all.
__device__ __forceinline__ void wait_vm_all() {
    __builtin_amdgcn_s_waitcnt(0x0f70);
    asm volatile("" ::: "memory");
}
// s_waitcnt vmcnt(N): all but the N most recently issued vector memory
// operations have completed (they complete in issue order).
template <int N>
__device__ __forceinline__ void wait_vm_n() {
    static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
    __builtin_amdgcn_s_waitcnt(0x0f70 | (N & 0xf) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}
__device__ __forceinline__ void wait_lds_all() {
    __builtin_amdgcn_s_waitcnt(0xc07f);
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ uint64_t low_bits(int n) {
    return n <= 0 ? 0ull : n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and broadcasts.
__device__ __forceinline__ int wave_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); // row_bcast:31
    return v;
}

// A double moved across lanes by a DPP pattern (both halves); every source
// lane must be active. The patterns used here read a lane of the same row,
// so no lane falls back to the bound value (and the move needs no old value).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}

// Sum over aligned groups of 2^lg lanes (lg uniform, 0..6); every lane of a
// group gets the group's total. Within a 16-lane row the partners come from
// DPP patterns (xor 1, xor 2, the mirrored lane in the 8-lane half, the
// mirrored lane in the row), which stay in the vector unit; wider groups
// finish with cross-row shuffles. The order of additions is fixed.
__device__ __forceinline__ double group_sum(double v, int lg) {
    if (lg >= 1) v += dpp_f64<0xb1>(v);   // quad_perm [1,0,3,2]
    if (lg >= 2) v += dpp_f64<0x4e>(v);   // quad_perm [2,3,0,1]
    if (lg >= 3) v += dpp_f64<0x141>(v);  // row_half_mirror
    if (lg >= 4) v += dpp_f64<0x140>(v);  // row_mirror
    if (lg >= 5) v += __shfl_xor(v, 16, 64);
    if (lg >= 6) v += __shfl_xor(v, 32, 64);
    return v;
}

// Sum over the aligned groups of G lanes (G = 4 or 8, the block width) of a
// value every lane holds; each lane of a group gets the group's total, added
// in a fixed order.
template <int G, class T>
__device__ __forceinline__ T row_group_sum(T v) {
    static_assert(G == 4 || G == 8, "block widths are 4 or 8");
    if constexpr (sizeof(T) == 8) {
        v += dpp_f64<0xb1>(v);                          // quad_perm [1,0,3,2]
        v += dpp_f64<0x4e>(v);                          // quad_perm [2,3,0,1]
        if constexpr (G == 8) v += dpp_f64<0x141>(v);   // row_half_mirror
    } else {
        v += dpp_f32<0xb1>(v);                          // quad_perm [1,0,3,2]
        v += dpp_f32<0x4e>(v);                          // quad_perm [2,3,0,1]
        if constexpr (G == 8) v += dpp_f32<0x141>(v);   // row_half_mirror
    }
    return v;
}

// Lane-select from a 64-bit uniform mask without touching the exec mask.
template <class V>
__device__ __forceinline__ V pick(uint64_t m, V if_set, V if_clear) {
    return __builtin_amdgcn_inverse_ballot_w64(m) ? if_set : if_clear;
}

// Raw buffer resources: loads past num_records return 0 and touch no memory,
// which replaces every bounds test of the tile's streams.
constexpr int kBufFlags = 0x00020000;   // gfx9 buffer descriptor word 3
constexpr int kNT = 2;                  // non-temporal (streamed once)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufFlags);
}

template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, int aux = 0);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, int aux) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, int aux) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}


}  // namespace dev
}  // namespace spc
