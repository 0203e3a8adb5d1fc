// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "spc5hip.h"

namespace spc {

// ---------------------------------------------------------------------------
// Error reporting: a thread-local message behind spc_last_error().
void set_error(const char *fmt, ...);
spc_status hip_fail(hipError_t e, const char *what, const char *file, int line);

#define SPC_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) return ::spc::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define SPC_REQUIRE(cond, code, ...)        \
    do {                                    \
        if (!(cond)) {                      \
            ::spc::set_error(__VA_ARGS__);  \
            return (code);                  \
        }                                   \
    } while (0)

// ---------------------------------------------------------------------------
// Block shapes. Index order follows the paper's list of optimized kernels.
constexpr int kShapeR[SPC_N_SHAPES] = {1, 2, 2, 4, 4, 8};
constexpr int kShapeC[SPC_N_SHAPES] = {8, 4, 8, 4, 8, 4};

inline int shape_of(int r, int c) {
    for (int s = 0; s < SPC_N_SHAPES; ++s)
        if (kShapeR[s] == r && kShapeC[s] == c) return s;
    return -1;
}

template <int R_, int C_>
struct Shape {
    static constexpr int R = R_;
    static constexpr int C = C_;
    static constexpr int RC = R_ * C_;          // mask bits per block: 8, 16 or 32
    static constexpr int BPW = 64 / RC;         // blocks per 64-bit mask word
    static constexpr int MB = RC / 8;           // mask bytes per block
    static constexpr uint32_t RCMASK = (RC == 32) ? 0xffffffffu : ((1u << RC) - 1u);
    static constexpr uint32_t CMASK = (1u << C_) - 1u;
};

// Calls f(Shape<r,c>{}) for a runtime shape index.
template <class F>
inline auto with_shape(int s, F &&f) {
    switch (s) {
    case 0: return f(Shape<1, 8>{});
    case 1: return f(Shape<2, 4>{});
    case 2: return f(Shape<2, 8>{});
    case 3: return f(Shape<4, 4>{});
    case 4: return f(Shape<4, 8>{});
    default: return f(Shape<8, 4>{});
    }
}

template <class F>
inline auto with_dtype(int dtype, F &&f) {
    if (dtype == SPC_F64) return f(double{});
    return f(float{});
}

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Tile of a plan: the intervals [i0, i1), their blocks [b0, b1), the
// packed-value offset of the tile's first block and the tile's value count.
// 32 bytes, read with one scalar load.
struct TileDesc {
    int64_t vbase;
    int32_t i0, i1;
    int32_t b0, b1;
    int32_t nv;
    int32_t reserved;
};

// One matrix of a batch, as the batched kernel reads it (device table).
struct BatchMat {
    const int32_t *brow;
    const int32_t *bcol;
    const uint64_t *mw;
    const void *vals;
    const void *x;
    void *y;
    int64_t n_rows, nnz, n_blocks, n_cols;
    int32_t shape;
    int32_t reserved;
};

// Batched product over a concatenated tile list (TileDesc::reserved holds
// the matrix index). grid_blocks 0: one wavefront per tile; > 0: that many
// workgroups loop over the tiles. single_shape: the shape index when all
// matrices share it (a kernel without the shape switch), else -1.
spc_status batched_launch(int dtype, int kq, const BatchMat *d_mats, const TileDesc *d_tiles, int64_t n_tiles,
                          int accumulate, int grid_blocks, int single_shape, hipStream_t stream);
// Batched test tiles (mode 2) of one shape (0 or 1): TileDesc::reserved
// holds (matrix index << 1) | long flag. grid_blocks as above.
spc_status batched_launch_test(int dtype, int shape, int kq, const BatchMat *d_mats, const TileDesc *d_tiles,
                               int64_t n_tiles, int accumulate, int grid_blocks, hipStream_t stream);
// Batched block-row-lane (mode 3) or value-lane (mode 4, beta(1,8)) tiles of
// one shape and chunk count; TileDesc::reserved holds the matrix index.
spc_status batched_launch_lanes(int dtype, int mode, int shape, int kq, const BatchMat *d_mats,
                                const TileDesc *d_tiles, int64_t n_tiles, int accumulate, int grid_blocks,
                                hipStream_t stream);

// Workgroups of the pipelined mode-0 kernel resident at once (occupancy x CUs).
spc_status spmv_resident_groups(int shape, int dtype, int kq, int *out);

// Dynamic LDS bytes that keep at most cu_groups workgroups of a kernel (whose
// static LDS is static_lds bytes) resident per compute unit; 0 when
// cu_groups is 0 or the kernel already holds no more than that.
size_t lds_reserve_for(size_t static_lds, int cu_groups);

// Launches kernel(args); with cu_groups > 0 it reserves the LDS that keeps at
// most that many of its workgroups on a compute unit.
template <class K, class Args>
spc_status launch_capped(K kernel, int cu_groups, dim3 grid, dim3 block, hipStream_t s, const Args &args) {
    size_t dyn = 0;
    if (cu_groups > 0) {
        hipFuncAttributes fa;
        SPC_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kernel)));
        dyn = lds_reserve_for(fa.sharedSizeBytes, cu_groups);
    }
    hipLaunchKernelGGL(kernel, grid, block, dyn, s, args);
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

// Validation of a view on the host.
spc_status check_view(const spc_beta_view *A);

// Exclusive prefix sum of n int32 counts into out[0..n] (int64), on stream.
// temp must hold scan_temp_elems(n) int64. Asynchronous.
int64_t scan_temp_elems(int64_t n);
spc_status scan_counts_i64(const int32_t *counts, int64_t n, int64_t *out, int64_t *temp,
                           hipStream_t stream);
// Same, from int64 counts.
spc_status scan_counts64_i64(const int64_t *counts, int64_t n, int64_t *out, int64_t *temp,
                             hipStream_t stream);

// Small RAII holder for device scratch used by setup routines (conversion,
// plan creation); the SpMV entry points allocate nothing.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// A plan that lives for one call: released after the work queued on its
// stream has finished (its tile descriptors are read by that work).
struct TempPlan {
    spc_plan *p = nullptr;
    hipStream_t s;
    explicit TempPlan(hipStream_t stream) : s(stream) {}
    ~TempPlan() {
        if (p) {
            (void)hipStreamSynchronize(s);
            (void)spc_plan_destroy(p);
        }
    }
    TempPlan(const TempPlan &) = delete;
    TempPlan &operator=(const TempPlan &) = delete;
};

}  // namespace spc

struct spc_plan {
    spc_beta_view A;
    int shape;
    int tile_bits;
    int xcd_remap;
    int mode;
    int kq;
    int pipeline;  // mode 0: persistent wavefronts that prefetch their next tile
    int resident;  // workgroups of the pipelined kernel resident at once
    int cu_groups; // 0, or at most this many workgroups per compute unit (non-persistent launches)
    int wave_tiles; // mode 0: 1, or 2 consecutive tiles per wavefront (the second staged in registers)
    int spmm_path;  // SPC_SPMM_AUTO, SPC_SPMM_BITS or SPC_SPMM_ROWS
    int device;
    int64_t n_tiles;
    int64_t n_long;
    spc::TileDesc *d_tiles;
};
