// Tile plans: the static partition of row intervals the SpMV kernels run on.
//
// The paper assigns each OpenMP thread one run of consecutive intervals and
// moves an interval boundary to where the running block count is closest to
// the thread's share (Design, "Parallelization"). On the GPU the shares are
// tiles sized to one workgroup's LDS: consecutive intervals are packed while
// the tile holds at most tile_bits / (r*c) blocks and kThreads / r intervals;
// an interval never splits, and one with more blocks than a tile holds gets a
// tile of its own (the long path of the kernel). Building a plan also checks
// the view once (row pointers, columns inside the matrix, no bits in rows
// past n_rows, mask bits adding up to nnz), so the SpMV launches read only
// inside the arrays.
#include <vector>

#include "common.hpp"

namespace spc {

int spmv_max_intervals_per_tile(int r, int mode);
int wave_tile_bits(int dtype, int kq);
int test_tile_blocks(int shape, int dtype, int kq);
int brow_tile_blocks(int shape, int dtype, int kq);

namespace {

enum : int { kBadColumn = 1, kBadPhantomRow = 2 };

template <int MB> struct MaskT;
template <> struct MaskT<1> { using T = uint8_t; };
template <> struct MaskT<2> { using T = uint16_t; };
template <> struct MaskT<4> { using T = uint32_t; };

template <int R, int C>
__global__ __launch_bounds__(256) void k_tile_counts(const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                     const int32_t *__restrict__ brow,
                                                     const int32_t *__restrict__ bcol,
                                                     const uint8_t *__restrict__ masks, int64_t n_rows,
                                                     int64_t n_cols, int64_t *__restrict__ cnt, int *err) {
    using Sh = Shape<R, C>;
    using MW = typename MaskT<Sh::MB>::T;
    __shared__ int64_t part[4];
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDesc d = tiles[t];
        int64_t s = 0;
        for (int I = d.i0; I < d.i1; ++I) {
            const int b0 = brow[I], b1 = brow[I + 1];
            // rows of this interval that exist
            const int64_t rows_here = min<int64_t>(R, n_rows - (int64_t)I * R);
            const uint32_t row_bits = rows_here >= R ? Sh::RCMASK : ((1u << (rows_here * C)) - 1u);
            for (int b = b0 + (int)threadIdx.x; b < b1; b += blockDim.x) {
                const uint32_t m = reinterpret_cast<const MW *>(masks)[b];
                s += __popc(m);
                if (m & ~row_bits) atomicOr(err, kBadPhantomRow);
                // highest column offset used by any row of the block
                uint32_t cols = 0;
                for (int i = 0; i < R; ++i) cols |= (m >> (i * C)) & Sh::CMASK;
                const int64_t hi = cols ? (int64_t)bcol[b] + (31 - __clz(cols)) : (int64_t)bcol[b];
                if (bcol[b] < 0 || hi >= n_cols) atomicOr(err, kBadColumn);
            }
        }
        for (int d2 = 32; d2 >= 1; d2 >>= 1) s += __shfl_xor(s, d2, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) cnt[t] = part[0] + part[1] + part[2] + part[3];
        __syncthreads();
    }
}

// Per interval: its value count and its blocks holding more than one value
// (what test tiles and block-row-lane tiles are planned on). MB: mask bytes
// per block.
template <int MB>
__global__ __launch_bounds__(256) void k_interval_stats(const int32_t *__restrict__ brow, int64_t n_int,
                                                        const uint8_t *__restrict__ masks, int32_t *__restrict__ nval,
                                                        int32_t *__restrict__ nmulti) {
    using MW = typename MaskT<MB>::T;
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (I >= n_int) return;
    int v = 0, m = 0;
    for (int b = brow[I]; b < brow[I + 1]; ++b) {
        const int pc = __popc((uint32_t)reinterpret_cast<const MW *>(masks)[b]);
        v += pc;
        m += pc >= 2;
    }
    nval[I] = v;
    nmulti[I] = m;
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_plan_create(const spc_beta_view *A, const spc_plan_params *params,
                                      spc_plan **plan_out, hipStream_t stream) {
    spc_status st = check_view(A);
    if (st != SPC_OK) return st;
    SPC_REQUIRE(plan_out != nullptr, SPC_ERR_INVALID_ARG, "null plan_out");
    *plan_out = nullptr;
    const int tile_bits = params && params->tile_bits ? params->tile_bits : 2048;
    spc_plan_params dflt{};
    if (!params) {
        spc_plan_default_params(A, &dflt);
        params = &dflt;
    }
    SPC_REQUIRE(params->tile_order == SPC_ORDER_XCD || params->tile_order == SPC_ORDER_HW, SPC_ERR_INVALID_ARG,
                "tile_order must be SPC_ORDER_XCD (0) or SPC_ORDER_HW (1)");
    const int xcd_remap = params->tile_order == SPC_ORDER_XCD;
    const int mode = params ? params->mode : 0;
    SPC_REQUIRE(mode >= 0 && mode <= 4, SPC_ERR_INVALID_ARG, "mode must be 0, 1, 2, 3 or 4");
    SPC_REQUIRE(mode != 2 || (A->r * A->c == 8), SPC_ERR_UNSUPPORTED_SHAPE,
                "mode 2 (test tiles) is for beta(1,8) and beta(2,4)");
    SPC_REQUIRE(mode != 4 || (A->r == 1 && A->c == 8), SPC_ERR_UNSUPPORTED_SHAPE,
                "mode 4 (value lanes) is for beta(1,8)");
    const int kq = params && params->wave_chunks ? params->wave_chunks : 4;
    const int pipeline = params ? params->pipeline : 0;
    SPC_REQUIRE(pipeline >= 0, SPC_ERR_INVALID_ARG, "pipeline must be >= 0");
    const int cu_groups = params ? params->cu_groups : 0;
    const int wave_tiles = params ? params->wave_tiles : 0;
    SPC_REQUIRE(wave_tiles >= 0 && wave_tiles <= 2, SPC_ERR_INVALID_ARG, "wave_tiles must be 0, 1 or 2");
    SPC_REQUIRE(!(wave_tiles == 2 && (mode != 0 || pipeline)), SPC_ERR_INVALID_ARG,
                "wave_tiles = 2 applies to mode 0 without pipeline");
    const int spmm_path = params ? params->spmm_path : SPC_SPMM_AUTO;
    SPC_REQUIRE(spmm_path == SPC_SPMM_AUTO || spmm_path == SPC_SPMM_BITS || spmm_path == SPC_SPMM_ROWS,
                SPC_ERR_INVALID_ARG, "spmm_path must be 0, 1 or 2");
    SPC_REQUIRE(cu_groups == 0 || (cu_groups >= 2 && cu_groups <= 8), SPC_ERR_INVALID_ARG,
                "cu_groups must be 0 or 2..8 (got %d)", cu_groups);
    SPC_REQUIRE(!(cu_groups && mode == 1), SPC_ERR_INVALID_ARG, "cu_groups applies to modes 0, 2, 3 and 4 only");
    SPC_REQUIRE(!(pipeline && mode != 0), SPC_ERR_INVALID_ARG, "pipeline applies to mode 0 only");
    SPC_REQUIRE(kq == 2 || kq == 4 || kq == 6 || kq == 8, SPC_ERR_INVALID_ARG,
                "wave_chunks must be 2, 4, 6 or 8");
    SPC_REQUIRE(tile_bits == 1024 || tile_bits == 2048 || tile_bits == 3072 || tile_bits == 4032,
                SPC_ERR_INVALID_ARG, "tile_bits must be 1024, 2048, 3072 or 4032 (got %d)", tile_bits);
    const int shape = shape_of(A->r, A->c);
    const int r = A->r, rc = A->r * A->c;
    const int64_t n_int = div_up(A->n_rows, r);

    // Row-interval pointers on the host: checked, then partitioned.
    std::vector<int32_t> brow((size_t)n_int + 1, 0);
    if (n_int > 0) {
        SPC_HIP(hipMemcpyAsync(brow.data(), A->block_rowptr, sizeof(int32_t) * (n_int + 1),
                               hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipStreamSynchronize(stream));
    }
    SPC_REQUIRE(brow[0] == 0 && brow[n_int] == A->n_blocks, SPC_ERR_INDEX_RANGE,
                "block_rowptr must run from 0 to n_blocks (%lld)", (long long)A->n_blocks);
    for (int64_t t = 0; t < n_int; ++t)
        SPC_REQUIRE(brow[t] <= brow[t + 1], SPC_ERR_INDEX_RANGE, "block_rowptr decreases at %lld",
                    (long long)t);

    const int cap_bits = mode == 1 ? tile_bits : wave_tile_bits(A->dtype, kq);
    const int64_t target = cap_bits / rc;           // blocks per tile
    const int64_t max_int = spmv_max_intervals_per_tile(r, mode == 1 ? 1 : 0);
    std::vector<TileDesc> tiles;
    tiles.reserve((size_t)(A->n_blocks / (target ? target : 1) + n_int / max_int + 2));
    int64_t n_long = 0;
    // Test tiles (mode 2), block-row-lane and value-lane tiles (modes 3, 4) are planned on
    // each interval's value count (and count of blocks with several values)
    std::vector<int32_t> hv, hm;
    if (mode >= 2 && n_int > 0) {
        hv.resize((size_t)n_int);
        hm.resize((size_t)n_int);
        DevBuf dv, dm;
        SPC_HIP(dv.alloc(sizeof(int32_t) * n_int));
        SPC_HIP(dm.alloc(sizeof(int32_t) * n_int));
        const dim3 g((unsigned)div_up(n_int, 256)), b(256);
        const uint8_t *mk = static_cast<const uint8_t *>(A->block_masks);
        if (rc == 8)
            hipLaunchKernelGGL(k_interval_stats<1>, g, b, 0, stream, A->block_rowptr, n_int, mk, dv.as<int32_t>(),
                               dm.as<int32_t>());
        else if (rc == 16)
            hipLaunchKernelGGL(k_interval_stats<2>, g, b, 0, stream, A->block_rowptr, n_int, mk, dv.as<int32_t>(),
                               dm.as<int32_t>());
        else
            hipLaunchKernelGGL(k_interval_stats<4>, g, b, 0, stream, A->block_rowptr, n_int, mk, dv.as<int32_t>(),
                               dm.as<int32_t>());
        SPC_HIP(hipGetLastError());
        SPC_HIP(hipMemcpyAsync(hv.data(), dv.p, sizeof(int32_t) * n_int, hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipMemcpyAsync(hm.data(), dm.p, sizeof(int32_t) * n_int, hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipStreamSynchronize(stream));
    }
    if (mode == 2 && n_int > 0) {
        // test tiles: at most NB2 blocks, 64 of them with several values, and
        // no more values than the buffer holds; an interval beyond any limit
        // becomes a tile of its own on the long path (flag in `reserved`)
        const int64_t nb2 = test_tile_blocks(shape, A->dtype, kq);
        const int64_t vcap = cap_bits;
        constexpr int64_t kMulti = 64;
        for (int64_t i = 0; i < n_int;) {
            const int64_t nb = brow[i + 1] - brow[i];
            if (nb > nb2 || hm[i] > kMulti || hv[i] > vcap) {
                tiles.push_back({0, (int32_t)i, (int32_t)(i + 1), brow[i], brow[i + 1], 0, 1});
                ++n_long;
                ++i;
                continue;
            }
            const int64_t start = i;
            int64_t blocks = 0, multi = 0, values = 0;
            while (i < n_int && i - start < max_int) {
                const int64_t b = brow[i + 1] - brow[i];
                if (b > nb2 || hm[i] > kMulti || hv[i] > vcap || blocks + b > nb2 || multi + hm[i] > kMulti ||
                    values + hv[i] > vcap)
                    break;
                blocks += b;
                multi += hm[i];
                values += hv[i];
                ++i;
            }
            tiles.push_back({0, (int32_t)start, (int32_t)i, brow[start], brow[i], 0, 0});
        }
    }
    if ((mode == 3 || mode == 4) && n_int > 0) {
        // block-row-lane and value-lane tiles: up to the buffer's values and NBX blocks; an
        // interval beyond either becomes a tile of its own on the long path
        // (the kernel tells it by the same two counts)
        const int64_t nbx = brow_tile_blocks(shape, A->dtype, kq);
        const int64_t vcap = cap_bits;
        for (int64_t i = 0; i < n_int;) {
            const int64_t nb = brow[i + 1] - brow[i];
            if (nb > nbx || hv[i] > vcap) {
                tiles.push_back({0, (int32_t)i, (int32_t)(i + 1), brow[i], brow[i + 1], 0, 0});
                ++n_long;
                ++i;
                continue;
            }
            const int64_t start = i;
            int64_t blocks = 0, values = 0;
            while (i < n_int && i - start < max_int) {
                const int64_t b = brow[i + 1] - brow[i];
                if (b > nbx || hv[i] > vcap || blocks + b > nbx || values + hv[i] > vcap) break;
                blocks += b;
                values += hv[i];
                ++i;
            }
            tiles.push_back({0, (int32_t)start, (int32_t)i, brow[start], brow[i], 0, 0});
        }
    }
    for (int64_t i = mode >= 2 ? n_int : 0; i < n_int;) {
        const int64_t nb = brow[i + 1] - brow[i];
        if (nb > target) {
            tiles.push_back({0, (int32_t)i, (int32_t)(i + 1), brow[i], brow[i + 1], 0, 0});
            ++n_long;
            ++i;
            continue;
        }
        const int64_t start = i;
        int64_t blocks = 0;
        while (i < n_int && i - start < max_int) {
            const int64_t b = brow[i + 1] - brow[i];
            if (b > target || blocks + b > target) break;
            blocks += b;
            ++i;
        }
        tiles.push_back({0, (int32_t)start, (int32_t)i, brow[start], brow[i], 0, 0});
    }
    const int64_t n_tiles = (int64_t)tiles.size();
    SPC_REQUIRE(n_tiles < (int64_t(1) << 31) / 8, SPC_ERR_CAPACITY, "too many tiles");

    spc_plan *P = new (std::nothrow) spc_plan();
    SPC_REQUIRE(P, SPC_ERR_CAPACITY, "out of host memory");
    P->A = *A;
    P->shape = shape;
    P->tile_bits = cap_bits;
    P->kq = kq;
    P->pipeline = pipeline > 0;
    P->resident = 0;
    P->cu_groups = cu_groups;
    P->wave_tiles = wave_tiles == 2 ? 2 : 1;
    P->spmm_path = spmm_path;
    if (pipeline) {
        int g = 0;
        spc_status rs = spmv_resident_groups(shape, A->dtype, kq, &g);
        if (rs != SPC_OK) {
            delete P;
            return rs;
        }
        P->resident = pipeline > 1 && pipeline < g ? pipeline : g;
    }
    P->xcd_remap = xcd_remap;
    P->mode = mode;
    P->n_tiles = n_tiles;
    P->n_long = n_long;
    P->d_tiles = nullptr;
    (void)hipGetDevice(&P->device);
    auto fail = [&](spc_status s) {
        if (P->d_tiles) (void)hipFree(P->d_tiles);
        delete P;
        return s;
    };
    if (n_tiles == 0) {
        *plan_out = P;
        return SPC_OK;
    }
    hipError_t he = hipMalloc(&P->d_tiles, sizeof(TileDesc) * n_tiles);
    if (he != hipSuccess) return fail(hip_fail(he, "hipMalloc(tiles)", __FILE__, __LINE__));
    he = hipMemcpyAsync(P->d_tiles, tiles.data(), sizeof(TileDesc) * n_tiles, hipMemcpyHostToDevice, stream);
    if (he != hipSuccess) return fail(hip_fail(he, "hipMemcpyAsync(tiles)", __FILE__, __LINE__));

    // Value count per tile (and the view checks), then the tile offsets.
    DevBuf cnt, err;
    if ((he = cnt.alloc(sizeof(int64_t) * n_tiles)) != hipSuccess ||
        (he = err.alloc(sizeof(int))) != hipSuccess)
        return fail(hip_fail(he, "hipMalloc(plan scratch)", __FILE__, __LINE__));
    if ((he = hipMemsetAsync(err.p, 0, sizeof(int), stream)) != hipSuccess)
        return fail(hip_fail(he, "hipMemsetAsync", __FILE__, __LINE__));
    const unsigned grid = (unsigned)(n_tiles < 65536 ? n_tiles : 65536);
    with_shape(shape, [&](auto sh) {
        using Sh = decltype(sh);
        hipLaunchKernelGGL((k_tile_counts<Sh::R, Sh::C>), dim3(grid), dim3(256), 0, stream, P->d_tiles, n_tiles,
                           A->block_rowptr, A->block_colidx, static_cast<const uint8_t *>(A->block_masks),
                           A->n_rows, A->n_cols, cnt.as<int64_t>(), err.as<int>());
        return 0;
    });
    if ((he = hipGetLastError()) != hipSuccess) return fail(hip_fail(he, "k_tile_counts", __FILE__, __LINE__));
    std::vector<int64_t> hcnt((size_t)n_tiles);
    int herr = 0;
    if ((he = hipMemcpyAsync(hcnt.data(), cnt.p, sizeof(int64_t) * n_tiles, hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (he = hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (he = hipStreamSynchronize(stream)) != hipSuccess)
        return fail(hip_fail(he, "plan readback", __FILE__, __LINE__));
    if (herr & kBadColumn) {
        set_error("a block reaches a column outside [0, n_cols) or starts below 0");
        return fail(SPC_ERR_INDEX_RANGE);
    }
    if (herr & kBadPhantomRow) {
        set_error("a mask has bits for rows past n_rows");
        return fail(SPC_ERR_INDEX_RANGE);
    }
    int64_t run = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
        tiles[t].vbase = run;
        tiles[t].nv = (int32_t)hcnt[t];
        run += hcnt[t];
    }
    if (run != A->nnz) {
        set_error("mask bits count %lld entries but the view says nnz = %lld", (long long)run, (long long)A->nnz);
        return fail(SPC_ERR_INVALID_ARG);
    }
    if ((he = hipMemcpyAsync(P->d_tiles, tiles.data(), sizeof(TileDesc) * n_tiles, hipMemcpyHostToDevice,
                             stream)) != hipSuccess ||
        (he = hipStreamSynchronize(stream)) != hipSuccess)
        return fail(hip_fail(he, "plan upload", __FILE__, __LINE__));
    *plan_out = P;
    return SPC_OK;
}

extern "C" spc_status spc_plan_default_params(const spc_beta_view *A, spc_plan_params *params_out) {
    SPC_REQUIRE(A && params_out, SPC_ERR_INVALID_ARG, "null view or params_out");
    spc_plan_params p{};
    p.mode = 0;
    p.tile_order = SPC_ORDER_XCD;
    p.wave_chunks = A->nnz >= (int64_t(1) << 24) ? 8 : A->nnz >= (int64_t(1) << 20) ? 4 : 2;
    *params_out = p;
    return SPC_OK;
}

extern "C" spc_status spc_plan_destroy(spc_plan *plan) {
    if (!plan) return SPC_OK;
    if (plan->d_tiles) SPC_HIP(hipFree(plan->d_tiles));
    delete plan;
    return SPC_OK;
}

extern "C" spc_status spc_plan_info(const spc_plan *plan, int64_t *n_tiles, int64_t *n_long, int32_t *tile_bits) {
    SPC_REQUIRE(plan, SPC_ERR_INVALID_ARG, "null plan");
    if (n_tiles) *n_tiles = plan->n_tiles;
    if (n_long) *n_long = plan->n_long;
    if (tile_bits) *tile_bits = plan->tile_bits;
    return SPC_OK;
}

namespace spc {
spc_status spmv_launch(const spc_beta_view *A, const spc_plan *P, const void *x, void *y, int accumulate,
                       hipStream_t stream);
}

// Views are compared field by field: a plan is only valid for its own matrix.
static bool same_view(const spc_beta_view &a, const spc_beta_view &b) {
    return a.r == b.r && a.c == b.c && a.dtype == b.dtype && a.n_rows == b.n_rows && a.n_cols == b.n_cols &&
           a.nnz == b.nnz && a.n_blocks == b.n_blocks && a.block_rowptr == b.block_rowptr &&
           a.block_colidx == b.block_colidx && a.block_masks == b.block_masks && a.values == b.values;
}

extern "C" spc_status spc_spmv_beta(const spc_beta_view *A, const spc_plan *plan, const void *x, void *y,
                                    int32_t accumulate, hipStream_t stream) {
    spc_status st = check_view(A);
    if (st != SPC_OK) return st;
    SPC_REQUIRE(plan == nullptr || same_view(*A, plan->A), SPC_ERR_INVALID_ARG,
                "plan was built for a different matrix view");
    SPC_REQUIRE(accumulate == 0 || accumulate == 1, SPC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    if (A->n_rows == 0) return SPC_OK;
    SPC_REQUIRE(y != nullptr, SPC_ERR_INVALID_ARG, "null y");
    SPC_REQUIRE(A->n_cols == 0 || x != nullptr, SPC_ERR_INVALID_ARG, "null x");
    const size_t es = A->dtype == SPC_F64 ? 8 : 4;
    SPC_REQUIRE(reinterpret_cast<uintptr_t>(y) % es == 0 && reinterpret_cast<uintptr_t>(x) % es == 0,
                SPC_ERR_INVALID_ARG, "x and y must be aligned to the element size");
    if (plan == nullptr) {
        // one-off product: a default plan that lives for this call only
        TempPlan tp(stream);
        if ((st = spc_plan_create(A, nullptr, &tp.p, stream)) != SPC_OK) return st;
        if (tp.p->n_tiles == 0) return SPC_OK;
        return spmv_launch(A, tp.p, x, y, accumulate, stream);
    }
    if (plan->n_tiles == 0) return SPC_OK;
    return spmv_launch(A, plan, x, y, accumulate, stream);
}
