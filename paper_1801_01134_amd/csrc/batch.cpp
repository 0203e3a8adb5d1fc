// Batches: y_i = A_i x_i for many beta(r,c) matrices of uneven size and
// different shapes. Each matrix gets its own plan (the partition of the
// section "Parallelization": whole intervals, about equal blocks per tile),
// in mode 0 (wavefront tiles), mode 3 (block-row lanes), for beta(1,8) mode
// 4 (value lanes), or for beta(1,8) and beta(2,4) mode 2 (the test tiles of
// Algorithm 2), with its own chunk count. The matrices are
// grouped by (shape, mode, chunks); the tiles of a group are concatenated,
// each tagged with its matrix, and one kernel built for that group runs the
// group's whole list. A batch is therefore one launch per group present
// (one for a batch of one kind), each with that shape's registers and LDS
// only; small matrices no longer pay a launch each, and the tiles of all
// matrices of a group fill the device together. The launches can be
// captured once in a HIP graph and replayed.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace {
struct BatchGroup {
    int shape, mode, kq;
    int64_t off, n;  // tiles [off, off + n) of the batch's list
};
}  // namespace

struct spc_batch {
    int count = 0;
    int dtype = 0;
    int device = -1;
    std::vector<spc_beta_view> views;
    std::vector<spc::BatchMat> h_mats;
    std::vector<BatchGroup> groups;
    spc::BatchMat *d_mats = nullptr;
    spc::TileDesc *d_tiles = nullptr;
    int64_t n_tiles = 0;
    int64_t n_long = 0;
    bool vectors_set = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_accumulate = -1;
    int g_grid = -1;
    int single_shape = -1;  // shape index shared by all matrices, else -1
    int general_kq = 0;     // the chunk count when every matrix is mode 0 with one count, else 0
    int force_general = 0;  // one launch of the shape-switching kernel over the whole list
};

namespace {

void drop_graph(spc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_accumulate = b->g_grid = -1;
}

void release(spc_batch *b) {
    drop_graph(b);
    if (b->d_mats) (void)hipFree(b->d_mats);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    delete b;
}

spc_status check_batch_params(const spc_plan_params &p, const spc_beta_view &v, int i) {
    SPC_REQUIRE(p.mode == 0 || p.mode == 2 || p.mode == 3 || p.mode == 4, SPC_ERR_INVALID_ARG,
                "matrix %d: batches run wavefront tiles (modes 0, 2, 3 and 4), got mode %d", i, p.mode);
    SPC_REQUIRE(p.mode != 2 || (v.r * v.c == 8), SPC_ERR_UNSUPPORTED_SHAPE,
                "matrix %d: test tiles are for beta(1,8) and beta(2,4)", i);
    SPC_REQUIRE(p.mode != 4 || (v.r == 1 && v.c == 8), SPC_ERR_UNSUPPORTED_SHAPE,
                "matrix %d: value lanes are for beta(1,8)", i);
    SPC_REQUIRE(p.pipeline == 0 && p.wave_tiles <= 1, SPC_ERR_INVALID_ARG,
                "matrix %d: batches run one tile per wavefront (pipeline 0, wave_tiles 0 or 1)", i);
    return SPC_OK;
}

// Launches the batch's groups (or the one shape-switching launch) on stream.
spc_status launch_all(spc_batch *b, int accumulate, int grid_blocks, hipStream_t stream) {
    using namespace spc;
    if (b->force_general)
        return batched_launch(b->dtype, b->general_kq, b->d_mats, b->d_tiles, b->n_tiles, accumulate, grid_blocks,
                              -1, stream);
    for (const BatchGroup &g : b->groups) {
        const spc_status st =
            g.mode == 2   ? batched_launch_test(b->dtype, g.shape, g.kq, b->d_mats, b->d_tiles + g.off, g.n,
                                                accumulate, grid_blocks, stream)
            : g.mode >= 3 ? batched_launch_lanes(b->dtype, g.mode, g.shape, g.kq, b->d_mats, b->d_tiles + g.off, g.n,
                                                 accumulate, grid_blocks, stream)
                          : batched_launch(b->dtype, g.kq, b->d_mats, b->d_tiles + g.off, g.n, accumulate,
                                           grid_blocks, g.shape, stream);
        if (st != SPC_OK) return st;
    }
    return SPC_OK;
}

}  // namespace

using namespace spc;

extern "C" spc_status spc_batch_create(int32_t count, const spc_beta_view *views, const spc_plan_params *params,
                                       int32_t n_params, spc_batch **out, hipStream_t stream) {
    SPC_REQUIRE(out != nullptr, SPC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    SPC_REQUIRE(count >= 1 && views != nullptr, SPC_ERR_INVALID_ARG, "need count >= 1 views");
    SPC_REQUIRE(n_params == 0 || ((n_params == 1 || n_params == count) && params != nullptr), SPC_ERR_INVALID_ARG,
                "n_params must be 0, 1 or count (%d) with a non-NULL params, got %d", count, n_params);
    for (int i = 0; i < count; ++i) {
        spc_status st = check_view(&views[i]);
        if (st != SPC_OK) return st;
        SPC_REQUIRE(views[i].dtype == views[0].dtype, SPC_ERR_INVALID_ARG, "matrix %d has another dtype", i);
        SPC_REQUIRE((reinterpret_cast<uintptr_t>(views[i].values) & 15u) == 0 || views[i].nnz == 0,
                    SPC_ERR_INVALID_ARG, "matrix %d: values must be 16-byte aligned", i);
        const uint64_t es = views[i].dtype == SPC_F64 ? 8 : 4;
        SPC_REQUIRE((uint64_t)views[i].n_cols * es < 0xf0000000ull, SPC_ERR_CAPACITY,
                    "matrix %d: x must be smaller than 3.75 GiB", i);
        SPC_REQUIRE(i < (1 << 29), SPC_ERR_CAPACITY, "at most 2^29 matrices per batch");
        if (n_params > 0) {
            st = check_batch_params(params[n_params == 1 ? 0 : i], views[i], i);
            if (st != SPC_OK) return st;
        }
    }
    spc_batch *b = new spc_batch();
    b->count = count;
    b->dtype = views[0].dtype;
    b->views.assign(views, views + count);
    b->h_mats.resize(count);
    hipError_t he = hipGetDevice(&b->device);
    if (he != hipSuccess) {
        release(b);
        return hip_fail(he, "hipGetDevice", __FILE__, __LINE__);
    }
    // tiles of each (mode, shape, chunks) group, in matrix order
    std::map<std::tuple<int, int, int>, std::vector<TileDesc>> by_group;
    std::vector<TileDesc> tiles;
    for (int i = 0; i < count; ++i) {
        spc_plan_params p{};
        spc_status st = SPC_OK;
        if (n_params > 0) p = params[n_params == 1 ? 0 : i];
        else st = spc_plan_default_params(&views[i], &p);
        spc_plan *pl = nullptr;
        if (st == SPC_OK) st = spc_plan_create(&views[i], &p, &pl, stream);
        if (st != SPC_OK) {
            release(b);
            return st;
        }
        const int shape = shape_of(views[i].r, views[i].c);
        b->n_long += pl->n_long;
        tiles.resize((size_t)pl->n_tiles);
        if (pl->n_tiles > 0)
            he = hipMemcpy(tiles.data(), pl->d_tiles, sizeof(TileDesc) * (size_t)pl->n_tiles, hipMemcpyDeviceToHost);
        const int mode = pl->mode, kq = pl->kq;
        (void)spc_plan_destroy(pl);
        if (he != hipSuccess) {
            release(b);
            return hip_fail(he, "hipMemcpy (plan tiles)", __FILE__, __LINE__);
        }
        for (TileDesc &t : tiles) t.reserved = mode == 2 ? (i << 1) | (t.reserved & 1) : i;
        std::vector<TileDesc> &dst = by_group[std::make_tuple(mode, shape, kq)];
        dst.insert(dst.end(), tiles.begin(), tiles.end());
        BatchMat &m = b->h_mats[i];
        m.brow = views[i].block_rowptr;
        m.bcol = views[i].block_colidx;
        m.mw = static_cast<const uint64_t *>(views[i].block_masks);
        m.vals = views[i].values;
        m.x = nullptr;
        m.y = nullptr;
        m.n_rows = views[i].n_rows;
        m.nnz = views[i].nnz;
        m.n_blocks = views[i].n_blocks;
        m.n_cols = views[i].n_cols;
        m.shape = shape;
        m.reserved = 0;
    }
    std::vector<TileDesc> all;
    for (auto &kv : by_group) {
        BatchGroup g;
        g.mode = std::get<0>(kv.first);
        g.shape = std::get<1>(kv.first);
        g.kq = std::get<2>(kv.first);
        g.off = (int64_t)all.size();
        g.n = (int64_t)kv.second.size();
        all.insert(all.end(), kv.second.begin(), kv.second.end());
        b->groups.push_back(g);
    }
    b->n_tiles = (int64_t)all.size();
    b->single_shape = b->h_mats[0].shape;
    for (int i = 1; i < count; ++i)
        if (b->h_mats[i].shape != b->single_shape) b->single_shape = -1;
    b->general_kq = b->groups.empty() ? 4 : b->groups[0].kq;
    for (const BatchGroup &g : b->groups)
        if (g.mode != 0 || g.kq != b->general_kq) b->general_kq = 0;
    if ((he = hipMalloc(&b->d_mats, sizeof(BatchMat) * count)) != hipSuccess ||
        (he = hipMalloc(&b->d_tiles, sizeof(TileDesc) * (all.empty() ? 1 : all.size()))) != hipSuccess ||
        (he = hipMemcpy(b->d_tiles, all.data(), sizeof(TileDesc) * all.size(), hipMemcpyHostToDevice)) !=
            hipSuccess) {
        release(b);
        return hip_fail(he, "hipMalloc/hipMemcpy (batch tables)", __FILE__, __LINE__);
    }
    *out = b;
    return SPC_OK;
}

extern "C" spc_status spc_batch_destroy(spc_batch *b) {
    if (b) release(b);
    return SPC_OK;
}

extern "C" spc_status spc_batch_info(const spc_batch *b, int64_t *n_tiles, int64_t *n_long, int32_t *single_shape,
                                     int32_t *n_groups) {
    SPC_REQUIRE(b != nullptr, SPC_ERR_INVALID_ARG, "null batch");
    if (n_tiles) *n_tiles = b->n_tiles;
    if (n_long) *n_long = b->n_long;
    if (single_shape) *single_shape = b->single_shape;
    if (n_groups) *n_groups = (int32_t)b->groups.size();
    return SPC_OK;
}

extern "C" spc_status spc_batch_set_kernel(spc_batch *b, int32_t general) {
    SPC_REQUIRE(b != nullptr, SPC_ERR_INVALID_ARG, "null batch");
    SPC_REQUIRE(general == 0 || general == 1, SPC_ERR_INVALID_ARG, "general must be 0 or 1");
    SPC_REQUIRE(general == 0 || b->general_kq > 0, SPC_ERR_INVALID_ARG,
                "the shape-switching kernel needs every matrix in mode 0 with one chunk count");
    if (b->force_general != general) drop_graph(b);
    b->force_general = general;
    return SPC_OK;
}

extern "C" spc_status spc_batch_set_vectors(spc_batch *b, const void *const *xs, void *const *ys) {
    SPC_REQUIRE(b && xs && ys, SPC_ERR_INVALID_ARG, "null argument");
    const size_t es = b->dtype == SPC_F64 ? 8 : 4;
    for (int i = 0; i < b->count; ++i) {
        SPC_REQUIRE((xs[i] || b->views[i].n_cols == 0) && (ys[i] || b->views[i].n_rows == 0),
                    SPC_ERR_INVALID_ARG, "matrix %d: null x or y", i);
        SPC_REQUIRE(reinterpret_cast<uintptr_t>(xs[i]) % es == 0 && reinterpret_cast<uintptr_t>(ys[i]) % es == 0,
                    SPC_ERR_INVALID_ARG, "matrix %d: x or y not aligned to the element size", i);
        b->h_mats[i].x = xs[i];
        b->h_mats[i].y = ys[i];
    }
    int dev = 0;
    SPC_HIP(hipGetDevice(&dev));
    SPC_REQUIRE(dev == b->device, SPC_ERR_INVALID_ARG, "batch was created on device %d, current is %d",
                b->device, dev);
    SPC_HIP(hipMemcpy(b->d_mats, b->h_mats.data(), sizeof(BatchMat) * b->count, hipMemcpyHostToDevice));
    b->vectors_set = true;
    return SPC_OK;
}

extern "C" spc_status spc_spmv_batched(spc_batch *b, int32_t accumulate, int32_t grid_blocks, int32_t use_graph,
                                       hipStream_t stream) {
    SPC_REQUIRE(b != nullptr, SPC_ERR_INVALID_ARG, "null batch");
    SPC_REQUIRE(b->vectors_set, SPC_ERR_INVALID_ARG, "call spc_batch_set_vectors first");
    SPC_REQUIRE(accumulate == 0 || accumulate == 1, SPC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    SPC_REQUIRE(grid_blocks >= 0, SPC_ERR_INVALID_ARG, "grid_blocks must be >= 0");
    SPC_REQUIRE(!use_graph || stream != nullptr, SPC_ERR_INVALID_ARG, "graph capture needs a non-NULL stream");
    if (!use_graph) return launch_all(b, accumulate, grid_blocks, stream);
    if (!b->exec || b->g_accumulate != accumulate || b->g_grid != grid_blocks) {
        drop_graph(b);
        SPC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        spc_status st = launch_all(b, accumulate, grid_blocks, stream);
        hipError_t he = hipStreamEndCapture(stream, &b->graph);
        if (st != SPC_OK) {
            drop_graph(b);
            return st;
        }
        SPC_HIP(he);
        SPC_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->g_accumulate = accumulate;
        b->g_grid = grid_blocks;
    }
    SPC_HIP(hipGraphLaunch(b->exec, stream));
    return SPC_OK;
}
