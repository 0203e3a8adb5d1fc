// Batches: y_i = A_i x_i for many beta(r,c) matrices of uneven size and
// different shapes in one launch. Each matrix gets its own mode-0 plan (the
// partition of the section "Parallelization": whole intervals, about equal
// blocks per tile); the tiles of all plans are concatenated, each tagged
// with its matrix, and one kernel runs the whole list. Small matrices no
// longer pay a launch each, and the tiles of all matrices fill the device
// together. The launch can be captured once in a HIP graph and replayed.
#include <vector>

#include "common.hpp"

struct spc_batch {
    int count = 0;
    int dtype = 0;
    int kq = 4;
    int device = -1;
    std::vector<spc_beta_view> views;
    std::vector<spc::BatchMat> h_mats;
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
    int force_general = 0;  // run the shape-switching kernel even for one shape
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

}  // namespace

using namespace spc;

extern "C" spc_status spc_batch_create(int32_t count, const spc_beta_view *views, const spc_plan_params *params,
                                       spc_batch **out, hipStream_t stream) {
    SPC_REQUIRE(out != nullptr, SPC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    SPC_REQUIRE(count >= 1 && views != nullptr, SPC_ERR_INVALID_ARG, "need count >= 1 views");
    SPC_REQUIRE(params == nullptr || params->mode == 0, SPC_ERR_INVALID_ARG,
                "batches run wavefront tiles (mode 0)");
    for (int i = 0; i < count; ++i) {
        spc_status st = check_view(&views[i]);
        if (st != SPC_OK) return st;
        SPC_REQUIRE(views[i].dtype == views[0].dtype, SPC_ERR_INVALID_ARG, "matrix %d has another dtype", i);
        SPC_REQUIRE((reinterpret_cast<uintptr_t>(views[i].values) & 15u) == 0 || views[i].nnz == 0,
                    SPC_ERR_INVALID_ARG, "matrix %d: values must be 16-byte aligned", i);
        const uint64_t es = views[i].dtype == SPC_F64 ? 8 : 4;
        SPC_REQUIRE((uint64_t)views[i].n_cols * es < 0xf0000000ull, SPC_ERR_CAPACITY,
                    "matrix %d: x must be smaller than 3.75 GiB", i);
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
    std::vector<TileDesc> all;
    for (int i = 0; i < count; ++i) {
        spc_plan *p = nullptr;
        spc_status st = spc_plan_create(&views[i], params, &p, stream);
        if (st != SPC_OK) {
            release(b);
            return st;
        }
        b->kq = p->kq;
        b->n_long += p->n_long;
        const size_t at = all.size();
        all.resize(at + (size_t)p->n_tiles);
        if (p->n_tiles > 0) {
            he = hipMemcpy(all.data() + at, p->d_tiles, sizeof(TileDesc) * (size_t)p->n_tiles,
                           hipMemcpyDeviceToHost);
        }
        (void)spc_plan_destroy(p);
        if (he != hipSuccess) {
            release(b);
            return hip_fail(he, "hipMemcpy (plan tiles)", __FILE__, __LINE__);
        }
        for (size_t t = at; t < all.size(); ++t) all[t].reserved = i;
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
        m.shape = shape_of(views[i].r, views[i].c);
        m.reserved = 0;
    }
    b->n_tiles = (int64_t)all.size();
    b->single_shape = b->h_mats[0].shape;
    for (int i = 1; i < count; ++i)
        if (b->h_mats[i].shape != b->single_shape) b->single_shape = -1;
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

extern "C" spc_status spc_batch_info(const spc_batch *b, int64_t *n_tiles, int64_t *n_long, int32_t *single_shape) {
    SPC_REQUIRE(b != nullptr, SPC_ERR_INVALID_ARG, "null batch");
    if (n_tiles) *n_tiles = b->n_tiles;
    if (n_long) *n_long = b->n_long;
    if (single_shape) *single_shape = b->single_shape;
    return SPC_OK;
}

extern "C" spc_status spc_batch_set_kernel(spc_batch *b, int32_t general) {
    SPC_REQUIRE(b != nullptr, SPC_ERR_INVALID_ARG, "null batch");
    SPC_REQUIRE(general == 0 || general == 1, SPC_ERR_INVALID_ARG, "general must be 0 or 1");
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
    const int single = b->force_general ? -1 : b->single_shape;
    if (!use_graph) return batched_launch(b->dtype, b->kq, b->d_mats, b->d_tiles, b->n_tiles, accumulate,
                                          grid_blocks, single, stream);
    if (!b->exec || b->g_accumulate != accumulate || b->g_grid != grid_blocks) {
        drop_graph(b);
        SPC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        spc_status st = batched_launch(b->dtype, b->kq, b->d_mats, b->d_tiles, b->n_tiles, accumulate,
                                       grid_blocks, single, stream);
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
