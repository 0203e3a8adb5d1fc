// Timing records and the autotuner: every candidate plan is built and timed
// on the device; the fastest parameter set wins.
#include <vector>

#include "common.hpp"

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" spc_status spc_time_spmv(const spc_beta_view *A, const spc_plan *plan, const void *x, void *y,
                                    int32_t warmup, int32_t reps, float *us_out, hipStream_t stream) {
    SPC_REQUIRE(us_out && reps > 0 && warmup >= 0, SPC_ERR_INVALID_ARG, "bad timing arguments");
    spc_status st;
    for (int i = 0; i < warmup; ++i)
        if ((st = spc_spmv_beta(A, plan, x, y, 0, stream)) != SPC_OK) return st;
    EventPair ev;
    SPC_HIP(hipEventCreate(&ev.a));
    SPC_HIP(hipEventCreate(&ev.b));
    SPC_HIP(hipEventRecord(ev.a, stream));
    for (int i = 0; i < reps; ++i)
        if ((st = spc_spmv_beta(A, plan, x, y, 0, stream)) != SPC_OK) return st;
    SPC_HIP(hipEventRecord(ev.b, stream));
    SPC_HIP(hipEventSynchronize(ev.b));
    float ms = 0.f;
    SPC_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    *us_out = ms * 1000.f / (float)reps;
    return SPC_OK;
}

extern "C" spc_status spc_autotune(const spc_beta_view *A, const void *x, void *y, int32_t reps,
                                   spc_plan_params *best, float *best_us, spc_tune_record *records,
                                   int32_t max_records, int32_t *n_records, hipStream_t stream) {
    spc_status st = spc::check_view(A);
    if (st != SPC_OK) return st;
    SPC_REQUIRE(best && best_us && reps > 0, SPC_ERR_INVALID_ARG, "bad autotune arguments");
    if (n_records) *n_records = 0;
    std::vector<spc_plan_params> cands;
    for (int order : {SPC_ORDER_XCD, SPC_ORDER_HW}) {
        for (int kq : {2, 4, 6, 8}) {
            spc_plan_params p{};
            p.mode = 0;
            p.wave_chunks = kq;
            p.tile_order = order;
            cands.push_back(p);
            if (order == SPC_ORDER_XCD) {
                if (kq >= 4) {
                    for (int cap : {2, 4}) {  // fewer resident workgroups per compute unit
                        spc_plan_params q = p;
                        q.cu_groups = cap;
                        cands.push_back(q);
                    }
                }
                if (kq >= 4) {  // two tiles per wavefront
                    spc_plan_params q = p;
                    q.wave_tiles = 2;
                    cands.push_back(q);
                    if (kq == 8) {
                        q.cu_groups = 4;
                        cands.push_back(q);
                    }
                }
                p.pipeline = 1;  // persistent: the grid order does not apply
                cands.push_back(p);
            }
        }
        for (int tb : {1024, 2048, 3072, 4032}) {
            spc_plan_params p{};
            p.mode = 1;
            p.tile_bits = tb;
            p.tile_order = order;
            cands.push_back(p);
        }
    }
    // block-row lanes, and for beta(1,8) value lanes: their tiles are sized
    // by values, so small chunk counts already fill them
    for (int mode : {3, 4}) {
        if (mode == 4 && !(A->r == 1 && A->c == 8)) continue;
        for (int kq : {2, 4, 6, 8}) {
            spc_plan_params p{};
            p.mode = mode;
            p.wave_chunks = kq;
            cands.push_back(p);
        }
    }
    if (A->r * A->c == 8) {
        for (int kq : {2, 4, 6, 8}) {  // test tiles (Algorithm 2)
            spc_plan_params p{};
            p.mode = 2;
            p.wave_chunks = kq;
            cands.push_back(p);
        }
    }
    float best_t = -1.f;
    int nrec = 0;
    for (const spc_plan_params &p : cands) {
        spc_plan *plan = nullptr;
        if ((st = spc_plan_create(A, &p, &plan, stream)) != SPC_OK) return st;
        float us = 0.f;
        st = spc_time_spmv(A, plan, x, y, 2, reps, &us, stream);
        int64_t nt = plan->n_tiles;
        spc_plan_destroy(plan);
        if (st != SPC_OK) return st;
        if (records && nrec < max_records) records[nrec++] = {p, us, (int32_t)nt};
        if (best_t < 0.f || us < best_t) {
            best_t = us;
            *best = p;
        }
    }
    if (n_records) *n_records = nrec;
    *best_us = best_t;
    return SPC_OK;
}
