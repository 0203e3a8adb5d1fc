// Conjugate gradients for k independent right-hand sides that share one
// beta(r,c) matrix: one SpMM per iteration (the multi-vector product of
// this library) plus column-wise dot products and updates. The paper
// motivates fast SpMV by Krylov solvers such as CG, where one matrix is
// applied many times.
//
// Every scalar (alpha, beta, the residual norms, a done flag per column)
// lives in device memory, so an iteration is a fixed sequence of launches
// that can be captured once in a HIP graph and replayed; the host looks at
// the done flags every check_every iterations. A column stops (its alpha and
// beta become 0) as soon as ||r|| <= rel_tol * ||b||. Reductions run in two
// fixed passes (per-block partials, then one block), so results repeat bit
// for bit.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace spc {
spc_status spmm_launch(const spc_beta_view *A, const spc_plan *P, int k, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, int accumulate, hipStream_t stream);
spc_status spmv_launch(const spc_beta_view *A, const spc_plan *P, const void *x, void *y, int accumulate,
                       hipStream_t stream);

namespace {

constexpr int kT = 256;          // threads per block of the vector kernels
constexpr int kBlocks = 4096;    // most blocks of the vector kernels
constexpr int kMaxK = 16;

struct Scal {                    // per-column state, in device memory
    double rr[kMaxK];            // current ||r||^2
    double bb[kMaxK];            // ||b||^2
    double pq[kMaxK];
    double alpha[kMaxK];
    double beta[kMaxK];
    int done[kMaxK];
    int iter_done[kMaxK];
    int iter;                    // iterations run so far
};

// Vector kernels. The n x k arrays R, P, Q (leading dimension k) are walked
// as flat arrays, one element per thread and step: thread t of the grid
// takes elements t, t + S, t + 2S, ... with S = (threads / k) * k, so a
// thread always meets the same column q = t mod k and every load is
// coalesced. X and B (leading dimensions ldx, ldb) are addressed as
// (e / k) * ld + q. Per-column sums: each thread keeps one partial; a
// block adds the partials of its threads column by column in a fixed
// order; a second pass adds the blocks' sums in a fixed order.
constexpr int kU = 4;  // independent elements in flight per thread

struct Flat {
    int64_t N, S;      // elements, grid step
    int64_t t;         // this thread's first element (t < S, else idle)
    int q;             // its column
};

__device__ __forceinline__ Flat flat(int64_t n, int k) {
    Flat f;
    f.N = n * k;
    const int64_t threads = (int64_t)gridDim.x * kT;
    f.S = threads / k * k;
    f.t = (int64_t)blockIdx.x * kT + threadIdx.x;
    f.q = (int)(f.t % k);
    return f;
}

// part[blockIdx][q] = sum of v over this block's threads of column q.
__device__ void block_cols(double v, int k, const Flat &f, double *red, double *part) {
    red[threadIdx.x] = f.t < f.S ? v : 0.0;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int64_t base = (int64_t)blockIdx.x * kT;
        double s = 0.0;
        for (int u = 0; u < kT; ++u)
            if ((int)((base + u) % k) == (int)threadIdx.x) s += red[u];
        part[(int64_t)blockIdx.x * kMaxK + threadIdx.x] = s;
    }
}

// R = B, P = B, X = 0; partial sums of B*B per column.
template <class T>
__global__ __launch_bounds__(kT) void k_init(int64_t n, int k, const T *__restrict__ B, int64_t ldb,
                                             T *__restrict__ X, int64_t ldx, T *__restrict__ R,
                                             T *__restrict__ P, double *part) {
    __shared__ double red[kT];
    const Flat f = flat(n, k);
    double acc = 0.0;
    if (f.t < f.S) {
        for (int64_t e = f.t; e < f.N; e += f.S) {
            const int64_t i = e / k;
            const T b = B[i * ldb + f.q];
            R[e] = b;
            P[e] = b;
            X[i * ldx + f.q] = T(0);
            acc += (double)b * (double)b;
        }
    }
    block_cols(acc, k, f, red, part);
}

// Partial sums of U*V per column.
template <class T>
__global__ __launch_bounds__(kT) void k_dot(int64_t n, int k, const T *__restrict__ U, const T *__restrict__ V,
                                            double *part) {
    __shared__ double red[kT];
    const Flat f = flat(n, k);
    double a0 = 0.0, a1 = 0.0;
    if (f.t < f.S) {
        int64_t e = f.t;
        for (; e + (kU - 1) * f.S < f.N; e += kU * f.S) {
            T u[kU], v[kU];
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                u[j] = U[e + j * f.S];
                v[j] = V[e + j * f.S];
            }
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                if (j & 1) a1 += (double)u[j] * (double)v[j];
                else a0 += (double)u[j] * (double)v[j];
            }
        }
        for (; e < f.N; e += f.S) a0 += (double)U[e] * (double)V[e];
    }
    block_cols(a0 + a1, k, f, red, part);
}

// Totals of the partials of nblk blocks, in one block, fixed order.
__device__ void total_cols(const double *part, int nblk, int k, double *out, double *sm) {
    // thread t < kT adds blocks t, t + kT, ... for every column; then the
    // kT partials of each column are added in thread order
    double acc[kMaxK];
#pragma unroll
    for (int q = 0; q < kMaxK; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kT)
#pragma unroll
        for (int q = 0; q < kMaxK; ++q)
            if (q < k) acc[q] += part[(int64_t)b * kMaxK + q];
#pragma unroll
    for (int q = 0; q < kMaxK; ++q)
        if (q < k) sm[threadIdx.x * kMaxK + q] = acc[q];
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double s = 0.0;
        for (int u = 0; u < kT; ++u) s += sm[u * kMaxK + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(kT) void k_start(const double *part, int nblk, int k, Scal *s) {
    __shared__ double sm[kT * kMaxK];
    __shared__ double tot[kMaxK];
    total_cols(part, nblk, k, tot, sm);
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int q = threadIdx.x;
        s->bb[q] = tot[q];
        s->rr[q] = tot[q];
        s->done[q] = (tot[q] == 0.0) ? 1 : 0;
        s->iter_done[q] = s->done[q] ? 0 : -1;
        s->alpha[q] = 0.0;
        s->beta[q] = 0.0;
    }
    if (threadIdx.x == 0) s->iter = 0;
}

// alpha = rr / (p . q) for running columns, 0 for finished ones.
__global__ __launch_bounds__(kT) void k_alpha(const double *part, int nblk, int k, Scal *s) {
    __shared__ double sm[kT * kMaxK];
    __shared__ double tot[kMaxK];
    total_cols(part, nblk, k, tot, sm);
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int q = threadIdx.x;
        s->pq[q] = tot[q];
        s->alpha[q] = (s->done[q] || tot[q] == 0.0) ? 0.0 : s->rr[q] / tot[q];
    }
}

// R -= alpha Q; partial sums of R*R per column. (X moves with the
// direction update, which reads P anyway.)
template <class T>
__global__ __launch_bounds__(kT) void k_update(int64_t n, int k, const Scal *s, T *__restrict__ R,
                                               const T *__restrict__ Q, double *part) {
    __shared__ double red[kT];
    const Flat f = flat(n, k);
    double a0 = 0.0, a1 = 0.0;
    if (f.t < f.S) {
        const double al = s->alpha[f.q];
        int64_t e = f.t;
        for (; e + (kU - 1) * f.S < f.N; e += kU * f.S) {
            T r[kU], qq[kU];
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                const int64_t ej = e + j * f.S;
                r[j] = R[ej];
                qq[j] = Q[ej];
            }
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                const int64_t ej = e + j * f.S;
                const T rn = (T)((double)r[j] - al * (double)qq[j]);
                R[ej] = rn;
                if (j & 1) a1 += (double)rn * (double)rn;
                else a0 += (double)rn * (double)rn;
            }
        }
        for (; e < f.N; e += f.S) {
            const T rn = (T)((double)R[e] - al * (double)Q[e]);
            R[e] = rn;
            a0 += (double)rn * (double)rn;
        }
    }
    block_cols(a0 + a1, k, f, red, part);
}

// beta = rr_new / rr; convergence test; iteration count.
__global__ __launch_bounds__(kT) void k_beta(const double *part, int nblk, int k, Scal *s, double tol2) {
    __shared__ double sm[kT * kMaxK];
    __shared__ double tot[kMaxK];
    total_cols(part, nblk, k, tot, sm);
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int q = threadIdx.x;
        const int it = s->iter + 1;
        if (s->done[q]) {
            s->beta[q] = 0.0;
        } else {
            const double rn = tot[q];
            s->beta[q] = s->rr[q] > 0.0 ? rn / s->rr[q] : 0.0;
            s->rr[q] = rn;
            if (rn <= tol2 * s->bb[q]) {
                s->done[q] = 1;
                s->iter_done[q] = it;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) s->iter = s->iter + 1;
}

// X += alpha P with this iteration's direction, then P = R + beta P. A
// finished column gets beta = 0 and keeps alpha = 0, so its X and R no
// longer change.
template <class T>
__global__ __launch_bounds__(kT) void k_direction(int64_t n, int k, const Scal *s, T *__restrict__ X, int64_t ldx,
                                                  const T *__restrict__ R, T *__restrict__ P) {
    const Flat f = flat(n, k);
    if (f.t >= f.S) return;
    const double al = s->alpha[f.q];
    const double be = s->beta[f.q];
    int64_t e = f.t;
    for (; e + (kU - 1) * f.S < f.N; e += kU * f.S) {
        T x[kU], r[kU], p[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int64_t ej = e + j * f.S;
            x[j] = X[(ej / k) * ldx + f.q];
            r[j] = R[ej];
            p[j] = P[ej];
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int64_t ej = e + j * f.S;
            X[(ej / k) * ldx + f.q] = (T)((double)x[j] + al * (double)p[j]);
            P[ej] = (T)((double)r[j] + be * (double)p[j]);
        }
    }
    for (; e < f.N; e += f.S) {
        const T p = P[e];
        X[(e / k) * ldx + f.q] = (T)((double)X[(e / k) * ldx + f.q] + al * (double)p);
        P[e] = (T)((double)R[e] + be * (double)p);
    }
}

struct Work {
    void *R, *P, *Q;
    double *part;
    Scal *s;
};

int64_t work_bytes(int64_t n, int k, int dtype) {
    const int64_t es = dtype == SPC_F64 ? 8 : 4;
    const int64_t vec = (n * k * es + 255) / 256 * 256;
    return 3 * vec + (int64_t)kBlocks * kMaxK * 8 + (int64_t)((sizeof(Scal) + 255) / 256 * 256);
}

Work carve(void *ws, int64_t n, int k, int dtype) {
    const int64_t es = dtype == SPC_F64 ? 8 : 4;
    const int64_t vec = (n * k * es + 255) / 256 * 256;
    char *p = static_cast<char *>(ws);
    Work w;
    w.R = p;
    w.P = p + vec;
    w.Q = p + 2 * vec;
    w.part = reinterpret_cast<double *>(p + 3 * vec);
    w.s = reinterpret_cast<Scal *>(p + 3 * vec + (int64_t)kBlocks * kMaxK * 8);
    return w;
}

// Blocks of the vector kernels: enough for kU elements per thread and
// step, at most kBlocks.
unsigned vec_blocks(int64_t n, int k) {
    const int64_t b = div_up(n > 0 ? n * k : 1, (int64_t)kT * kU);
    return (unsigned)(b < kBlocks ? b : kBlocks);
}

template <class T>
spc_status iteration(const spc_beta_view *A, const spc_plan *P, int k, const Work &w, T *X, int64_t ldx,
                     int64_t n, double tol2, hipStream_t st) {
    const unsigned nb = vec_blocks(n, k);
    spc_status r = k == 1 ? spmv_launch(A, P, w.P, w.Q, 0, st) : spmm_launch(A, P, k, w.P, k, w.Q, k, 0, st);
    if (r != SPC_OK) return r;
    hipLaunchKernelGGL(k_dot<T>, dim3(nb), dim3(kT), 0, st, n, k, (const T *)w.P, (const T *)w.Q, w.part);
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kT), 0, st, w.part, (int)nb, k, w.s);
    hipLaunchKernelGGL(k_update<T>, dim3(nb), dim3(kT), 0, st, n, k, (const Scal *)w.s, (T *)w.R,
                       (const T *)w.Q, w.part);
    hipLaunchKernelGGL(k_beta, dim3(1), dim3(kT), 0, st, w.part, (int)nb, k, w.s, tol2);
    hipLaunchKernelGGL(k_direction<T>, dim3(nb), dim3(kT), 0, st, n, k, (const Scal *)w.s, X, ldx,
                       (const T *)w.R, (T *)w.P);
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" int64_t spc_cg_workspace_bytes(int64_t n, int32_t k, int32_t dtype) {
    if (n < 0 || k < 1 || k > kMaxK) return -1;
    return work_bytes(n, k, dtype);
}

extern "C" spc_status spc_cg_solve(const spc_beta_view *A, const spc_plan *plan, int32_t k, const void *B,
                                   int64_t ldb, void *X, int64_t ldx, double rel_tol, int32_t max_iter,
                                   int32_t check_every, int32_t use_graph, void *workspace,
                                   int64_t workspace_bytes, int32_t *iters_out, double *rel_res_out,
                                   int32_t *total_iters_out, hipStream_t stream) {
    spc_status st = check_view(A);
    if (st != SPC_OK) return st;
    SPC_REQUIRE(plan && plan->mode == 0, SPC_ERR_INVALID_ARG, "spc_cg_solve needs a mode-0 plan of A");
    SPC_REQUIRE(plan->A.block_rowptr == A->block_rowptr && plan->A.values == A->values &&
                    plan->A.block_masks == A->block_masks && plan->A.n_rows == A->n_rows,
                SPC_ERR_INVALID_ARG, "plan was built for a different matrix view");
    SPC_REQUIRE((reinterpret_cast<uintptr_t>(A->values) & 15u) == 0, SPC_ERR_INVALID_ARG,
                "spc_cg_solve needs a 16-byte aligned values array");
    SPC_REQUIRE(A->n_rows == A->n_cols, SPC_ERR_INVALID_ARG, "CG needs a square matrix");
    SPC_REQUIRE(k >= 1 && k <= kMaxK, SPC_ERR_CAPACITY, "k must be in 1..%d", kMaxK);
    SPC_REQUIRE(ldb >= k && ldx >= k, SPC_ERR_INVALID_ARG, "leading dimensions must be at least k");
    SPC_REQUIRE(rel_tol > 0.0 && max_iter >= 0 && check_every >= 1, SPC_ERR_INVALID_ARG, "bad iteration controls");
    const int64_t n = A->n_rows;
    SPC_REQUIRE(workspace && workspace_bytes >= work_bytes(n, k, A->dtype), SPC_ERR_INVALID_ARG,
                "workspace smaller than spc_cg_workspace_bytes");
    SPC_REQUIRE(B && X, SPC_ERR_INVALID_ARG, "null B or X");
    {
        const uint64_t es = A->dtype == SPC_F64 ? 8 : 4;
        SPC_REQUIRE((uint64_t)n * (uint64_t)k * es < 0xf0000000ull, SPC_ERR_CAPACITY,
                    "n * k must stay below 3.75 GiB (32-bit offsets of the product)");
        SPC_REQUIRE(reinterpret_cast<uintptr_t>(B) % es == 0 && reinterpret_cast<uintptr_t>(X) % es == 0,
                    SPC_ERR_INVALID_ARG, "B and X must be aligned to the element size");
    }
    const Work w = carve(workspace, n, k, A->dtype);
    if (stream == nullptr) use_graph = 0;  // the legacy default stream cannot be captured
    const double tol2 = rel_tol * rel_tol;
    const unsigned nb = vec_blocks(n, k);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    };
    st = with_dtype(A->dtype, [&](auto tv) -> spc_status {
        using T = decltype(tv);
        hipLaunchKernelGGL(k_init<T>, dim3(nb), dim3(kT), 0, stream, n, k, (const T *)B, ldb, (T *)X, ldx,
                           (T *)w.R, (T *)w.P, w.part);
        hipLaunchKernelGGL(k_start, dim3(1), dim3(kT), 0, stream, w.part, (int)nb, k, w.s);
        SPC_HIP(hipGetLastError());
        if (use_graph) {
            SPC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            spc_status r = iteration<T>(A, plan, k, w, (T *)X, ldx, n, tol2, stream);
            hipError_t e = hipStreamEndCapture(stream, &graph);
            if (r != SPC_OK) return r;
            SPC_HIP(e);
            SPC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        std::vector<int> done(k);
        int it = 0;
        while (it < max_iter) {
            const int batch = check_every < max_iter - it ? check_every : max_iter - it;
            for (int b = 0; b < batch; ++b) {
                if (use_graph) {
                    SPC_HIP(hipGraphLaunch(exec, stream));
                } else {
                    spc_status r = iteration<T>(A, plan, k, w, (T *)X, ldx, n, tol2, stream);
                    if (r != SPC_OK) return r;
                }
            }
            it += batch;
            SPC_HIP(hipMemcpyAsync(done.data(), w.s->done, sizeof(int) * k, hipMemcpyDeviceToHost, stream));
            SPC_HIP(hipStreamSynchronize(stream));
            bool all = true;
            for (int q = 0; q < k; ++q) all = all && done[q];
            if (all) break;
        }
        Scal hs;
        SPC_HIP(hipMemcpyAsync(&hs, w.s, sizeof(Scal), hipMemcpyDeviceToHost, stream));
        SPC_HIP(hipStreamSynchronize(stream));
        for (int q = 0; q < k; ++q) {
            if (iters_out) iters_out[q] = hs.iter_done[q];
            if (rel_res_out) rel_res_out[q] = hs.bb[q] > 0.0 ? std::sqrt(hs.rr[q] / hs.bb[q]) : 0.0;
        }
        if (total_iters_out) *total_iters_out = hs.iter;
        return SPC_OK;
    });
    cleanup();
    return st;
}
