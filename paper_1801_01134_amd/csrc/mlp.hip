// The learned kernel selector: a 16 -> 64 -> 64 -> K ReLU network in FP32
// (K kernel classes: the six block shapes, or eight with the two "test"
// kernels of Algorithm 2), trained on the device by hand-written forward,
// backward and Adam kernels.
//
// The paper picks a kernel from recorded speeds with one polynomial per
// kernel of its Avg(r,c) (section "Performance polynomial interpolation"),
// and its conclusions name selection from several matrix properties as the
// next step; this network is that step. It maps standardized features
// x^ = (x - mu) / sd to one score per block shape, trained to predict
// tau_k = log2(t_k / min_j t_j) (the kernel's time relative to the best one)
// under the mean squared error; the selected shape is the smallest score.
//
// Training runs in ONE workgroup: a step's batch (at most 64 rows) keeps
// its activations in LDS with the parameters, so a whole run of steps is a
// single launch with no grid-wide synchronisation. Each thread owns the
// parameters p = tid, tid + 256, ...: it forms their gradients (sums over
// the batch) and applies Adam to them in place.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace spc {
namespace {

constexpr int NI = SPC_MLP_N_IN, NH = SPC_MLP_N_HIDDEN;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH;
// layout of a network with NO outputs: W3[NO][NH] at OW3, then b3[NO]
template <int NO>
struct Lay {
    static_assert(NO >= 1 && NO <= 8, "the output buffers hold 8 scores per row");
    static constexpr int OB3 = OW3 + NO * NH, NP = OB3 + NO;
};
static_assert(Lay<SPC_MLP_N_OUT>::NP == SPC_MLP_N_PARAMS, "parameter count");
static_assert(Lay<SPC_MLP_MAX_OUT>::NP == SPC_MLP_PARAMS(SPC_MLP_MAX_OUT), "parameter count");
constexpr int NPMAX = Lay<SPC_MLP_MAX_OUT>::NP;
constexpr int kMT = 256;                          // threads of the training workgroup
constexpr int kMaxB = SPC_MLP_MAX_BATCH;
constexpr int kOwn = (NPMAX + kMT - 1) / kMT;     // parameters per thread

struct MlpSmem {
    float P[NPMAX + 2];
    float X[kMaxB * NI];
    float H1[kMaxB * NH];
    float H2[kMaxB * NH];
    float O[kMaxB * 8];       // outputs, then dL/do
    float D2[kMaxB * NH];     // dL/dz2
    float D1[kMaxB * NH];     // dL/dz1
    float red[kMT];
};

struct Adam {
    float lr, b1, b2, eps;
};

// Gradient of parameter p from the batch's activations (B rows).
template <int NO>
__device__ __forceinline__ float param_grad(const MlpSmem &s, int p, int B) {
    constexpr int OB3 = Lay<NO>::OB3;
    float g = 0.f;
    if (p < OB1) {                      // W1[o][i]
        const int o = (p - OW1) / NI, i = (p - OW1) % NI;
        for (int b = 0; b < B; ++b) g = fmaf(s.D1[b * NH + o], s.X[b * NI + i], g);
    } else if (p < OW2) {               // b1[o]
        const int o = p - OB1;
        for (int b = 0; b < B; ++b) g += s.D1[b * NH + o];
    } else if (p < OB2) {               // W2[o][i]
        const int o = (p - OW2) / NH, i = (p - OW2) % NH;
        for (int b = 0; b < B; ++b) g = fmaf(s.D2[b * NH + o], s.H1[b * NH + i], g);
    } else if (p < OW3) {               // b2[o]
        const int o = p - OB2;
        for (int b = 0; b < B; ++b) g += s.D2[b * NH + o];
    } else if (p < OB3) {               // W3[k][i]
        const int k = (p - OW3) / NH, i = (p - OW3) % NH;
        for (int b = 0; b < B; ++b) g = fmaf(s.O[b * 8 + k], s.H2[b * NH + i], g);
    } else {                            // b3[k]
        const int k = p - OB3;
        for (int b = 0; b < B; ++b) g += s.O[b * 8 + k];
    }
    return g;
}

// Forward and backward of one batch; leaves dL/do in O, dL/dz2 in D2,
// dL/dz1 in D1 and returns the batch loss in red[0] (thread 0 reads it).
template <int NO>
__device__ void forward_backward(MlpSmem &s, const float *__restrict__ X, const float *__restrict__ tau,
                                 const float *__restrict__ mu, const float *__restrict__ sd,
                                 const int32_t *__restrict__ rows, int B) {
    constexpr int OB3 = Lay<NO>::OB3;
    const int t = threadIdx.x;
    for (int e = t; e < B * NI; e += kMT) {
        const int b = e / NI, i = e % NI;
        const int64_t r = rows[b];
        s.X[e] = (X[r * NI + i] - mu[i]) / sd[i];
    }
    __syncthreads();
    for (int e = t; e < B * NH; e += kMT) {
        const int b = e / NH, o = e % NH;
        float z = s.P[OB1 + o];
#pragma unroll
        for (int i = 0; i < NI; ++i) z = fmaf(s.P[OW1 + o * NI + i], s.X[b * NI + i], z);
        s.H1[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    for (int e = t; e < B * NH; e += kMT) {
        const int b = e / NH, o = e % NH;
        float z = s.P[OB2 + o];
#pragma unroll 16
        for (int i = 0; i < NH; ++i) z = fmaf(s.P[OW2 + o * NH + i], s.H1[b * NH + i], z);
        s.H2[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    float sq = 0.f;
    const float scale = 2.0f / (float)(B * NO);
    for (int e = t; e < B * NO; e += kMT) {
        const int b = e / NO, k = e % NO;
        float z = s.P[OB3 + k];
#pragma unroll 16
        for (int i = 0; i < NH; ++i) z = fmaf(s.P[OW3 + k * NH + i], s.H2[b * NH + i], z);
        const float d = z - tau[(int64_t)rows[b] * NO + k];
        sq = fmaf(d, d, sq);
        s.O[b * 8 + k] = scale * d;
    }
    s.red[t] = sq;
    __syncthreads();
    for (int st = kMT / 2; st > 0; st >>= 1) {
        if (t < st) s.red[t] += s.red[t + st];
        __syncthreads();
    }
    for (int e = t; e < B * NH; e += kMT) {
        const int b = e / NH, o = e % NH;
        float g = 0.f;
#pragma unroll
        for (int k = 0; k < NO; ++k) g = fmaf(s.O[b * 8 + k], s.P[OW3 + k * NH + o], g);
        s.D2[e] = s.H2[e] > 0.f ? g : 0.f;
    }
    __syncthreads();
    for (int e = t; e < B * NH; e += kMT) {
        const int b = e / NH, i = e % NH;
        float g = 0.f;
#pragma unroll 16
        for (int o = 0; o < NH; ++o) g = fmaf(s.D2[b * NH + o], s.P[OW2 + o * NH + i], g);
        s.D1[e] = s.H1[e] > 0.f ? g : 0.f;
    }
    __syncthreads();
}

template <int NO>
__global__ __launch_bounds__(kMT) void k_mlp_grad(const float *__restrict__ params, const float *__restrict__ mu,
                                                  const float *__restrict__ sd, const float *__restrict__ X,
                                                  const float *__restrict__ tau, const int32_t *__restrict__ rows,
                                                  int B, float *__restrict__ grad, float *__restrict__ loss) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MlpSmem &s = *reinterpret_cast<MlpSmem *>(smem_raw);
    constexpr int NP = Lay<NO>::NP;
    for (int p = threadIdx.x; p < NP; p += kMT) s.P[p] = params[p];
    __syncthreads();
    forward_backward<NO>(s, X, tau, mu, sd, rows, B);
    if (threadIdx.x == 0) loss[0] = s.red[0] / (float)(B * NO);
    for (int p = threadIdx.x; p < NP; p += kMT) grad[p] = param_grad<NO>(s, p, B);
}

template <int NO>
__global__ __launch_bounds__(kMT) void k_mlp_train(float *__restrict__ params, float *__restrict__ am,
                                                   float *__restrict__ av, int step0, Adam opt,
                                                   const float *__restrict__ mu, const float *__restrict__ sd,
                                                   const float *__restrict__ X, const float *__restrict__ tau,
                                                   const int32_t *__restrict__ order, int n_steps, int B,
                                                   float *__restrict__ losses) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MlpSmem &s = *reinterpret_cast<MlpSmem *>(smem_raw);
    constexpr int NP = Lay<NO>::NP;
    const int t = threadIdx.x;
    for (int p = t; p < NP; p += kMT) s.P[p] = params[p];
    // this thread's Adam moments stay in registers for the whole run
    float m[kOwn], v[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
        const int p = t + q * kMT;
        m[q] = p < NP ? am[p] : 0.f;
        v[q] = p < NP ? av[p] : 0.f;
    }
    __syncthreads();
    for (int st = 0; st < n_steps; ++st) {
        forward_backward<NO>(s, X, tau, mu, sd, order + (int64_t)st * B, B);
        if (t == 0) losses[st] = s.red[0] / (float)(B * NO);
        const int step = step0 + st + 1;
        const float c1 = (float)(1.0 - pow((double)opt.b1, (double)step));
        const float c2 = (float)(1.0 - pow((double)opt.b2, (double)step));
#pragma unroll
        for (int q = 0; q < kOwn; ++q) {
            const int p = t + q * kMT;
            if (p < NP) {
                const float g = param_grad<NO>(s, p, B);
                m[q] = opt.b1 * m[q] + (1.f - opt.b1) * g;
                v[q] = opt.b2 * v[q] + (1.f - opt.b2) * g * g;
                const float mh = m[q] / c1, vh = v[q] / c2;
                s.P[p] -= opt.lr * mh / (sqrtf(vh) + opt.eps);
            }
        }
        __syncthreads();
    }
    for (int p = t; p < NP; p += kMT) params[p] = s.P[p];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
        const int p = t + q * kMT;
        if (p < NP) {
            am[p] = m[q];
            av[p] = v[q];
        }
    }
}

// One thread per sample: scores and the smallest-score class (lowest index
// on ties).
template <int NO>
__global__ __launch_bounds__(256) void k_mlp_infer(const float *__restrict__ params, const float *__restrict__ mu,
                                                   const float *__restrict__ sd, const float *__restrict__ X,
                                                   int n, float *__restrict__ scores, int32_t *__restrict__ choice) {
    constexpr int NP = Lay<NO>::NP, OB3 = Lay<NO>::OB3;
    __shared__ float P[NP + 2];
    for (int p = threadIdx.x; p < NP; p += blockDim.x) P[p] = params[p];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float x[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) x[i] = (X[(int64_t)b * NI + i] - mu[i]) / sd[i];
    float h1[NH];
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float z = P[OB1 + o];
#pragma unroll
        for (int i = 0; i < NI; ++i) z = fmaf(P[OW1 + o * NI + i], x[i], z);
        h1[o] = z > 0.f ? z : 0.f;
    }
    float out[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) out[k] = P[OB3 + k];
    for (int o = 0; o < NH; ++o) {
        float z = P[OB2 + o];
#pragma unroll
        for (int i = 0; i < NH; ++i) z = fmaf(P[OW2 + o * NH + i], h1[i], z);
        const float h2 = z > 0.f ? z : 0.f;
#pragma unroll
        for (int k = 0; k < NO; ++k) out[k] = fmaf(P[OW3 + k * NH + o], h2, out[k]);
    }
    int best = 0;
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        if (scores) scores[(int64_t)b * NO + k] = out[k];
        if (out[k] < out[best]) best = k;
    }
    if (choice) choice[b] = best;
}

// Mean and population spread of each feature column (two passes in double);
// a spread below 1e-12 is replaced by 1.
__global__ __launch_bounds__(256) void k_mlp_standardizer(const float *__restrict__ X, int n,
                                                          float *__restrict__ mu, float *__restrict__ sd) {
    __shared__ double red[256];
    for (int i = 0; i < NI; ++i) {
        double a = 0.0;
        for (int b = threadIdx.x; b < n; b += 256) a += (double)X[(int64_t)b * NI + i];
        red[threadIdx.x] = a;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        const double mean = red[0] / (double)n;
        __syncthreads();
        double q = 0.0;
        for (int b = threadIdx.x; b < n; b += 256) {
            const double d = (double)X[(int64_t)b * NI + i] - mean;
            q += d * d;
        }
        red[threadIdx.x] = q;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double s = sqrt(red[0] / (double)n);
            mu[i] = (float)mean;
            sd[i] = (float)(s > 1e-12 ? s : 1.0);
        }
        __syncthreads();
    }
}

// tau[b][k] = log2(t[b][k] / min_j t[b][j]), in double, rounded once.
template <int NO>
__global__ void k_mlp_targets(const float *__restrict__ times, int n, float *__restrict__ tau) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double mn = (double)times[(int64_t)b * NO];
#pragma unroll
    for (int k = 1; k < NO; ++k) mn = fmin(mn, (double)times[(int64_t)b * NO + k]);
#pragma unroll
    for (int k = 0; k < NO; ++k) tau[(int64_t)b * NO + k] = (float)log2((double)times[(int64_t)b * NO + k] / mn);
}

constexpr size_t kSmemBytes = sizeof(MlpSmem);
static_assert(kSmemBytes <= 160 * 1024, "training workgroup must fit in LDS");

spc_status check_out(int32_t n_out) {
    SPC_REQUIRE(n_out == SPC_MLP_N_OUT || n_out == SPC_MLP_MAX_OUT, SPC_ERR_INVALID_ARG,
                "n_out must be %d (the six shapes) or %d (with the two test kernels), got %d", SPC_MLP_N_OUT,
                SPC_MLP_MAX_OUT, n_out);
    return SPC_OK;
}

// f(integral_constant<NO>) for the two output counts
template <class F>
auto with_out(int n_out, F &&f) {
    if (n_out == SPC_MLP_MAX_OUT) return f(std::integral_constant<int, SPC_MLP_MAX_OUT>{});
    return f(std::integral_constant<int, SPC_MLP_N_OUT>{});
}

spc_status check_rows(const int32_t *rows, int64_t count, int32_t n) {
    SPC_REQUIRE(rows != nullptr, SPC_ERR_INVALID_ARG, "null row index array");
    for (int64_t k = 0; k < count; ++k)
        SPC_REQUIRE(rows[k] >= 0 && rows[k] < n, SPC_ERR_INDEX_RANGE, "row index %d at position %lld outside [0, %d)",
                    rows[k], (long long)k, n);
    return SPC_OK;
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_mlp_standardizer(const float *X, int32_t n, float *mu_out, float *sd_out,
                                           hipStream_t stream) {
    SPC_REQUIRE(n >= 1 && X && mu_out && sd_out, SPC_ERR_INVALID_ARG, "need n >= 1 and non-null arrays");
    hipLaunchKernelGGL(k_mlp_standardizer, dim3(1), dim3(256), 0, stream, X, n, mu_out, sd_out);
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

extern "C" spc_status spc_mlp_targets(const float *times, int32_t n, int32_t n_out, float *tau_out,
                                      hipStream_t stream) {
    SPC_REQUIRE(n >= 0 && (n == 0 || (times && tau_out)), SPC_ERR_INVALID_ARG, "bad arguments");
    spc_status st = check_out(n_out);
    if (st != SPC_OK) return st;
    if (n == 0) return SPC_OK;
    with_out(n_out, [&](auto no) {
        hipLaunchKernelGGL(k_mlp_targets<decltype(no)::value>, dim3((n + 255) / 256), dim3(256), 0, stream, times, n,
                           tau_out);
        return 0;
    });
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

extern "C" spc_status spc_mlp_loss_grad(const float *params, const float *mu, const float *sd, const float *X,
                                        const float *tau, int32_t n, int32_t n_out, const int32_t *rows,
                                        int32_t batch, float *grad_out, float *loss_out, hipStream_t stream) {
    SPC_REQUIRE(params && mu && sd && X && tau && grad_out && loss_out, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(batch >= 1 && batch <= kMaxB, SPC_ERR_CAPACITY, "batch must be in 1..%d", kMaxB);
    spc_status st = check_out(n_out);
    if (st != SPC_OK) return st;
    st = check_rows(rows, batch, n);
    if (st != SPC_OK) return st;
    DevBuf d;
    SPC_HIP(d.alloc(sizeof(int32_t) * batch));
    SPC_HIP(hipMemcpyAsync(d.p, rows, sizeof(int32_t) * batch, hipMemcpyHostToDevice, stream));
    st = with_out(n_out, [&](auto no) -> spc_status {
        auto k = k_mlp_grad<decltype(no)::value>;
        SPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kSmemBytes));
        hipLaunchKernelGGL(k, dim3(1), dim3(kMT), kSmemBytes, stream, params, mu, sd, X, tau, d.as<int32_t>(), batch,
                           grad_out, loss_out);
        return SPC_OK;
    });
    if (st != SPC_OK) return st;
    SPC_HIP(hipGetLastError());
    SPC_HIP(hipStreamSynchronize(stream));  // the row buffer is freed on return
    return SPC_OK;
}

extern "C" spc_status spc_mlp_train(float *params, float *adam_m, float *adam_v, int32_t step0, float lr,
                                    const float *mu, const float *sd, const float *X, const float *tau, int32_t n,
                                    int32_t n_out, const int32_t *order, int32_t n_steps, int32_t batch,
                                    float *losses_out, hipStream_t stream) {
    SPC_REQUIRE(params && adam_m && adam_v && mu && sd && X && tau && losses_out, SPC_ERR_INVALID_ARG,
                "null argument");
    if (spc_status so = check_out(n_out); so != SPC_OK) return so;
    SPC_REQUIRE(batch >= 1 && batch <= kMaxB, SPC_ERR_CAPACITY, "batch must be in 1..%d", kMaxB);
    SPC_REQUIRE(n_steps >= 0 && step0 >= 0 && lr > 0.f, SPC_ERR_INVALID_ARG, "bad step count or learning rate");
    if (n_steps == 0) return SPC_OK;
    spc_status st = check_rows(order, (int64_t)n_steps * batch, n);
    if (st != SPC_OK) return st;
    DevBuf d;
    const size_t bytes = sizeof(int32_t) * (size_t)n_steps * batch;
    SPC_HIP(d.alloc(bytes));
    SPC_HIP(hipMemcpyAsync(d.p, order, bytes, hipMemcpyHostToDevice, stream));
    const Adam opt{lr, 0.9f, 0.999f, 1e-8f};
    st = with_out(n_out, [&](auto no) -> spc_status {
        auto k = k_mlp_train<decltype(no)::value>;
        SPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kSmemBytes));
        hipLaunchKernelGGL(k, dim3(1), dim3(kMT), kSmemBytes, stream, params, adam_m, adam_v, step0, opt, mu, sd, X,
                           tau, d.as<int32_t>(), n_steps, batch, losses_out);
        return SPC_OK;
    });
    if (st != SPC_OK) return st;
    SPC_HIP(hipGetLastError());
    SPC_HIP(hipStreamSynchronize(stream));
    return SPC_OK;
}

extern "C" spc_status spc_mlp_infer(const float *params, const float *mu, const float *sd, const float *X,
                                    int32_t n, int32_t n_out, float *scores_out, int32_t *choice_out,
                                    hipStream_t stream) {
    SPC_REQUIRE(params && mu && sd && n >= 0 && (n == 0 || X), SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(scores_out || choice_out, SPC_ERR_INVALID_ARG, "need scores_out or choice_out");
    if (spc_status so = check_out(n_out); so != SPC_OK) return so;
    if (n == 0) return SPC_OK;
    with_out(n_out, [&](auto no) {
        hipLaunchKernelGGL(k_mlp_infer<decltype(no)::value>, dim3((n + 255) / 256), dim3(256), 0, stream, params, mu,
                           sd, X, n, scores_out, choice_out);
        return 0;
    });
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}
