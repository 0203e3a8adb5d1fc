// Kernel selection (section "Performance prediction and optimal kernel
// selection").
//
// Interpolation (the paper's method, subsection "Performance polynomial
// interpolation"): for every shape a polynomial of the shape's speed
// (GFlop/s) against its Avg(r,c) is fitted by least squares to recorded
// runs; a new matrix gets each shape's predicted speed at its own Avg,
// clamped to the range seen in the records, and the fastest prediction wins.
// The fit is host code (at most a few thousand records, degree <= 3):
// Householder QR of the column-scaled Vandermonde matrix.
//
// MLP (this library's extension): the trained network's scores, computed by
// the inference kernel; the smallest predicted log time ratio wins.
//
// Both choose among kernel classes: the six shapes, and optionally the two
// "test" kernels of Algorithm 2 (beta(1,8) and beta(2,4) in plan mode 2),
// whose Avg is that of their shape.
#include <algorithm>
#include <cmath>
#include <set>
#include <vector>

#include "common.hpp"

extern "C" spc_status spc_mlp_infer(const float *params, const float *mu, const float *sd, const float *X,
                                    int32_t n, int32_t n_out, float *scores_out, int32_t *choice_out,
                                    hipStream_t stream);

namespace spc {
namespace {

constexpr int kMaxDeg = 3;
constexpr int kMaxDegShare = 2;

// Least-squares solution of V c = rhs for an n x m design matrix V
// (row-major, overwritten): columns scaled to unit norm, Householder QR
// applied to the right-hand side as it goes, back substitution, unscaled.
std::vector<double> lstsq(std::vector<double> &V, std::vector<double> rhs, int n, int m) {
    std::vector<double> scale(m, 1.0);
    for (int j = 0; j < m; ++j) {
        double q = 0.0;
        for (int i = 0; i < n; ++i) q += V[(size_t)i * m + j] * V[(size_t)i * m + j];
        scale[j] = q > 0.0 ? std::sqrt(q) : 1.0;
        for (int i = 0; i < n; ++i) V[(size_t)i * m + j] /= scale[j];
    }
    // Householder QR, applied to the right-hand side as it goes
    for (int j = 0; j < m; ++j) {
        double nrm = 0.0;
        for (int i = j; i < n; ++i) nrm += V[(size_t)i * m + j] * V[(size_t)i * m + j];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = V[(size_t)j * m + j] > 0 ? -nrm : nrm;
        std::vector<double> u(n - j);
        for (int i = j; i < n; ++i) u[i - j] = V[(size_t)i * m + j];
        u[0] -= alpha;
        double un = 0.0;
        for (double w : u) un += w * w;
        if (un == 0.0) continue;
        for (int k = j; k < m; ++k) {
            double dot = 0.0;
            for (int i = j; i < n; ++i) dot += u[i - j] * V[(size_t)i * m + k];
            const double f = 2.0 * dot / un;
            for (int i = j; i < n; ++i) V[(size_t)i * m + k] -= f * u[i - j];
        }
        double dot = 0.0;
        for (int i = j; i < n; ++i) dot += u[i - j] * rhs[i];
        const double f = 2.0 * dot / un;
        for (int i = j; i < n; ++i) rhs[i] -= f * u[i - j];
    }
    std::vector<double> c(m, 0.0);
    for (int j = m - 1; j >= 0; --j) {
        double v = rhs[j];
        for (int k = j + 1; k < m; ++k) v -= V[(size_t)j * m + k] * c[k];
        const double dj = V[(size_t)j * m + j];
        c[j] = dj != 0.0 ? v / dj : 0.0;
    }
    for (int j = 0; j < m; ++j) c[j] /= scale[j];
    return c;
}

// Least-squares coefficients (lowest power first) of a degree-d polynomial.
std::vector<double> polyfit(const std::vector<double> &a, const std::vector<double> &s, int d) {
    const int n = (int)a.size(), m = d + 1;
    std::vector<double> V((size_t)n * m);
    for (int i = 0; i < n; ++i) {
        double p = 1.0;
        for (int j = 0; j < m; ++j) {
            V[(size_t)i * m + j] = p;
            p *= a[i];
        }
    }
    return lstsq(V, s, n, m);
}

// Least-squares coefficients of the tensor polynomial sum c[i][j] a^i u^j,
// i <= da, j <= du (c row-major in i, then j).
std::vector<double> polyfit2(const std::vector<double> &a, const std::vector<double> &u,
                             const std::vector<double> &s, int da, int du) {
    const int n = (int)a.size(), m = (da + 1) * (du + 1);
    std::vector<double> V((size_t)n * m);
    for (int r = 0; r < n; ++r) {
        double pa = 1.0;
        for (int i = 0; i <= da; ++i) {
            double pu = 1.0;
            for (int j = 0; j <= du; ++j) {
                V[(size_t)r * m + i * (du + 1) + j] = pa * pu;
                pu *= u[r];
            }
            pa *= a[r];
        }
    }
    return lstsq(V, s, n, m);
}

}  // namespace
}  // namespace spc

struct spc_selector {
    bool has_interp = false;
    int n_interp = 0;  // classes of the 1-D fit (6 or 8)
    double coef[SPC_N_CLASSES][spc::kMaxDeg + 1] = {};
    int deg[SPC_N_CLASSES] = {};
    double lo[SPC_N_CLASSES] = {}, hi[SPC_N_CLASSES] = {};
    // 2-D fit: speed against (Avg, log2 of the compute-unit share)
    bool has_interp2 = false;
    double coef2[SPC_N_SHAPES][spc::kMaxDeg + 1][spc::kMaxDegShare + 1] = {};
    int deg2a[SPC_N_SHAPES] = {}, deg2u[SPC_N_SHAPES] = {};
    double lo2[SPC_N_SHAPES] = {}, hi2[SPC_N_SHAPES] = {}, ulo = 0.0, uhi = 0.0;
    bool has_mlp = false;
    int n_mlp = 0;  // network outputs (6 or 8)
    int device = -1;
    float *d_buf = nullptr;  // params | mu | sd | features | scores, then one int32 choice
};

namespace {
constexpr size_t kParamsOff = 0, kMuOff = SPC_MLP_PARAMS(SPC_MLP_MAX_OUT), kSdOff = kMuOff + SPC_MLP_N_IN,
                 kFeatOff = kSdOff + SPC_MLP_N_IN, kScoreOff = kFeatOff + SPC_MLP_N_IN,
                 kChoiceOff = kScoreOff + 8, kBufFloats = kChoiceOff + 4;
}

using namespace spc;

extern "C" int32_t spc_class_shape(int32_t k) {
    if (k >= 0 && k < SPC_N_SHAPES) return k;
    if (k == SPC_CLASS_TEST_B1X8) return 0;
    if (k == SPC_CLASS_TEST_B2X4) return 1;
    return -1;
}

extern "C" int32_t spc_class_mode(int32_t k) {
    return (k == SPC_CLASS_TEST_B1X8 || k == SPC_CLASS_TEST_B2X4) ? 2 : -1;
}

extern "C" int32_t spc_selector_n_classes(const spc_selector *sel, int32_t method) {
    if (!sel) return 0;
    if (method == SPC_SEL_INTERP) return sel->has_interp ? sel->n_interp : 0;
    if (method == SPC_SEL_MLP) return sel->has_mlp ? sel->n_mlp : 0;
    return 0;
}

extern "C" spc_status spc_selector_create(spc_selector **out) {
    SPC_REQUIRE(out != nullptr, SPC_ERR_INVALID_ARG, "null output pointer");
    *out = new spc_selector();
    return SPC_OK;
}

extern "C" spc_status spc_selector_destroy(spc_selector *sel) {
    if (!sel) return SPC_OK;
    if (sel->d_buf) (void)hipFree(sel->d_buf);
    delete sel;
    return SPC_OK;
}

extern "C" spc_status spc_selector_fit_interp(spc_selector *sel, int32_t n, int32_t n_classes, const double *avg,
                                              const double *speed, int32_t degree) {
    SPC_REQUIRE(sel && avg && speed, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(n >= 1, SPC_ERR_INVALID_ARG, "need at least one record");
    SPC_REQUIRE(n_classes == SPC_N_SHAPES || n_classes == SPC_N_CLASSES, SPC_ERR_INVALID_ARG,
                "n_classes must be %d or %d, got %d", SPC_N_SHAPES, SPC_N_CLASSES, n_classes);
    SPC_REQUIRE(degree >= 0 && degree <= kMaxDeg, SPC_ERR_INVALID_ARG, "degree must be in 0..%d", kMaxDeg);
    const int K = n_classes;
    for (int64_t k = 0; k < (int64_t)n * K; ++k)
        SPC_REQUIRE(std::isfinite(avg[k]) && std::isfinite(speed[k]), SPC_ERR_INVALID_ARG,
                    "record %lld is not finite", (long long)(k / K));
    for (int s = 0; s < K; ++s) {
        std::vector<double> a(n), v(n);
        std::set<double> distinct;
        for (int i = 0; i < n; ++i) {
            a[i] = avg[(int64_t)i * K + s];
            v[i] = speed[(int64_t)i * K + s];
            distinct.insert(a[i]);
        }
        // fewer distinct abscissae than coefficients: lower the degree
        const int d = std::min<int>(degree, std::max<int>(0, (int)distinct.size() - 1));
        const std::vector<double> c = polyfit(a, v, d);
        for (int j = 0; j <= kMaxDeg; ++j) sel->coef[s][j] = j <= d ? c[j] : 0.0;
        sel->deg[s] = d;
        sel->lo[s] = *std::min_element(a.begin(), a.end());
        sel->hi[s] = *std::max_element(a.begin(), a.end());
    }
    sel->n_interp = K;
    sel->has_interp = true;
    return SPC_OK;
}

extern "C" spc_status spc_selector_fit_interp2d(spc_selector *sel, int32_t n, const double *avg,
                                                const double *log2_share, const double *speed, int32_t deg_avg,
                                                int32_t deg_share) {
    SPC_REQUIRE(sel && avg && log2_share && speed, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(n >= 1, SPC_ERR_INVALID_ARG, "need at least one record");
    SPC_REQUIRE(deg_avg >= 0 && deg_avg <= kMaxDeg && deg_share >= 0 && deg_share <= kMaxDegShare,
                SPC_ERR_INVALID_ARG, "degrees must be in 0..%d (Avg) and 0..%d (share)", kMaxDeg, kMaxDegShare);
    for (int64_t k = 0; k < (int64_t)n * SPC_N_SHAPES; ++k)
        SPC_REQUIRE(std::isfinite(avg[k]) && std::isfinite(speed[k]), SPC_ERR_INVALID_ARG,
                    "record %lld is not finite", (long long)(k / SPC_N_SHAPES));
    std::set<double> us;
    for (int i = 0; i < n; ++i) {
        SPC_REQUIRE(std::isfinite(log2_share[i]), SPC_ERR_INVALID_ARG, "share of record %d is not finite", i);
        us.insert(log2_share[i]);
    }
    const int du0 = std::min<int>(deg_share, (int)us.size() - 1);
    std::vector<double> u(log2_share, log2_share + n);
    for (int s = 0; s < SPC_N_SHAPES; ++s) {
        std::vector<double> a(n), v(n);
        std::set<double> distinct;
        for (int i = 0; i < n; ++i) {
            a[i] = avg[(int64_t)i * SPC_N_SHAPES + s];
            v[i] = speed[(int64_t)i * SPC_N_SHAPES + s];
            distinct.insert(a[i]);
        }
        int da = std::min<int>(deg_avg, std::max<int>(0, (int)distinct.size() - 1)), du = du0;
        // no more coefficients than records: lower the share degree, then Avg's
        while ((da + 1) * (du + 1) > n) {
            if (du > 0) --du;
            else --da;
        }
        const std::vector<double> c = polyfit2(a, u, v, da, du);
        for (int i = 0; i <= kMaxDeg; ++i)
            for (int j = 0; j <= kMaxDegShare; ++j)
                sel->coef2[s][i][j] = (i <= da && j <= du) ? c[(size_t)i * (du + 1) + j] : 0.0;
        sel->deg2a[s] = da;
        sel->deg2u[s] = du;
        sel->lo2[s] = *std::min_element(a.begin(), a.end());
        sel->hi2[s] = *std::max_element(a.begin(), a.end());
    }
    sel->ulo = *us.begin();
    sel->uhi = *us.rbegin();
    sel->has_interp2 = true;
    return SPC_OK;
}

extern "C" spc_status spc_selector_interp2d_coeffs(const spc_selector *sel, double *coeffs_out, double *lo_out,
                                                   double *hi_out, double *share_range_out) {
    SPC_REQUIRE(sel && coeffs_out, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(sel->has_interp2, SPC_ERR_NO_MODEL, "the selector has no 2-D interpolation fit");
    constexpr int M = (kMaxDeg + 1) * (kMaxDegShare + 1);
    for (int s = 0; s < SPC_N_SHAPES; ++s) {
        for (int i = 0; i <= kMaxDeg; ++i)
            for (int j = 0; j <= kMaxDegShare; ++j) coeffs_out[s * M + i * (kMaxDegShare + 1) + j] = sel->coef2[s][i][j];
        if (lo_out) lo_out[s] = sel->lo2[s];
        if (hi_out) hi_out[s] = sel->hi2[s];
    }
    if (share_range_out) {
        share_range_out[0] = sel->ulo;
        share_range_out[1] = sel->uhi;
    }
    return SPC_OK;
}

extern "C" spc_status spc_select_kernel_at(spc_selector *sel, const float *features, double cu_share,
                                           int32_t *shape_out, float *scores_out) {
    SPC_REQUIRE(sel && features && shape_out, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(std::isfinite(cu_share) && cu_share > 0.0 && cu_share <= 1.0, SPC_ERR_INVALID_ARG,
                "cu_share must be in (0, 1]");
    SPC_REQUIRE(sel->has_interp2, SPC_ERR_NO_MODEL, "the selector has no 2-D interpolation fit");
    const double u = std::min(std::max(std::log2(cu_share), sel->ulo), sel->uhi);
    double best = 0.0;
    int arg = 0;
    for (int s = 0; s < SPC_N_SHAPES; ++s) {
        const double a = std::min(std::max((double)features[8 + s], sel->lo2[s]), sel->hi2[s]);
        double p = 0.0, pa = 1.0;
        for (int i = 0; i <= sel->deg2a[s]; ++i) {
            double pu = 1.0;
            for (int j = 0; j <= sel->deg2u[s]; ++j) {
                p += sel->coef2[s][i][j] * pa * pu;
                pu *= u;
            }
            pa *= a;
        }
        if (scores_out) scores_out[s] = (float)p;
        if (s == 0 || p > best) {
            best = p;
            arg = s;
        }
    }
    *shape_out = arg;
    return SPC_OK;
}

extern "C" spc_status spc_selector_interp_coeffs(const spc_selector *sel, double *coeffs_out, double *lo_out,
                                                 double *hi_out, int32_t *n_classes_out) {
    SPC_REQUIRE(sel && coeffs_out, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(sel->has_interp, SPC_ERR_NO_MODEL, "the selector has no interpolation fit");
    if (n_classes_out) *n_classes_out = sel->n_interp;
    for (int s = 0; s < sel->n_interp; ++s) {
        for (int j = 0; j <= kMaxDeg; ++j) coeffs_out[s * (kMaxDeg + 1) + j] = sel->coef[s][j];
        if (lo_out) lo_out[s] = sel->lo[s];
        if (hi_out) hi_out[s] = sel->hi[s];
    }
    return SPC_OK;
}

extern "C" spc_status spc_selector_set_mlp(spc_selector *sel, int32_t n_out, const float *params, const float *mu,
                                           const float *sd) {
    SPC_REQUIRE(sel && params && mu && sd, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(n_out == SPC_MLP_N_OUT || n_out == SPC_MLP_MAX_OUT, SPC_ERR_INVALID_ARG,
                "n_out must be %d or %d, got %d", SPC_MLP_N_OUT, SPC_MLP_MAX_OUT, n_out);
    for (int i = 0; i < SPC_MLP_N_IN; ++i)
        SPC_REQUIRE(std::isfinite(mu[i]) && std::isfinite(sd[i]) && sd[i] > 0.f, SPC_ERR_INVALID_ARG,
                    "standardizer entry %d is not finite or not positive", i);
    int dev = 0;
    SPC_HIP(hipGetDevice(&dev));
    if (sel->d_buf && sel->device != dev) {
        (void)hipFree(sel->d_buf);
        sel->d_buf = nullptr;
    }
    if (!sel->d_buf) {
        SPC_HIP(hipMalloc(&sel->d_buf, kBufFloats * sizeof(float)));
        sel->device = dev;
    }
    SPC_HIP(hipMemcpy(sel->d_buf + kParamsOff, params, SPC_MLP_PARAMS(n_out) * sizeof(float), hipMemcpyHostToDevice));
    SPC_HIP(hipMemcpy(sel->d_buf + kMuOff, mu, SPC_MLP_N_IN * sizeof(float), hipMemcpyHostToDevice));
    SPC_HIP(hipMemcpy(sel->d_buf + kSdOff, sd, SPC_MLP_N_IN * sizeof(float), hipMemcpyHostToDevice));
    sel->n_mlp = n_out;
    sel->has_mlp = true;
    return SPC_OK;
}

extern "C" spc_status spc_select_kernel(spc_selector *sel, const float *features, int32_t method,
                                        int32_t *class_out, float *scores_out, hipStream_t stream) {
    SPC_REQUIRE(sel && features && class_out, SPC_ERR_INVALID_ARG, "null argument");
    SPC_REQUIRE(method == SPC_SEL_INTERP || method == SPC_SEL_MLP, SPC_ERR_INVALID_ARG, "unknown method %d", method);
    if (method == SPC_SEL_INTERP) {
        SPC_REQUIRE(sel->has_interp, SPC_ERR_NO_MODEL, "the selector has no interpolation fit");
        double best = 0.0;
        int arg = 0;
        for (int s = 0; s < sel->n_interp; ++s) {
            const double a = std::min(std::max((double)features[8 + spc_class_shape(s)], sel->lo[s]), sel->hi[s]);
            double p = 0.0;
            for (int j = sel->deg[s]; j >= 0; --j) p = p * a + sel->coef[s][j];
            if (scores_out) scores_out[s] = (float)p;
            if (s == 0 || p > best) {
                best = p;
                arg = s;
            }
        }
        *class_out = arg;
        return SPC_OK;
    }
    SPC_REQUIRE(sel->has_mlp, SPC_ERR_NO_MODEL, "the selector has no trained network");
    int dev = 0;
    SPC_HIP(hipGetDevice(&dev));
    SPC_REQUIRE(dev == sel->device, SPC_ERR_INVALID_ARG, "the network was loaded on device %d, current is %d",
                sel->device, dev);
    float *b = sel->d_buf;
    SPC_HIP(hipMemcpyAsync(b + kFeatOff, features, SPC_MLP_N_IN * sizeof(float), hipMemcpyHostToDevice, stream));
    spc_status st = spc_mlp_infer(b + kParamsOff, b + kMuOff, b + kSdOff, b + kFeatOff, 1, sel->n_mlp,
                                  b + kScoreOff, reinterpret_cast<int32_t *>(b + kChoiceOff), stream);
    if (st != SPC_OK) return st;
    float host[8 + 4];
    SPC_HIP(hipMemcpyAsync(host, b + kScoreOff, sizeof(host), hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    if (scores_out)
        for (int s = 0; s < sel->n_mlp; ++s) scores_out[s] = host[s];
    *class_out = *reinterpret_cast<int32_t *>(&host[8]);
    return SPC_OK;
}
