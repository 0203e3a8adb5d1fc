// Status strings, error detail, small helpers of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace spc {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

spc_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
    const char *base = strrchr(file, '/');
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), base ? base + 1 : file, line);
    return SPC_ERR_HIP;
}

size_t lds_reserve_for(size_t static_lds, int cu_groups) {
    if (cu_groups <= 0) return 0;
    int dev = 0, per_cu = 0, per_group = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_group, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        per_cu <= 0 || per_group <= 0)
        return 0;
    // the smallest per-group LDS with floor(per_cu / lds) <= cu_groups
    size_t want = (size_t)per_cu / (size_t)(cu_groups + 1) + 1;
    if (want > (size_t)per_group) want = (size_t)per_group;
    return want > static_lds ? want - static_lds : 0;
}

spc_status check_view(const spc_beta_view *A) {
    SPC_REQUIRE(A != nullptr, SPC_ERR_INVALID_ARG, "null matrix view");
    SPC_REQUIRE(shape_of(A->r, A->c) >= 0, SPC_ERR_UNSUPPORTED_SHAPE,
                "block shape (%d,%d) is not one of the six supported shapes", A->r, A->c);
    SPC_REQUIRE(A->dtype == SPC_F32 || A->dtype == SPC_F64, SPC_ERR_INVALID_ARG, "bad dtype %d",
                A->dtype);
    SPC_REQUIRE(A->n_rows >= 0 && A->n_cols >= 0 && A->nnz >= 0 && A->n_blocks >= 0,
                SPC_ERR_INVALID_ARG, "negative size in view");
    SPC_REQUIRE(A->n_rows < (int64_t(1) << 31) && A->n_cols < (int64_t(1) << 31) &&
                    A->nnz < (int64_t(1) << 40) && A->n_blocks < (int64_t(1) << 31),
                SPC_ERR_OVERFLOW, "view sizes exceed the int32 index range");
    if (A->n_rows > 0) SPC_REQUIRE(A->block_rowptr, SPC_ERR_INVALID_ARG, "null block_rowptr");
    if (A->n_blocks > 0) {
        SPC_REQUIRE(A->block_colidx && A->block_masks, SPC_ERR_INVALID_ARG,
                    "null block_colidx or block_masks");
        SPC_REQUIRE((reinterpret_cast<uintptr_t>(A->block_masks) & 7u) == 0, SPC_ERR_INVALID_ARG,
                    "block_masks must be 8-byte aligned");
    }
    if (A->nnz > 0) {
        SPC_REQUIRE(A->values, SPC_ERR_INVALID_ARG, "null values");
        size_t es = A->dtype == SPC_F64 ? 8 : 4;
        SPC_REQUIRE((reinterpret_cast<uintptr_t>(A->values) % es) == 0, SPC_ERR_INVALID_ARG,
                    "values not aligned to the element size");
    }
    return SPC_OK;
}

}  // namespace spc

extern "C" {

const char *spc_status_string(spc_status s) {
    switch (s) {
    case SPC_OK: return "SPC_OK";
    case SPC_ERR_INVALID_ARG: return "SPC_ERR_INVALID_ARG";
    case SPC_ERR_UNSUPPORTED_SHAPE: return "SPC_ERR_UNSUPPORTED_SHAPE";
    case SPC_ERR_CSR_UNSORTED_OR_DUP: return "SPC_ERR_CSR_UNSORTED_OR_DUP";
    case SPC_ERR_INDEX_RANGE: return "SPC_ERR_INDEX_RANGE";
    case SPC_ERR_OVERFLOW: return "SPC_ERR_OVERFLOW";
    case SPC_ERR_HIP: return "SPC_ERR_HIP";
    case SPC_ERR_NO_MODEL: return "SPC_ERR_NO_MODEL";
    case SPC_ERR_CAPACITY: return "SPC_ERR_CAPACITY";
    default: return "SPC_ERR_UNKNOWN";
    }
}

const char *spc_last_error(void) { return spc::g_err; }

int32_t spc_version(void) { return 1 * 10000 + 0 * 100 + 0; }

spc_status spc_shape_index(int32_t r, int32_t c) {
    int s = spc::shape_of(r, c);
    return s < 0 ? SPC_ERR_UNSUPPORTED_SHAPE : s;
}

int64_t spc_mask_bytes(int32_t r, int32_t c, int64_t n_blocks) {
    if (spc::shape_of(r, c) < 0 || n_blocks < 0) return -1;
    int64_t b = n_blocks * (r * c / 8);
    return (b + 7) / 8 * 8 + 512;  // kernels read up to 64 mask words at a time
}

}  // extern "C"
