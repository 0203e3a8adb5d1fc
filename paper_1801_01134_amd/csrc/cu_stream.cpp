// Streams restricted to a share of the compute units: the GPU counterpart of
// running the kernels on fewer threads, which section "Parallel performance
// estimation" makes the second input of its performance regression.
#include <vector>

#include "common.hpp"

extern "C" spc_status spc_stream_create_cu(int32_t n_cus, hipStream_t *stream_out) {
    SPC_REQUIRE(stream_out != nullptr, SPC_ERR_INVALID_ARG, "null stream_out");
    int dev = 0, total = 0;
    SPC_HIP(hipGetDevice(&dev));
    SPC_HIP(hipDeviceGetAttribute(&total, hipDeviceAttributeMultiprocessorCount, dev));
    SPC_REQUIRE(n_cus >= 1 && n_cus <= total, SPC_ERR_INVALID_ARG, "n_cus must be in 1..%d (got %d)", total, n_cus);
    std::vector<uint32_t> mask((size_t)(total + 31) / 32, 0u);
    if (total == 256) {
        // 8 XCDs of 32 units. The share must stay even over the XCDs whether
        // the runtime reads the mask as 32-bit words per XCD or deals its
        // bits out to the XCDs in turn (bit i to XCD i mod 8), so every
        // 32-bit word gets n/8 bits and every residue mod 8 gets n/8 bits:
        // word b takes residues (b m + j) mod 8 (j < m) for m = n/8 < 8, or
        // m/8 whole runs of 8 consecutive bits for m >= 8.
        SPC_REQUIRE(n_cus % 8 == 0, SPC_ERR_INVALID_ARG,
                    "n_cus must be a multiple of 8 (one share per XCD), got %d", n_cus);
        const int m = n_cus / 8;
        for (int b = 0; b < 8; ++b) {
            for (int j = 0; j < m; ++j) {
                const int q = m < 8 ? 8 * j + (b * m + j) % 8 : j;
                mask[(size_t)b] |= 1u << q;
            }
        }
    } else {
        // every (total / n_cus)-th unit
        for (int k = 0; k < n_cus; ++k) {
            const int bit = (int)((int64_t)k * total / n_cus);
            mask[(size_t)bit / 32] |= 1u << (bit % 32);
        }
    }
    SPC_HIP(hipExtStreamCreateWithCUMask(stream_out, (uint32_t)mask.size(), mask.data()));
    return SPC_OK;
}

extern "C" spc_status spc_stream_destroy(hipStream_t stream) {
    SPC_REQUIRE(stream != nullptr, SPC_ERR_INVALID_ARG, "null stream");
    SPC_HIP(hipStreamDestroy(stream));
    return SPC_OK;
}

extern "C" int32_t spc_device_cu_count(void) {
    int dev = 0, total = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&total, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return SPC_ERR_HIP;
    return total;
}
