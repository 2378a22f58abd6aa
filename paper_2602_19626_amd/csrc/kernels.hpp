// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nc {

// CDF-24 quantise + scan, reduce-then-scan over 4096-entry segments (k_cdf.hip).  The workspace
// holds quantize_workspace_bytes(rows, V) bytes of device memory.
size_t quantize_workspace_bytes(uint32_t rows, uint32_t V);
void launch_quantize_cdf(const float* p, uint32_t rows, uint32_t V, uint32_t total, uint32_t* cdf,
                         int32_t* status, void* workspace, hipStream_t s);
void launch_cdf_interval(const uint32_t* cdf, uint32_t rows, uint32_t V, const uint32_t* key,
                         int mode, uint32_t* out, hipStream_t s);

}  // namespace nc
