// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nc {

// CDF-24 quantise + scan, reduce-then-scan over 4096-entry segments (k_cdf.hip).  The workspace
// holds quantize_workspace_bytes(rows, V) bytes of device memory.
size_t quantize_workspace_bytes(uint32_t rows, uint32_t V);
// Bytes of workspace the launch for these rows actually uses (0 on the one-workgroup-per-row path).
size_t quantize_workspace_needed(const float* p, uint32_t rows, uint32_t V);
// The no-allocation variant's workspace: a fixed device array of kScratchParts segment partials
// (16 bytes each), its address on the current device resolved on first use.
constexpr size_t kScratchParts = 65536;
constexpr size_t kScratchBytes = kScratchParts * 16;
void* quantize_scratch_address();
void launch_quantize_cdf(const float* p, uint32_t rows, uint32_t V, uint32_t total, uint32_t* cdf,
                         int32_t* status, void* workspace, hipStream_t s);
void launch_cdf_interval(const uint32_t* cdf, uint32_t rows, uint32_t V, const uint32_t* key,
                         int mode, uint32_t* out, hipStream_t s);

}  // namespace nc
