// CDF-24 quantise + scan over batches of probability rows (paper section 3.4) and the interval
// lookup used by the arithmetic coder (section 3.9).
#include "cdf_dev.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace nc {

template <bool kVec4>
__device__ __forceinline__ void load_seg(const float* __restrict__ p, uint32_t seg, uint32_t V,
                                         float (&v)[4][4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t idx = seg_index(seg, j, tid, 0);
    if (kVec4 && idx + 3 < V) {
      const f4v q = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p + idx));
#pragma unroll
      for (int i = 0; i < 4; ++i) v[j][i] = q[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[j][i] = (idx + i < V) ? p[idx + i] : 0.f;
    }
  }
}

// Pass 1: one workgroup per (segment, row) writes the segment's SegPartial.
template <bool kVec4>
__global__ __launch_bounds__(kSegThreads) void cdf24_reduce_kernel(
    const float* __restrict__ probs, uint32_t V, uint32_t total, uint32_t nseg,
    SegPartial* __restrict__ parts) {
  __shared__ SegLds L;
  const uint32_t seg = blockIdx.x, row = blockIdx.y;
  float v[4][4];
  load_seg<kVec4>(probs + size_t(row) * V, seg, V, v);
  const SegPartial r = seg_reduce(v, seg, V, total - V, L);
  if (threadIdx.x == 0) parts[size_t(row) * nseg + seg] = r;
}

// Pass 2: combine the row's partials in order, re-read the segment, scan it and write the CDF.
template <bool kVec4>
__global__ __launch_bounds__(kSegThreads) void cdf24_scan_kernel(
    const float* __restrict__ probs, uint32_t V, uint32_t total, uint32_t nseg,
    const SegPartial* __restrict__ parts, uint32_t* __restrict__ cdf,
    int32_t* __restrict__ status) {
  __shared__ SegLds L;
  const uint32_t seg = blockIdx.x, row = blockIdx.y;
  const int tid = threadIdx.x;
  if (tid < int(nseg)) L.parts[tid] = parts[size_t(row) * nseg + tid];
  float v[4][4];
  load_seg<kVec4>(probs + size_t(row) * V, seg, V, v);
  __syncthreads();
  const RowQuant q = seg_combine(L.parts, nseg, seg, V, total);
  uint32_t base[4];
  seg_scan(v, seg, V, q, base, L);
  uint32_t* out = cdf + size_t(row) * (size_t(V) + 1);
  if (seg == 0 && tid == 0) {
    out[0] = 0;
    if (status) status[row] = q.status;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t run = base[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t idx = seg_index(seg, j, tid, i);
      if (idx < V) {
        run += corrected_count(v[j][i], idx, q);
        __builtin_nontemporal_store(run, out + idx + 1);
      }
    }
  }
}

size_t quantize_workspace_bytes(uint32_t rows, uint32_t V) {
  return size_t(rows) * ceil_div(V, kSeg) * sizeof(SegPartial);
}

void launch_quantize_cdf(const float* p, uint32_t rows, uint32_t V, uint32_t total, uint32_t* cdf,
                         int32_t* status, void* workspace, hipStream_t s) {
  if (rows == 0) return;
  const uint32_t nseg = uint32_t(ceil_div(V, kSeg));
  const bool vec = (V % 4 == 0) && (reinterpret_cast<uintptr_t>(p) % 16 == 0);
  SegPartial* parts = static_cast<SegPartial*>(workspace);
  const dim3 grid(nseg, rows);
  if (vec) {
    hipLaunchKernelGGL(cdf24_reduce_kernel<true>, grid, dim3(kSegThreads), 0, s, p, V, total, nseg,
                       parts);
    hipLaunchKernelGGL(cdf24_scan_kernel<true>, grid, dim3(kSegThreads), 0, s, p, V, total, nseg,
                       parts, cdf, status);
  } else {
    hipLaunchKernelGGL(cdf24_reduce_kernel<false>, grid, dim3(kSegThreads), 0, s, p, V, total,
                       nseg, parts);
    hipLaunchKernelGGL(cdf24_scan_kernel<false>, grid, dim3(kSegThreads), 0, s, p, V, total, nseg,
                       parts, cdf, status);
  }
  NC_HIP(hipGetLastError());
}

// mode 0: out = (s, cdf[s], cdf[s+1]) for s = key; mode 1: largest s with cdf[s] <= key.
__global__ void cdf_interval_kernel(const uint32_t* __restrict__ cdf, uint32_t rows, uint32_t V,
                                    const uint32_t* __restrict__ key, int mode,
                                    uint32_t* __restrict__ out) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const uint32_t* c = cdf + size_t(r) * (size_t(V) + 1);
  uint32_t s = key[r];
  if (mode == 0) {
    s = s < V ? s : V - 1;
  } else {
    uint32_t lo = 0, hi = V - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (c[mid] <= key[r])
        lo = mid;
      else
        hi = mid - 1;
    }
    s = lo;
  }
  out[3 * r + 0] = s;
  out[3 * r + 1] = c[s];
  out[3 * r + 2] = c[s + 1];
}

void launch_cdf_interval(const uint32_t* cdf, uint32_t rows, uint32_t V, const uint32_t* key,
                         int mode, uint32_t* out, hipStream_t s) {
  if (rows == 0) return;
  hipLaunchKernelGGL(cdf_interval_kernel, dim3(ceil_div(rows, 256)), dim3(256), 0, s, cdf, rows,
                     V, key, mode, out);
  NC_HIP(hipGetLastError());
}

}  // namespace nc
