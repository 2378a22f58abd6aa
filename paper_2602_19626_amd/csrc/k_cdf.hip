// CDF-24 quantise + scan over batches of probability rows (paper section 3.4) and the interval
// lookup used by the arithmetic coder (section 3.9).
#include <mutex>
#include <unordered_map>

#include "cdf_dev.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace nc {

// kLast: the final read of the row (streamed past the caches); the first pass keeps the row
// cached, where the second pass finds it.
template <bool kVec4, bool kLast>
__device__ __forceinline__ void load_seg(const float* __restrict__ p, uint32_t seg, uint32_t V,
                                         float (&v)[4][4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t idx = seg_index(seg, j, tid, 0);
    if (kVec4 && idx + 3 < V) {
      const f4v q = kLast ? __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p + idx))
                          : *reinterpret_cast<const f4v*>(p + idx);
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
  load_seg<kVec4, false>(probs + size_t(row) * V, seg, V, v);
  const SegPartial r = seg_reduce(v, seg, V, total - V, L, threadIdx.x);
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
  load_seg<kVec4, true>(probs + size_t(row) * V, seg, V, v);
  __syncthreads();
  const RowQuant q = seg_combine(L.parts, nseg, seg, V, total);
  uint32_t base[4], cnt[4][4];
  seg_scan(v, seg, V, q, base, cnt, L, tid);
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
        run += cnt[j][i];
        __builtin_nontemporal_store(run, out + idx + 1);
      }
    }
  }
}

// One workgroup per row for V <= 49,152, several rows resident per CU.  512 threads; thread t owns
// the four entries 2048 q + 4 t .. + 3 of each 2048-entry block q < 24.  Pass 1 reads the row and
// reduces the floor counts (each thread's four-entry sums are kept in LDS), the lowest-index
// argmax and the validity; one barrier round turns the sums into the CDF value before every
// thread's first entry of every block (a wave scan per block, block and wave offsets by a
// two-level scan of the wave totals).  Pass 2 reads the row again (a row read moments before, so
// it comes from the caches), recomputes each entry's count and writes the CDF with the widest
// stores the row's alignment allows.  The kernel holds no row in registers: its 48 KiB of LDS and
// few registers let three rows overlap on a CU, so one row's loads, another's scan and a third's
// stores keep the memory busy.  Every result is an integer or a comparison, so it equals the
// two-kernel result.
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
constexpr int kRowThreads = 512;
constexpr int kRowWaves = kRowThreads / 64;
constexpr int kRowBlock = kRowThreads * 4;  // 2048 entries
constexpr int kRowBlocks = 24;
constexpr int kRowBatch = 8;                // loads in flight per thread
constexpr uint32_t kRowMaxV = kRowBlocks * kRowBlock;
constexpr uint32_t kSegPathMaxRows = 64;

__global__ __launch_bounds__(kRowThreads, 6) void cdf24_row_kernel(const float* __restrict__ probs,
                                                                   uint32_t V, uint32_t total,
                                                                   uint32_t* __restrict__ cdf,
                                                                   int32_t* __restrict__ status) {
  __shared__ uint64_t s_sum[kRowWaves];
  __shared__ float s_best[kRowWaves];
  __shared__ uint32_t s_bi[kRowWaves];
  __shared__ int s_bad[kRowWaves];
  __shared__ uint32_t s_wt[kRowWaves][kRowBlocks];
  __shared__ uint32_t s_bt[kRowBlocks];
  __shared__ uint32_t s_off[kRowWaves][kRowBlocks];
  // per (block, thread): the four-entry count sum, then its exclusive prefix within the wave
  __shared__ uint32_t s_cnt[kRowBlocks][kRowThreads];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t row = blockIdx.x;
  const float* p = probs + size_t(row) * V;
  const f4v* p4 = reinterpret_cast<const f4v*>(p) + tid;
  const uint32_t m = total - V;
  // pass 1 (V % 4 == 0: a group of four is either whole or past the end)
  uint64_t sum = 0;
  float best = -1.f;
  uint32_t bi = 0xFFFFFFFFu;
  int bad = 0;
#pragma unroll 1
  for (int q0 = 0; q0 < kRowBlocks; q0 += kRowBatch) {
    f4v x[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int q = q0 + u;
      x[u] = q * kRowBlock + 4 * tid < V ? p4[q * kRowThreads] : f4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int q = q0 + u;
      const uint32_t i0 = q * kRowBlock + 4 * tid;
      uint32_t c4 = 0;
      if (i0 < V) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (!(x[u][i] >= 0.f && x[u][i] <= 1.f)) bad = 1;
          c4 += floor_count(x[u][i], m);
          if (x[u][i] > best) {
            best = x[u][i];
            bi = i0 + i;
          }
        }
      }
      s_cnt[q][tid] = c4;
      sum += c4;
    }
  }
  sum = wave_sum_u64(sum);
  wave_argmax(best, bi);
  bad = __any(bad) ? 1 : 0;
  if (lane == 0) {
    s_sum[w] = sum;
    s_best[w] = best;
    s_bi[w] = bi;
    s_bad[w] = bad;
  }
  __syncthreads();
  RowQuant rq;
  {
    uint64_t tot = 0;
    float bv = -1.f;
    uint32_t b = 0xFFFFFFFFu;
    int bd = 0;
    for (int k = 0; k < kRowWaves; ++k) {
      tot += s_sum[k];
      argmax_merge(bv, b, s_best[k], s_bi[k]);
      bd |= s_bad[k];
    }
    const int64_t r = int64_t(total) - int64_t(tot);
    rq.m = m;
    rq.argmax = b;
    rq.residual = int32_t(r);
    rq.status = bd | (tot >= 0xFFFFFFFFull ? 1 : 0) | (b < V ? 0 : 1);
    if (!rq.status && int64_t(floor_count(bv, m)) + r < 1) rq.status = 1;
    rq.start = 0;
  }
  // the residual belongs to the argmax entry (corrected_count); per-block wave scans
#pragma unroll
  for (int q = 0; q < kRowBlocks; ++q) {
    const uint32_t i0 = q * kRowBlock + 4 * tid;
    uint32_t c4 = s_cnt[q][tid];
    if (rq.argmax >= i0 && rq.argmax < i0 + 4) c4 = uint32_t(int32_t(c4) + rq.residual);
    uint32_t incl = c4;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) s_wt[w][q] = incl;
    s_cnt[q][tid] = incl - c4;
  }
  __syncthreads();
  // block totals, then the CDF value before wave k's part of block q: the earlier blocks' totals
  // plus the earlier waves of block q
  if (tid < kRowBlocks) {
    uint32_t t = 0;
    for (int k = 0; k < kRowWaves; ++k) t += s_wt[k][tid];
    s_bt[tid] = t;
  }
  __syncthreads();
  if (tid < kRowWaves * kRowBlocks) {
    const int k = tid / kRowBlocks, q = tid % kRowBlocks;
    uint32_t o = 0;
    for (int qq = 0; qq < q; ++qq) o += s_bt[qq];
    for (int kk = 0; kk < k; ++kk) o += s_wt[kk][q];
    s_off[k][q] = o;
  }
  __syncthreads();
  uint32_t* out = cdf + size_t(row) * (size_t(V) + 1);
  if (tid == 0) {
    out[0] = 0;
    if (status) status[row] = rq.status;
  }
  // pass 2: entries 2048 q + 4 t + i go to out[1 + 2048 q + 4 t + i]; every such group of four
  // starts at the same word phase within the row
  const uint32_t phase = uint32_t((reinterpret_cast<uintptr_t>(out + 1) >> 2) & 3);
#pragma unroll 1
  for (int q0 = 0; q0 < kRowBlocks; q0 += kRowBatch) {
    f4v x[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int q = q0 + u;
      x[u] = q * kRowBlock + 4 * tid < V ? __builtin_nontemporal_load(p4 + q * kRowThreads)
                                         : f4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int q = q0 + u;
      const uint32_t i0 = q * kRowBlock + 4 * tid;
      if (i0 >= V) continue;
      uint32_t r4[4], run = s_off[w][q] + s_cnt[q][tid];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        run += corrected_count(x[u][i], i0 + i, rq);
        r4[i] = run;
      }
      uint32_t* dst = out + 1 + i0;
      if (phase == 0) {
        __builtin_nontemporal_store(u4v{r4[0], r4[1], r4[2], r4[3]}, reinterpret_cast<u4v*>(dst));
      } else if (phase == 2) {
        __builtin_nontemporal_store(u2v{r4[0], r4[1]}, reinterpret_cast<u2v*>(dst));
        __builtin_nontemporal_store(u2v{r4[2], r4[3]}, reinterpret_cast<u2v*>(dst + 2));
      } else if (phase == 3) {
        dst[0] = r4[0];
        __builtin_nontemporal_store(u2v{r4[1], r4[2]}, reinterpret_cast<u2v*>(dst + 1));
        dst[3] = r4[3];
      } else {
        dst[0] = r4[0];
        dst[1] = r4[1];
        __builtin_nontemporal_store(u2v{r4[2], r4[3]}, reinterpret_cast<u2v*>(dst + 2));
      }
    }
  }
}

size_t quantize_workspace_bytes(uint32_t rows, uint32_t V) {
  return size_t(rows) * ceil_div(V, kSeg) * sizeof(SegPartial);
}

// The row kernel places one workgroup per row, so a few rows leave most CUs idle; up to
// kSegPathMaxRows rows the segment kernels (ceil(V / 4096) workgroups per row) finish sooner.
// Both give the same integers.
static bool vec_rows(const float* p, uint32_t V) {
  return (V % 4 == 0) && (reinterpret_cast<uintptr_t>(p) % 16 == 0);
}
static bool use_row_kernel(const float* p, uint32_t rows, uint32_t V) {
  return vec_rows(p, V) && V <= kRowMaxV && rows > kSegPathMaxRows;
}

size_t quantize_workspace_needed(const float* p, uint32_t rows, uint32_t V) {
  return use_row_kernel(p, rows, V) ? 0 : quantize_workspace_bytes(rows, V);
}

void launch_quantize_cdf(const float* p, uint32_t rows, uint32_t V, uint32_t total, uint32_t* cdf,
                         int32_t* status, void* workspace, hipStream_t s) {
  if (rows == 0) return;
  const bool vec = vec_rows(p, V);
  if (use_row_kernel(p, rows, V)) {
    hipLaunchKernelGGL(cdf24_row_kernel, dim3(rows), dim3(kRowThreads), 0, s, p, V, total, cdf,
                       status);
    NC_HIP(hipGetLastError());
    return;
  }
  const uint32_t nseg = uint32_t(ceil_div(V, kSeg));
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

// Scratch of the no-allocation variant: the segment partials of up to kScratchParts segments
// (1 MiB), one copy per device for the life of the process.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol); it passes the device
// address that hipGetSymbolAddress resolves once per device.
static_assert(sizeof(SegPartial) * kScratchParts == kScratchBytes, "scratch size");
static __device__ __align__(256) SegPartial scratch[kScratchParts];

void* quantize_scratch_address() {
  static std::mutex mu;
  static std::unordered_map<int, void*> addr;
  int dev = 0;
  NC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  NC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  NC_CHECK(ptr != nullptr, NC_E_DEVICE, "no device address for the CDF-24 scratch array");
  addr[dev] = ptr;
  return ptr;
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
