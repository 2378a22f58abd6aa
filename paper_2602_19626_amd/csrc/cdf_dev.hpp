// Device building blocks of the CDF-24 quantiser (paper section 3.4).
//
// Counts: c_i = max(1, floor(p_i * (T - V))) where the floor is exact (the 24-bit significand of
// p_i times the integer T - V in 64-bit integer arithmetic, never a rounded float product); the
// residual T - sum(c), which may be negative, goes to the lowest index among the maximal p_i;
// cdf[i + 1] = c_0 + ... + c_i.
//
// Work split: a row of V entries is cut into segments of kSeg = 4096 entries, one 256-thread
// workgroup per (row, segment).  A first pass reduces each segment to a SegPartial (sum of
// counts, argmax, validity); a second pass combines the row's partials in segment order (so the
// result never depends on scheduling), re-reads its segment, and scans it.  Inside a segment,
// thread t owns the four contiguous entries 4t..4t+3 of each of the four 1024-entry quarters,
// so every load and store instruction of a wave covers one contiguous 1 KiB span.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nc {

constexpr int kSegThreads = 256;
constexpr int kSegWaves = kSegThreads / 64;
constexpr int kQuarter = kSegThreads * 4;  // 1024 entries
constexpr int kSeg = kQuarter * 4;         // 4096 entries per segment
constexpr int kMaxSegs = 64;               // vocab <= 262,144

typedef float f4v __attribute__((ext_vector_type(4)));

// floor(p * m) of the exact real product, for finite p in [0, 1] and m < 2^24.
__device__ __forceinline__ uint32_t exact_floor_scaled(float p, uint32_t m) {
  const uint32_t bits = __float_as_uint(p);
  const uint32_t e = (bits >> 23) & 0xFFu;
  const uint64_t mant = (bits & 0x7FFFFFu) | 0x800000u;  // p = mant * 2^(e - 150)
  const int sh = 150 - int(e);
  // both factors are below 2^24 (the mask states it for m, which the callers' total <= 2^24
  // bounds), so the product is two full-rate 24-bit multiplies rather than a 64-bit one
  const uint32_t r = uint32_t((mant * uint64_t(m & 0xFFFFFFu)) >> (sh & 63));  // p <= 1: sh >= 23
  // zero or subnormal (p * m < 2^-126 * 2^24 < 1) and shifts of 64 or more give 0; selects
  // rather than branches, as this runs for every entry of a row
  return (e == 0 || sh >= 64) ? 0u : r;
}

__device__ __forceinline__ uint32_t floor_count(float p, uint32_t m) {
  const uint32_t c = exact_floor_scaled(p, m);
  return c < 1u ? 1u : c;
}

// (value, index) maximum with the lowest index winning ties.
__device__ __forceinline__ void argmax_merge(float& v, uint32_t& i, float v2, uint32_t i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
__device__ __forceinline__ void wave_argmax(float& v, uint32_t& i) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const float v2 = __shfl_xor(v, d, 64);
    const uint32_t i2 = __shfl_xor(i, d, 64);
    argmax_merge(v, i, v2, i2);
  }
}

// Per-(row, segment) reduction result.
struct SegPartial {
  uint32_t sum;   // sum of floor counts of the segment (saturated at 2^32 - 1)
  float maxv;     // largest probability of the segment
  uint32_t maxi;  // its lowest index (row-global)
  int32_t bad;    // 1 if a probability is NaN, negative or above one
};

// Whole-row quantities derived from the partials of one row, combined in segment order.
struct RowQuant {
  uint32_t argmax;
  int32_t residual;
  uint32_t m;      // T - V
  int status;      // 0 valid; 1 bad probability or mass above the total
  uint32_t start;  // cdf value at the first entry of this workgroup's segment
};

__device__ __forceinline__ uint32_t corrected_count(float x, uint32_t idx, const RowQuant& q) {
  const uint32_t cc = floor_count(x, q.m);
  return idx == q.argmax ? uint32_t(int32_t(cc) + q.residual) : cc;
}

// Element index of quarter j, sub-entry i of thread tid in segment seg.
__device__ __forceinline__ uint32_t seg_index(uint32_t seg, int j, int tid, int i) {
  return seg * kSeg + uint32_t(j) * kQuarter + 4u * uint32_t(tid) + uint32_t(i);
}

struct SegLds {
  uint64_t u64[kSegWaves];
  float f[kSegWaves];
  float f2[kSegWaves];
  uint32_t u32[kSegWaves];
  int flag[kSegWaves];
  uint32_t cols[kSegWaves * 4];
  SegPartial parts[kMaxSegs];
  uint32_t bcast[8];
};

// First pass: reduce one segment of probabilities p[j][i] (already zero at or beyond V); tid is
// the thread's index within its 256-thread segment group.
__device__ __forceinline__ SegPartial seg_reduce(const float (&p)[4][4], uint32_t seg, uint32_t V,
                                                 uint32_t m, SegLds& L, int tid) {
  const int lane = tid & 63, w = tid >> 6;
  int bad = 0;
  uint64_t sum = 0;
  float best = -1.f;
  uint32_t besti = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t idx = seg_index(seg, j, tid, i);
      const float x = p[j][i];
      if (idx < V) {
        if (!(x >= 0.f && x <= 1.f)) bad = 1;  // also catches NaN
        sum += floor_count(x, m);
        if (x > best) {  // increasing index order per thread: strict > keeps the first
          best = x;
          besti = idx;
        }
      }
    }
  sum = wave_sum_u64(sum);
  wave_argmax(best, besti);
  const int wbad = __any(bad) ? 1 : 0;
  if (lane == 0) {
    L.u64[w] = sum;
    L.f[w] = best;
    L.u32[w] = besti;
    L.flag[w] = wbad;
  }
  __syncthreads();
  SegPartial r;
  uint64_t tot = 0;
  r.maxv = -1.f;
  r.maxi = 0xFFFFFFFFu;
  r.bad = 0;
#pragma unroll
  for (int k = 0; k < kSegWaves; ++k) {
    tot += L.u64[k];
    argmax_merge(r.maxv, r.maxi, L.f[k], L.u32[k]);
    r.bad |= L.flag[k];
  }
  r.sum = tot >= 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(tot);
  return r;
}

// Second pass, row part: combine the row's partials (in LDS) in segment order into the residual,
// the argmax and this segment's starting CDF value.
// parts: kMaxSegs entries (in LDS), the first nseg of them the row's partials.
__device__ __forceinline__ RowQuant seg_combine(const SegPartial* parts, uint32_t nseg,
                                                uint32_t seg, uint32_t V, uint32_t total) {
  RowQuant q;
  q.m = total - V;
  uint64_t tot = 0, before = 0;
  float bv = -1.f;
  uint32_t bi = 0xFFFFFFFFu;
  int bad = 0;
  // partials read sixteen at a time (parts holds kMaxSegs entries, so every read is in range)
  // and combined in segment order
  for (uint32_t k0 = 0; k0 < nseg; k0 += 16) {
    SegPartial buf[16];
#pragma unroll
    for (uint32_t u = 0; u < 16; ++u) buf[u] = parts[k0 + u];
#pragma unroll
    for (uint32_t u = 0; u < 16; ++u) {
      const uint32_t k = k0 + u;
      if (k < nseg) {
        const SegPartial& s = buf[u];
        if (k < seg) before += s.sum;
        tot += s.sum;
        argmax_merge(bv, bi, s.maxv, s.maxi);
        bad |= s.bad;
      }
    }
  }
  const int64_t r = int64_t(total) - int64_t(tot);
  q.argmax = bi;
  q.residual = int32_t(r);
  q.status = bad | (tot >= 0xFFFFFFFFull ? 1 : 0) | (bi < V ? 0 : 1);
  if (!q.status && int64_t(floor_count(bv, q.m)) + r < 1) q.status = 1;
  if (bi < V && bi / kSeg < seg) before += uint64_t(int64_t(r));
  q.start = uint32_t(before);
  return q;
}

// Second pass, segment part: exclusive scan of the corrected counts of this segment.  On return
// base[j] = cdf[seg_index(seg, j, tid, 0)] and c[j][i] is the corrected count of entry (j, i)
// (0 at or beyond V), so cdf[idx + 1] = base[j] + c[j][0] + ... + c[j][i].
__device__ __forceinline__ void seg_scan(const float (&p)[4][4], uint32_t seg, uint32_t V,
                                         const RowQuant& q, uint32_t (&base)[4],
                                         uint32_t (&c)[4][4], SegLds& L, int tid) {
  const int lane = tid & 63, w = tid >> 6;
  uint32_t excl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t idx = seg_index(seg, j, tid, i);
      c[j][i] = idx < V ? corrected_count(p[j][i], idx, q) : 0u;
      s += c[j][i];
    }
    uint32_t v = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(v, d, 64);
      if (lane >= d) v += y;
    }
    if (lane == 63) L.cols[w * 4 + j] = v;
    excl[j] = v - s;
  }
  __syncthreads();
  uint32_t acc = q.start;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t off = 0, coltot = 0;
#pragma unroll
    for (int k = 0; k < kSegWaves; ++k) {
      const uint32_t s = L.cols[k * 4 + j];
      off += (k < w) ? s : 0u;
      coltot += s;
    }
    base[j] = acc + off + excl[j];
    acc += coltot;
  }
}

}  // namespace nc
