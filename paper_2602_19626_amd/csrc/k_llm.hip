// Transformer kernels of the 135M-shape decoder (paper section 3.2 Eq. (lm), section 3.10):
// MFMA GEMMs with a fused RMSNorm prologue and fused epilogues (RoPE + KV-ring write, residual
// add, SiLU-gated MLP, logits), GQA attention over the sliding window, embedding gather and
// precision conversion.
//
// Batch invariance.  Every output element of a GEMM is the sum over K in chunks of 32 taken in
// increasing order, each chunk by the same MFMA instruction (f32 16x16x4, bf16 16x16x32, fp8
// 16x16x32), whatever the tile shape or the number of rows M.  Attention splits the keys into
// 64-key chunks at fixed absolute positions and combines the chunk partials with one fixed
// two-level fold.  A token's logits are therefore bitwise the same whether it is evaluated in a
// 32,768-row prefill or in a one-row decode step, which the coder relies on.
#include "cdf_dev.hpp"
#include "common.hpp"
#include "llm_dev.hpp"

#include <algorithm>
#include <type_traits>

// Prefill and decode must round every shared expression identically: no contraction.
#pragma clang fp contract(off)

namespace nc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

// ---- number formats ------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// float -> OCP fp8 e4m3 (bias 7, max 448, no infinity), round to nearest even, saturating.
__device__ __forceinline__ uint8_t f2fp8(float f) {
  const uint32_t b = __float_as_uint(f);
  const uint32_t sign = (b >> 24) & 0x80u;
  const uint32_t u = b & 0x7FFFFFFFu;
  uint32_t r;
  if (u >= 0x43E00000u) {           // |f| >= 448
    r = 0x7Eu;
  } else if (u < 0x3C800000u) {     // |f| < 2^-6: subnormal grid of 2^-9
    r = uint32_t(rintf(__uint_as_float(u) * 512.0f));
  } else {
    const uint32_t ue = u - (120u << 23);  // rebias 127 -> 7
    r = (ue + 0x7FFFFu + ((ue >> 20) & 1u)) >> 20;
    if (r > 0x7Eu) r = 0x7Eu;
  }
  return uint8_t(r | sign);
}

template <int P>
struct PT;
template <>
struct PT<P_F32> {
  static constexpr int ES = 4;
  __device__ static void put4(uint8_t* dst, const float (&v)[4], float) {
    *reinterpret_cast<v4f*>(dst) = v4f{v[0], v[1], v[2], v[3]};
  }
  __device__ static void store(void* base, long long i, float v, float) {
    static_cast<float*>(base)[i] = v;
  }
  __device__ static float load(const void* base, long long i) {
    return static_cast<const float*>(base)[i];
  }
};
template <>
struct PT<P_BF16> {
  static constexpr int ES = 2;
  __device__ static void put4(uint8_t* dst, const float (&v)[4], float) {
    uint2 w;
    w.x = uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16);
    w.y = uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16);
    *reinterpret_cast<uint2*>(dst) = w;
  }
  __device__ static void store(void* base, long long i, float v, float) {
    static_cast<uint16_t*>(base)[i] = f2bf(v);
  }
  __device__ static float load(const void* base, long long i) {
    return bf2f(static_cast<const uint16_t*>(base)[i]);
  }
};
template <>
struct PT<P_FP8> {
  static constexpr int ES = 1;
  __device__ static void put4(uint8_t* dst, const float (&v)[4], float inv_scale) {
    *reinterpret_cast<uint32_t*>(dst) =
        uint32_t(f2fp8(v[0] * inv_scale)) | (uint32_t(f2fp8(v[1] * inv_scale)) << 8) |
        (uint32_t(f2fp8(v[2] * inv_scale)) << 16) | (uint32_t(f2fp8(v[3] * inv_scale)) << 24);
  }
  __device__ static void store(void* base, long long i, float v, float inv_scale) {
    static_cast<uint8_t*>(base)[i] = f2fp8(v * inv_scale);
  }
};

__device__ __forceinline__ void atomic_max_abs(float* p, float v) {
  // |v| >= 0, so the IEEE bit pattern orders like an unsigned integer: integer atomic max
  atomicMax(reinterpret_cast<unsigned int*>(p), __float_as_uint(fabsf(v)));
}

// ---- GEMM -----------------------------------------------------------------------------------
//
// Arithmetic of every output element (the same in every kernel and tile shape):
//   out = ((0 + P_0) + P_1) + ... + P_{S-1},  S = ceil(K / 64),
//   P_s = the chain of MFMAs over the 64 K entries of part s, starting from zero, where
//     f32 16x16x4:            16 steps, step t / lane group g consumes k = 16 g + t,
//     bf16 / fp8 16x16x32:     2 steps, step t / lane group g consumes k = 32 t + 8 g .. + 7,
//   with entries beyond K read as zero.
// A normed GEMM (A_NORM) then multiplies by deq (FP8) and by the row's RMSNorm scale, in that
// order.  The tile kernels (many rows) sum the parts as they walk K; the split kernel (few rows)
// computes each part in its own wave and the workgroup adds the parts in order.  All apply the
// same epilogue functions, so a row's outputs do not depend on how many rows are in the launch.

constexpr int KP = 64;

// RMSNorm scale of a row, 1 / sqrt(mean(x^2) + eps), from block sums of squares.  Whatever writes
// a residual row x (embedding, residual epilogues) also writes, for each 16-column block b,
// ssq[b] = sum of x^2 over the block by one fixed tree (block_ssq16); the scale adds the block
// sums in block order.  Prefill and decode kernels therefore derive bitwise equal scales.

// Block sum of squares of 16 values held by 16 consecutive lanes (lane % 16 = column); every lane
// of the group returns the same bits.
__device__ __forceinline__ float block_ssq16(float x) {
  float v = x * x;
  v += __shfl_xor(v, 8, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

__device__ __forceinline__ float inv_from_ssq(const float* ssq, int K, float eps) {
  const int nb = K / 16;
  float t = 0.f;
  for (int b = 0; b < nb; ++b) t += ssq[b];
  return 1.0f / sqrtf(t / float(K) + eps);
}

// the scale of A row ar of a normed GEMM
__device__ __forceinline__ float a_row_inv(const GemmArgs& a, int ar) {
  return a.inv ? a.inv[ar] : inv_from_ssq(a.ssq + (long long)ar * (a.K / 16), a.K, a.eps);
}

// ---- epilogue emitters ----

// RoPE table entry (cos, sin) used by column n of a q/k head at position pos
__device__ __forceinline__ float2 rope_cs(const GemmArgs& a, int pos, int n) {
  const int h2 = a.hd / 2, within = n % a.hd;
  const int i = within < h2 ? within : within - h2;
  return *reinterpret_cast<const float2*>(a.rope + ((long long)pos * h2 + i) * 2);
}

// q/k/v output (m, n) = v (partner: the RoPE partner column's value) with the row's metadata rm
// and, for q/k columns, its RoPE entry cs = rope_cs(a, rm.pos, n)
__device__ __forceinline__ void emit_qkv_core(const GemmArgs& a, int prec_att, int m, int n,
                                              float v, float partner, const RowMeta& rm,
                                              float2 cs) {
  const int hd = a.hd, h2 = hd / 2;
  const int nq = a.Hq * hd, nk = a.Hk * hd;
  const int within = n % hd;
  if (n < nq + nk)  // rotate-half RoPE on q and k
    v = within < h2 ? v * cs.x - partner * cs.y : v * cs.x + partner * cs.y;
  long long idx;
  void* base;
  if (n < nq) {
    idx = (long long)m * nq + n;
    base = a.q_out;
  } else {
    const int kv = n < nq + nk ? n - nq : n - nq - nk;
    const int kvh = kv / hd;
    const long long slot = rm.slot;
    const long long sb = (long long)rm.stream * a.kv_stride + (long long)kvh * a.ring * hd;
    if (n < nq + nk) {
      idx = sb + slot * hd + within;
      base = a.k_cache;
    } else {
      idx = sb + (long long)within * a.ring + slot;
      base = a.vt_cache;
    }
  }
  if (prec_att == P_F32)
    PT<P_F32>::store(base, idx, v, 1.f);
  else
    PT<P_BF16>::store(base, idx, v, 1.f);
}

__device__ __forceinline__ void emit_qkv_prec(const GemmArgs& a, int prec_att, int m, int n,
                                              float v, float partner) {
  const RowMeta rm = a.rows[m];
  const float2 cs = n < (a.Hq + a.Hk) * a.hd ? rope_cs(a, rm.pos, n) : float2{1.f, 0.f};
  emit_qkv_core(a, prec_att, m, n, v, partner, rm, cs);
}

// emit_qkv_prec for rows m .. m + 3 of one column (BF16 attention operands), element for element
// the same arithmetic, with the rows' metadata rm and RoPE table rows rr (cos, sin pairs of
// position rm[e].pos, in global memory or LDS) supplied by the caller; V^T gets one 8-byte store
// when the rows are 4 consecutive ring slots of one stream.
__device__ __forceinline__ void emit_qkv4_rows(const GemmArgs& a, int n, const RowMeta (&rm)[4],
                                               const bool (&ok)[4], const float* const (&rr)[4],
                                               const float (&v)[4], const float (&partner)[4],
                                               int m) {
  const int hd = a.hd, h2 = hd / 2;
  const int nq = a.Hq * hd, nk = a.Hk * hd;
  const int within = n % hd;
  uint16_t h[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float x = v[e];
    if (n < nq + nk && ok[e]) {
      const int i = within < h2 ? within : within - h2;
      const float cs = rr[e][i * 2 + 0];
      const float sn = rr[e][i * 2 + 1];
      x = within < h2 ? x * cs - partner[e] * sn : x * cs + partner[e] * sn;
    }
    h[e] = f2bf(x);
  }
  if (n < nq) {
    uint16_t* Q = static_cast<uint16_t*>(a.q_out);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (ok[e]) Q[(long long)(m + e) * nq + n] = h[e];
    return;
  }
  const int kv = n < nq + nk ? n - nq : n - nq - nk;
  const int kvh = kv / hd;
  if (n < nq + nk) {
    uint16_t* Kc = static_cast<uint16_t*>(a.k_cache);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (ok[e]) {
        const long long sb = (long long)rm[e].stream * a.kv_stride + (long long)kvh * a.ring * hd;
        Kc[sb + (long long)rm[e].slot * hd + within] = h[e];
      }
    return;
  }
  uint16_t* Vt = static_cast<uint16_t*>(a.vt_cache);
  const int slot0 = rm[0].slot;
  bool run = ok[3] && (slot0 & 3) == 0 && slot0 + 3 < a.ring;
#pragma unroll
  for (int e = 1; e < 4; ++e)
    run = run && rm[e].stream == rm[0].stream && rm[e].pos == rm[0].pos + e;
  if (run) {
    const long long sb = (long long)rm[0].stream * a.kv_stride + (long long)kvh * a.ring * hd;
    uint2 w;
    w.x = uint32_t(h[0]) | (uint32_t(h[1]) << 16);
    w.y = uint32_t(h[2]) | (uint32_t(h[3]) << 16);
    *reinterpret_cast<uint2*>(Vt + sb + (long long)within * a.ring + slot0) = w;
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (ok[e]) {
      const long long sb = (long long)rm[e].stream * a.kv_stride + (long long)kvh * a.ring * hd;
      Vt[sb + (long long)within * a.ring + rm[e].slot] = h[e];
    }
}

template <int P>
__device__ __forceinline__ float emit_glu(const GemmArgs& a, int m, int col, float g, float u) {
  const float h = g / (1.0f + expf(-g)) * u;
  const float oinv = (P == P_FP8) ? 1.0f / a.out_scale : 1.0f;
  PT<P>::store(a.out_p, (long long)m * (a.N / 2) + col, h, oinv);
  return fabsf(h);
}

// Column of the partner of q/k column n for RoPE (the same head, the other half).
__device__ __forceinline__ int rope_partner(const GemmArgs& a, int n) {
  const int h2 = a.hd / 2;
  return (n % a.hd) < h2 ? n + h2 : n - h2;
}

// ---- operand fragments (from LDS or global, row-major with K contiguous) ----

template <int P>
struct Frag;
template <>
struct Frag<P_F32> {
  typedef float T[16];  // 16 steps of one float
  __device__ static void load(T& f, const uint8_t* row, int g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const v4f v = *reinterpret_cast<const v4f*>(row + (16 * g + 4 * q) * 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) f[4 * q + e] = v[e];
    }
  }
  __device__ static void zero(T& f) {
#pragma unroll
    for (int t = 0; t < 16; ++t) f[t] = 0.f;
  }
  // straight from a global row (entries k0 + 16 g + 0..15, zero at or beyond K)
  __device__ static void load_raw(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 16 * g + 4 * q;
      const v4f v = k < K ? *reinterpret_cast<const v4f*>(row + (long long)k * 4)
                          : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) f[4 * q + e] = v[e];
    }
  }
  // as load_raw, but the load itself is unconditional (its offset clamped into the row), so that
  // no branch separates it from the loads issued around it
  __device__ static void load_clamped(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 16 * g + 4 * q;
      const v4f v = *reinterpret_cast<const v4f*>(row + (long long)min(k, K - 4) * 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) f[4 * q + e] = k < K ? v[e] : 0.f;
    }
  }
  __device__ static void mma(v4f& acc, const T& a, const T& b) {
#pragma unroll
    for (int t = 0; t < 16; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[t], acc, 0, 0, 0);
  }
};
template <>
struct Frag<P_BF16> {
  typedef v4i T[2];
  __device__ static void load(T& f, const uint8_t* row, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) f[t] = *reinterpret_cast<const v4i*>(row + (32 * t + 8 * g) * 2);
  }
  __device__ static void zero(T& f) { f[0] = f[1] = v4i{0, 0, 0, 0}; }
  __device__ static void load_raw(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = k0 + 32 * t + 8 * g;
      f[t] = k < K ? *reinterpret_cast<const v4i*>(row + (long long)k * 2) : v4i{0, 0, 0, 0};
    }
  }
  __device__ static void load_clamped(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = k0 + 32 * t + 8 * g;
      const v4i v = *reinterpret_cast<const v4i*>(row + (long long)min(k, K - 8) * 2);
      f[t] = k < K ? v : v4i{0, 0, 0, 0};
    }
  }
  __device__ static void mma(v4f& acc, const T& a, const T& b) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[t]),
                                                    __builtin_bit_cast(v8bf, b[t]), acc, 0, 0, 0);
  }
};
template <>
struct Frag<P_FP8> {
  typedef long T[2];
  __device__ static void load(T& f, const uint8_t* row, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) f[t] = *reinterpret_cast<const long*>(row + 32 * t + 8 * g);
  }
  __device__ static void zero(T& f) { f[0] = f[1] = 0; }
  __device__ static void load_raw(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = k0 + 32 * t + 8 * g;
      f[t] = k < K ? *reinterpret_cast<const long*>(row + k) : 0;
    }
  }
  __device__ static void load_clamped(T& f, const uint8_t* row, int k0, int K, int g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = k0 + 32 * t + 8 * g;
      const long v = *reinterpret_cast<const long*>(row + min(k, K - 8));
      f[t] = k < K ? v : 0;
    }
  }
  __device__ static void mma(v4f& acc, const T& a, const T& b) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[t], b[t], acc, 0, 0, 0);
  }
};

// Residual epilogue of element (m, n) after x[m][n] was updated to xn: the block sum of squares of
// row m over the 16-column block of n (held by the 16 lanes with lane % 16 = column), and the
// next normed GEMM's operand quantise(xn * y_gain[n]).  Every lane of the wave must call this;
// lanes with ok == false pass xn = 0 and store nothing.  Returns |xn * y_gain[n]|.
template <int P>
__device__ __forceinline__ float resid_out_g(const GemmArgs& a, int m, int n, float xn, int c,
                                             bool ok, float gain) {
  const float sq = block_ssq16(xn);
  if (!ok) return 0.f;
  if (a.ssq_out && c == 0) a.ssq_out[(long long)m * (a.N / 16) + n / 16] = sq;
  if (!a.y_out) return 0.f;
  const float yv = xn * gain;
  PT<P>::store(a.y_out, (long long)m * a.N + n, yv, a.y_inv_scale);
  return fabsf(yv);
}
template <int P>
__device__ __forceinline__ float resid_out(const GemmArgs& a, int m, int n, float xn, int c,
                                           bool ok) {
  const float sq = block_ssq16(xn);
  if (!ok) return 0.f;
  if (a.ssq_out && c == 0) a.ssq_out[(long long)m * (a.N / 16) + n / 16] = sq;
  if (!a.y_out) return 0.f;
  const float yv = xn * a.y_gain[n];
  PT<P>::store(a.y_out, (long long)m * a.N + n, yv, a.y_inv_scale);
  return fabsf(yv);
}

__device__ __forceinline__ void amax_flush(float* dst, float v, int lane) {
  if (!dst) return;
  v = wave_max_f(v);
  if (lane == 0) atomic_max_abs(dst, v);
}

// ---- tile kernel (many rows): LDS-staged 64-wide K parts ----

template <int P, int AM, int EPI, int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_kernel(const GemmArgs a) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = WM * WAVES_M, BN = WN * WAVES_N;
  constexpr int ES = PT<P>::ES;
  constexpr int ROWB = KP * ES + 16;  // padded LDS row (bytes)
  constexpr int RB = WM / 16, CB = WN / 16;
  constexpr int CPR = KP * ES / 16;  // 16-byte chunks per LDS row
  __shared__ __align__(16) uint8_t lds_a[BM * ROWB];
  __shared__ __align__(16) uint8_t lds_b[BN * ROWB];
  __shared__ float s_inv[BM];
  __shared__ int s_arow[BM];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int K = a.K;

  for (int r = tid; r < BM; r += NT) {
    const int m = m0 + r;
    s_arow[r] = m < a.M ? (a.a_rows ? a.a_rows[m] : m) : -1;
  }
  __syncthreads();
  for (int r = tid; r < BM; r += NT)
    s_inv[r] = (AM == A_NORM && s_arow[r] >= 0) ? a_row_inv(a, s_arow[r]) : 1.f;

  v4f tot[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) tot[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fg = lane >> 4;
  const uint8_t* A8 = static_cast<const uint8_t*>(a.A);
  const uint8_t* W8 = static_cast<const uint8_t*>(a.W);
  for (int k0 = 0; k0 < K; k0 += KP) {
    for (int c = tid; c < BM * CPR; c += NT) {
      const int r = c / CPR, kc = c % CPR;
      const int k = k0 + kc * (16 / ES);
      const int ar = s_arow[r];
      v4i v = {0, 0, 0, 0};
      if (ar >= 0 && k < K) v = *reinterpret_cast<const v4i*>(A8 + ((long long)ar * K + k) * ES);
      *reinterpret_cast<v4i*>(lds_a + r * ROWB + kc * 16) = v;
    }
    for (int c = tid; c < BN * CPR; c += NT) {
      const int r = c / CPR, kc = c % CPR;
      const int k = k0 + kc * (16 / ES);
      const int n = n0 + r;
      v4i v = {0, 0, 0, 0};
      if (n < a.N && k < K) v = *reinterpret_cast<const v4i*>(W8 + ((long long)n * K + k) * ES);
      *reinterpret_cast<v4i*>(lds_b + r * ROWB + kc * 16) = v;
    }
    __syncthreads();
    typename Frag<P>::T af[RB], bf[CB];
#pragma unroll
    for (int i = 0; i < RB; ++i) Frag<P>::load(af[i], lds_a + (wm * WM + i * 16 + fr) * ROWB, fg);
#pragma unroll
    for (int j = 0; j < CB; ++j) Frag<P>::load(bf[j], lds_b + (wn * WN + j * 16 + fr) * ROWB, fg);
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        Frag<P>::mma(acc, af[i], bf[j]);
        tot[i][j] += acc;
      }
    __syncthreads();
  }

  const float deq = (P == P_FP8) ? a.a_scale * a.w_scale : 1.0f;
  constexpr int PATT = P == P_F32 ? P_F32 : P_BF16;
  // output value of accumulator (i, j, e): (sum of parts) * deq * row scale
  auto val = [&](int i, int j, int e) {
    return tot[i][j][e] * deq * s_inv[wm * WM + i * 16 + fg * 4 + e];
  };

  if constexpr (EPI == E_STORE || EPI == E_RESID) {
    // residual values and gains are loaded before the first store (see the wide kernel)
    float xo[RB][CB][4], gn[CB];
    if constexpr (EPI == E_RESID) {
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int n = n0 + wn * WN + j * 16 + fr;
        gn[j] = (a.y_out && n < a.N) ? a.y_gain[n] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int m = m0 + wm * WM + i * 16 + fg * 4 + e;
            const int n = n0 + wn * WN + j * 16 + fr;
            xo[i][j][e] = (m < a.M && n < a.N) ? a.out_f32[(long long)m * a.ldo + n] : 0.f;
          }
    }
    float ymax = 0.f;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = m0 + wm * WM + i * 16 + fg * 4 + e;
          const int n = n0 + wn * WN + j * 16 + fr;
          const bool ok = m < a.M && n < a.N;
          if constexpr (EPI == E_RESID) {
            float xn = 0.f;
            if (ok) {
              xn = xo[i][j][e] + val(i, j, e);
              a.out_f32[(long long)m * a.ldo + n] = xn;
            }
            ymax = fmaxf(ymax, resid_out_g<P>(a, m, n, xn, fr, ok, gn[j]));
          } else if (ok) {
            a.out_f32[(long long)m * a.ldo + n] = val(i, j, e);
          }
        }
    if constexpr (EPI == E_RESID) amax_flush(a.y_amax, ymax, lane);
  } else if constexpr (EPI == E_GLU) {
    // W rows are interleaved in 16-row groups (gate, up, gate, up, ...)
    float omax = 0.f;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; j += 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = m0 + wm * WM + i * 16 + fg * 4 + e;
          const int nb = n0 + wn * WN + j * 16;
          const int col = (nb / 32) * 16 + fr;
          if (m < a.M && col < a.N / 2)
            omax = fmaxf(omax, emit_glu<P>(a, m, col, val(i, j, e), val(i, j + 1, e)));
        }
    amax_flush(a.out_amax, omax, lane);
  } else if constexpr (EPI == E_QKV) {
    __shared__ float ct[BM][BN + 1];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ct[wm * WM + i * 16 + fg * 4 + e][wn * WN + j * 16 + fr] = val(i, j, e);
    __syncthreads();
    const int nqk = (a.Hq + a.Hk) * a.hd;
    for (int c = tid; c < BM * BN; c += NT) {
      const int r = c / BN, cn = c % BN;
      const int m = m0 + r, n = n0 + cn;
      if (m >= a.M || n >= a.N) continue;
      const float partner = n < nqk ? ct[r][rope_partner(a, n) - n0] : 0.f;
      emit_qkv_prec(a, PATT, m, n, ct[r][cn], partner);
    }
  }
}

// ---- wide tile kernel (prefill): 128x128 tiles, four 64x64 waves, double-buffered LDS ----
//
// For bf16 / fp8 with many rows.  Each K part is staged global -> registers -> LDS one part ahead
// of the MFMAs, so one barrier per part suffices.  Tiles are ordered so that the workgroups of
// one XCD (dispatch is round-robin over the 8 XCDs) take consecutive tiles of the same A rows,
// which then stay in that XCD's L2 while every column tile reads them.  The QKV epilogue needs
// both RoPE halves of a head in one wave: a wave's 64 columns are 64-aligned, so for hd = 64 the
// partner of block j is block j ^ 2 and for hd = 32 block j ^ 1, in the same lane.

constexpr int WBM = 128, WBN = 128, WTHREADS = 256;

template <int P, int AM, int EPI>
__global__ __launch_bounds__(WTHREADS, 2) void gemm_wide_kernel(const GemmArgs a, int tiles_m,
                                                                int tiles_n) {
  constexpr int ES = PT<P>::ES;
  constexpr int ROWB = KP * ES + 16;
  constexpr int TILEB = (WBM + WBN) * ROWB;
  constexpr int CPR = KP * ES / 16;           // 16-byte chunks per staged row
  constexpr int NB16 = WBN * CPR / WTHREADS;  // chunks per thread (A and W alike)
  __shared__ __align__(16) uint8_t lds[2 * TILEB];
  __shared__ float s_inv[WBM];
  __shared__ int s_arow[WBM];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int fr = lane & 15, fg = lane >> 4;
  const int K = a.K, S = (K + KP - 1) / KP;

  // XCD-aware tile order (a bijection of [0, tiles)): XCD x owns a contiguous range of tiles
  const int nt = tiles_m * tiles_n, q = nt / 8, r8 = nt % 8;
  const int bx = blockIdx.x, xcd = bx % 8, slot = bx / 8;
  const int t = xcd * q + min(xcd, r8) + slot;
  const int m0 = (t / tiles_n) * WBM, n0 = (t % tiles_n) * WBN;

  for (int r = tid; r < WBM; r += WTHREADS) {
    const int m = m0 + r;
    s_arow[r] = m < a.M ? (a.a_rows ? a.a_rows[m] : m) : -1;
  }
  __syncthreads();
  for (int r = tid; r < WBM; r += WTHREADS)
    s_inv[r] = (AM == A_NORM && s_arow[r] >= 0) ? a_row_inv(a, s_arow[r]) : 1.f;

  // global -> register staging of one K part; each thread's row addresses are resolved once
  v4i ra[NB16], rb[NB16];
  const uint8_t* pa[NB16];
  const uint8_t* pw[NB16];
  int kc16[NB16];
  {
    const uint8_t* A8 = static_cast<const uint8_t*>(a.A);
    const uint8_t* W8 = static_cast<const uint8_t*>(a.W);
#pragma unroll
    for (int u = 0; u < NB16; ++u) {
      const int c = tid + u * WTHREADS, r = c / CPR;
      kc16[u] = (c % CPR) * (16 / ES);
      const int ar = s_arow[r], n = n0 + r;
      pa[u] = ar >= 0 ? A8 + ((long long)ar * K + kc16[u]) * ES : nullptr;
      pw[u] = n < a.N ? W8 + ((long long)n * K + kc16[u]) * ES : nullptr;
    }
  }
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NB16; ++u) {
      const bool kin = k0 + kc16[u] < K;
      ra[u] = (pa[u] && kin) ? *reinterpret_cast<const v4i*>(pa[u] + k0 * ES) : v4i{0, 0, 0, 0};
      rb[u] = (pw[u] && kin) ? *reinterpret_cast<const v4i*>(pw[u] + k0 * ES) : v4i{0, 0, 0, 0};
    }
  };
  auto stage = [&](uint8_t* buf) {
#pragma unroll
    for (int u = 0; u < NB16; ++u) {
      const int c = tid + u * WTHREADS;
      *reinterpret_cast<v4i*>(buf + (c / CPR) * ROWB + (c % CPR) * 16) = ra[u];
      *reinterpret_cast<v4i*>(buf + WBM * ROWB + (c / CPR) * ROWB + (c % CPR) * 16) = rb[u];
    }
  };

  v4f tot[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) tot[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  stage(lds);
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    if (s + 1 < S) fetch((s + 1) * KP);
    const uint8_t* la = lds + (s & 1) * TILEB;
    const uint8_t* lb = la + WBM * ROWB;
    typename Frag<P>::T bf[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) Frag<P>::load(bf[j], lb + (wn * 64 + j * 16 + fr) * ROWB, fg);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      typename Frag<P>::T af;
      Frag<P>::load(af, la + (wm * 64 + i * 16 + fr) * ROWB, fg);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        Frag<P>::mma(acc, af, bf[j]);
        tot[i][j] += acc;
      }
    }
    if (s + 1 < S) stage(lds + ((s + 1) & 1) * TILEB);
    __syncthreads();
  }

  const float deq = (P == P_FP8) ? a.a_scale * a.w_scale : 1.0f;
  const int mw = m0 + wm * 64, nw = n0 + wn * 64;
  auto val = [&](int i, int j, int e) {
    return tot[i][j][e] * deq * s_inv[wm * 64 + i * 16 + fg * 4 + e];
  };
  if constexpr (EPI == E_RESID) {
    // every residual value and gain of the lane is loaded before the first store, so the loads
    // overlap instead of each waiting behind the previous output's store
    float xo[4][4][4], gn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = nw + j * 16 + fr;
      gn[j] = (a.y_out && n < a.N) ? a.y_gain[n] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mw + i * 16 + fg * 4 + e;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = nw + j * 16 + fr;
          xo[i][j][e] = (m < a.M && n < a.N) ? a.out_f32[(long long)m * a.ldo + n] : 0.f;
        }
      }
    float ymax = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mw + i * 16 + fg * 4 + e;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = nw + j * 16 + fr;
          const bool ok = m < a.M && n < a.N;
          float xn = 0.f;
          if (ok) {
            xn = xo[i][j][e] + val(i, j, e);
            a.out_f32[(long long)m * a.ldo + n] = xn;
          }
          ymax = fmaxf(ymax, resid_out_g<P>(a, m, n, xn, fr, ok, gn[j]));
        }
      }
    amax_flush(a.y_amax, ymax, lane);
  } else if constexpr (EPI == E_STORE) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mw + i * 16 + fg * 4 + e;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = nw + j * 16 + fr;
          if (m < a.M && n < a.N) a.out_f32[(long long)m * a.ldo + n] = val(i, j, e);
        }
      }
  } else if constexpr (EPI == E_GLU) {
    float omax = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mw + i * 16 + fg * 4 + e;
        if (m >= a.M) continue;
#pragma unroll
        for (int j = 0; j < 4; j += 2) {
          const int col = ((nw + j * 16) / 32) * 16 + fr;
          if (col < a.N / 2) omax = fmaxf(omax, emit_glu<P>(a, m, col, val(i, j, e), val(i, j + 1, e)));
        }
      }
    amax_flush(a.out_amax, omax, lane);
  } else if constexpr (EPI == E_QKV) {
    // the staging LDS is free after the last part's barrier: stage the tile rows' metadata and,
    // when the tile holds q/k columns, their RoPE table rows, so that the epilogue issues no
    // dependent global loads
    const int nqk = (a.Hq + a.Hk) * a.hd;
    const int px = a.hd == 64 ? 2 : 1;
    const int h2 = a.hd / 2;
    RowMeta* s_rm = reinterpret_cast<RowMeta*>(lds);
    float* s_rope = reinterpret_cast<float*>(lds + WBM * sizeof(RowMeta));
    const bool rope = n0 < nqk;
    for (int r = tid; r < WBM; r += WTHREADS)
      s_rm[r] = m0 + r < a.M ? a.rows[m0 + r] : RowMeta{0, 0, 0, 0};
    __syncthreads();
    if (rope) {
      for (int t = tid; t < WBM * h2; t += WTHREADS) {
        const int r = t / h2, i = t % h2;
        if (m0 + r < a.M) {
          const float2 cs = *reinterpret_cast<const float2*>(a.rope +
                                                            ((long long)s_rm[r].pos * h2 + i) * 2);
          *reinterpret_cast<float2*>(s_rope + (r * h2 + i) * 2) = cs;
        }
      }
      __syncthreads();
    }
    // the partner block j ^ px must be a compile-time index, or the accumulators would be
    // addressed dynamically and leave the registers
    auto emit_all = [&](auto pxc) {
      constexpr int PX = decltype(pxc)::value;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rl = wm * 64 + i * 16 + fg * 4;  // tile row of e = 0
        const int m = m0 + rl;
        if (m >= a.M) continue;
        RowMeta rm[4];
        bool ok[4];
        const float* rr[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ok[e] = m + e < a.M;
          rm[e] = s_rm[rl + e];
          rr[e] = s_rope + (rl + e) * h2 * 2;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = nw + j * 16 + fr;
          if (n >= a.N) continue;
          float v[4], pr[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            v[e] = val(i, j, e);
            pr[e] = n < nqk ? val(i, j ^ PX, e) : 0.f;
          }
          emit_qkv4_rows(a, n, rm, ok, rr, v, pr, m);
        }
      }
    };
    if (px == 2)
      emit_all(std::integral_constant<int, 2>{});
    else
      emit_all(std::integral_constant<int, 1>{});
  }
}

template <int P, int AM, int EPI>
static void gemm_wide(const GemmArgs& a, hipStream_t s) {
  const int tm = (a.M + WBM - 1) / WBM, tn = (a.N + WBN - 1) / WBN;
  hipLaunchKernelGGL((gemm_wide_kernel<P, AM, EPI>), dim3(tm * tn), dim3(WTHREADS), 0, s, a, tm,
                     tn);
}

// ---- split kernel (few rows): one workgroup per (epilogue group, chunk of mb 16-row blocks) ----
//
// A group is the set of 16-column blocks one epilogue needs together: a RoPE pair of blocks
// {b, b + hd/32} for QKV (a single block when hd = 16), a gate/up block pair for the SiLU-gated
// MLP, two adjacent blocks for plain stores, one block for residual adds.  A chunk holds mb
// (1-4) blocks of 16 rows.  Wave w of nw takes K parts w, w + nw, ...: for a part it issues the
// loads of the chunk's A fragments and the group's W fragments together, runs every (row block,
// column block) MFMA chain from zero and leaves the partial in LDS.  After one barrier the workgroup adds each output's partials in part order and
// applies the epilogue.  No cross-workgroup communication is needed.

constexpr int SPLIT_WAVES = 16;
constexpr int SPLIT_ROWS = 64;
constexpr int kSsqPre = 4;    // staged block sums of squares held per thread during the parts
constexpr int kSsqStage = 64;  // staged only for K <= 16 * kSsqStage
// Fixed rule (used without tuning): the split kernel below SKINNY_ROWS rows, the 64 x 64 tile
// kernel below WIDE_ROWS, the 128 x 128 wide kernel (BF16 / FP8) above; at a few hundred rows the
// wide kernel has too few tiles to fill the chip (the tuner measured the split kernel 3-6x faster
// there).
constexpr int SKINNY_ROWS = 512;
constexpr int WIDE_ROWS = 4096;

// inv[a_rows[m]] = the RMSNorm scale of row a_rows[m] (for the output layer)
__global__ void row_rms_kernel(const GemmArgs a, float* __restrict__ inv) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const int ar = a.a_rows ? a.a_rows[m] : m;
  inv[ar] = inv_from_ssq(a.ssq + (long long)ar * (a.K / 16), a.K, a.eps);
}

__host__ __device__ __forceinline__ int group_size(int epi, int hd) {
  if (epi == E_QKV) return hd == 16 ? 1 : 2;
  return epi == E_RESID ? 1 : 2;
}

// Block j of group gi: QKV pairs blocks (b, b + half) within a head, the others take 2 gi + j.
__device__ __forceinline__ int group_block(int epi, int hd, int gi, int j) {
  if (epi == E_QKV) {
    const int nb = hd / 16;  // blocks per head
    if (nb == 1) return gi;
    const int half = nb / 2;
    const int head = gi / half, r = gi % half;
    return head * nb + r + j * half;
  }
  if (epi == E_RESID) return gi;
  return 2 * gi + j;
}

template <int P, int AM, int EPI, int MB>
__global__ __launch_bounds__(64 * SPLIT_WAVES) void gemm_split_kernel(const GemmArgs a) {
  constexpr int ES = PT<P>::ES;
  extern __shared__ float lds[];  // partials [part][block j][row block][16 rows][16 cols], inv[64]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int K = a.K, N = a.N;
  const int S = (K + KP - 1) / KP;
  const int gi = blockIdx.x, r0 = blockIdx.y * MB * 16;
  const int M = min(a.M - r0, MB * 16);
  const int gs = group_size(EPI, a.hd);
  float* s_inv = lds + S * gs * MB * 256;
  float* s_ssq = s_inv + SPLIT_ROWS;  // [row][K / 16] when staged
  const uint8_t* A8 = static_cast<const uint8_t*>(a.A);
  const uint8_t* W8 = static_cast<const uint8_t*>(a.W);
  // only the output layer gathers its A rows (launch_gemm checks this); elsewhere the row of
  // output m is r0 + m and the prologue has no gather loads
  const int32_t* const a_rows = EPI == E_STORE ? a.a_rows : nullptr;
  // Every load of the prologue and of the parts is issued unconditionally (indices clamped into
  // range; values past the end are masked afterwards or never stored).  A load skipped by a
  // branch would make the count of loads in flight path-dependent, and the wait for an earlier
  // load would then have to drain every later one: the operands' loads would wait for the weight
  // loads issued before them, one memory round trip after the other.  For the same reason a wave
  // without parts still issues the first part's loads, of a few bytes at the start of the
  // operands.
  constexpr int NBUF = EPI == E_RESID ? 2 : 1;
  typename Frag<P>::T bf[NBUF][2], af[NBUF][MB];
  const bool real = wave < S;  // wave-uniform
  // columns past N repeat column N - 1 (never stored); K entries past K are zero in both operands
  auto load_w = [&](int s, int q, bool use) {
    const int k0 = use ? s * KP : 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      // both blocks are loaded whenever the group size is not known at compile time (QKV with
      // hd = 16 uses one), so that the count of loads does not depend on it
      if (EPI == E_RESID && j >= 1) break;
      const int n = use ? min(group_block(EPI, a.hd, gi, j) * 16 + fr, N - 1) : 0;
      Frag<P>::load_clamped(bf[q][j], W8 + (long long)n * K * ES, k0, K, fg);
    }
  };
  // This lane's A row of each row block (rows past M repeat row M - 1; their outputs are never
  // stored), resolved once for every part.
  int arow[MB];
#pragma unroll
  for (int rb = 0; rb < MB; ++rb) arow[rb] = r0 + min(rb * 16 + fr, M - 1);
  // (a wave without parts reads the start of its first A row: with gathered rows, output row
  // indices are not A row indices, and the output layer may have more output rows than A rows)
  auto load_a = [&](int s, int q, bool use) {
    const int k0 = use ? s * KP : 0;
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
      Frag<P>::load_clamped(af[q][rb], A8 + (long long)(use ? arow[rb] : arow[0]) * K * ES, k0, K,
                            fg);
  };
  // Issue order of the first part: the output layer's weights go out ahead of its gathered rows
  // (the first wait for those also covers the weights, issued just before); elsewhere the row
  // statistics go first, so that the row scales can be prepared while the weights and operand
  // rows are still in flight.
  if constexpr (EPI == E_STORE) load_w(real ? wave : 0, 0, real);
  if (a_rows) {
#pragma unroll
    for (int rb = 0; rb < MB; ++rb) arow[rb] = a_rows[arow[rb]];
  }
  // A row of output row r0 + t for the given row scales, t = threadIdx.x < M (all in wave 0):
  // lane t holds it as arow[t / 16], with no load of its own
  int ar_t = arow[0];
#pragma unroll
  for (int rb = 1; rb < MB; ++rb) ar_t = (lane >> 4) == rb ? arow[rb] : ar_t;
  // Row scales of a normed GEMM: their inputs (the block sums of squares, or the given scales)
  // are loaded before the parts' operands are consumed, so that their latency overlaps the
  // parts' loads instead of following the last MFMA.
  const int nb16 = K / 16;
  const int nss = (AM == A_NORM && !a.inv) ? M * nb16 : 0;
  const bool staged = nss > 0 && nb16 <= kSsqStage && nss <= kSsqPre * int(blockDim.x);
  float pre[kSsqPre];
  float pre_inv = 1.f;
  if (staged) {
#pragma unroll
    for (int k = 0; k < kSsqPre; ++k) {
      const int i = min(int(threadIdx.x) + k * int(blockDim.x), nss - 1);
      const int m = i / nb16;
      const int ar = a_rows ? a_rows[r0 + m] : r0 + m;
      pre[k] = a.ssq[(long long)ar * nb16 + (i - m * nb16)];
    }
  }
  // (the residual GEMMs, whose waves may own two parts, request both at the top of their loop)
  if constexpr (EPI != E_STORE && NBUF == 1) load_w(real ? wave : 0, 0, real);
  // The inputs of this thread's first epilogue item are fetched now as well: the row metadata of
  // a q/k/v output (its RoPE entry follows once the metadata is in), or the residual value and
  // gain of a residual output.
  RowMeta pre_rm{0, 0, 0, 0};
  float2 pre_cs{1.f, 0.f};
  float pre_x = 0.f, pre_g = 0.f;
  if constexpr (EPI == E_QKV) {
    pre_rm = a.rows[r0 + min(int(threadIdx.x) / (gs * 16), M - 1)];
  } else if constexpr (EPI == E_RESID) {
    const int t = threadIdx.x;
    const int m = min(t >> 4, M - 1), n = min(gi * 16 + (t & 15), N - 1);
    const float* xp = a.out_f32 + (long long)(r0 + m) * a.ldo + n;
    pre_x = *xp;
    pre_g = *(a.y_out ? a.y_gain + n : xp);  // (unused without y_out)
  }
  if constexpr (NBUF == 1) load_a(real ? wave : 0, 0, real);
  if constexpr (AM == A_NORM) {
    // only wave 0 uses it (and only with given scales); the other waves read the start of a
    // weight row they load anyway rather than all hitting one line
    const float* ip = a.inv ? a.inv + ar_t : a.ssq;
    if (wave != 0) ip = reinterpret_cast<const float*>(W8 + (long long)min(gi * 16, N - 1) * K * ES);
    pre_inv = *ip;
  }
  // a later part: weights and operand rows together
  auto load_part = [&](int s, int q) {
    load_w(s, q, true);
    load_a(s, q, true);
  };
  auto compute_part = [&](int s, int q) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= gs) break;
#pragma unroll
      for (int rb = 0; rb < MB; ++rb) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        Frag<P>::mma(acc, af[q][rb], bf[q][j]);
        float* dst = lds + (((s * gs + j) * MB + rb) << 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[(fg * 4 + e) * 16 + fr] = acc[e];
      }
    }
  };
  // the RoPE entry of this thread's first q/k output (its metadata was requested first); every
  // thread loads one (a valid table entry for any column), the epilogue uses those of q/k outputs
  auto qkv_cs = [&]() {
    if constexpr (EPI == E_QKV) {
      const int t = threadIdx.x;
      const int n = group_block(EPI, a.hd, gi, (t >> 4) % gs) * 16 + (t & 15);
      pre_cs = rope_cs(a, pre_rm.pos, n);
    }
  };
  // the chunk's row scales into s_inv (read after the barrier that follows the parts)
  auto row_scales = [&]() {
    if (staged) {
#pragma unroll
      for (int k = 0; k < kSsqPre; ++k) {
        const int i = threadIdx.x + k * int(blockDim.x);
        if (i < nss) s_ssq[i] = pre[k];
      }
      __syncthreads();
      for (int m = threadIdx.x; m < M; m += blockDim.x)
        s_inv[m] = inv_from_ssq(s_ssq + m * nb16, K, a.eps);
    } else if (AM == A_NORM && a.inv) {
      if (int(threadIdx.x) < M) s_inv[threadIdx.x] = pre_inv;
      for (int m = threadIdx.x + blockDim.x; m < M; m += blockDim.x)
        s_inv[m] = a.inv[a_rows ? a_rows[r0 + m] : r0 + m];
    } else {
      for (int m = threadIdx.x; m < M; m += blockDim.x)
        s_inv[m] = AM == A_NORM ? a_row_inv(a, a_rows ? a_rows[r0 + m] : r0 + m) : 1.f;
    }
  };
  // parts wave, wave + nw, ...
  if constexpr (NBUF == 2) {
    // both parts' loads go out before either is consumed (a first part loaded ahead of the loop
    // would be waited for before the second part's loads were issued)
    for (int s = wave; s < S; s += 2 * nw) {
      load_part(s, 0);
      if (s + nw < S) load_part(s + nw, NBUF - 1);
      compute_part(s, 0);
      if (s + nw < S) compute_part(s + nw, NBUF - 1);
    }
    qkv_cs();
    row_scales();
  } else {
    // The first part's operands are in flight (issued above) while the row scales and the RoPE
    // entries are prepared.  Every wave reaches the scales' barrier.
    row_scales();
    qkv_cs();
    for (int s = wave; s < S; s += nw) {
      if (s != wave) load_part(s, 0);
      compute_part(s, 0);
    }
  }
  __syncthreads();
  const float deq = (P == P_FP8) ? a.a_scale * a.w_scale : 1.0f;
  // output (row m of the chunk, block j, column c) = (partials summed in part order) * deq * scale
  auto sum = [&](int m, int j, int c) {
    float v = 0.f;
    for (int s = 0; s < S; ++s) v += lds[(((s * gs + j) * MB + (m >> 4)) << 8) + (m & 15) * 16 + c];
    return v * deq * s_inv[m];
  };
  if constexpr (EPI == E_GLU) {
    float omax = 0.f;
    for (int t = threadIdx.x; t < M * 16; t += blockDim.x) {
      const int m = t >> 4, c = t & 15;
      const int col = gi * 16 + c;
      if (col < N / 2)
        omax = fmaxf(omax, emit_glu<P>(a, r0 + m, col, sum(m, 0, c), sum(m, 1, c)));
    }
    amax_flush(a.out_amax, omax, lane);
  } else if constexpr (EPI == E_RESID) {
    // one block per group; every lane takes part in the block sums of squares
    float ymax = 0.f;
    for (int t0 = 0; t0 < M * 16; t0 += blockDim.x) {
      const int t = t0 + threadIdx.x;
      const int m = t >> 4, c = t & 15;
      const int n = gi * 16 + c;
      const bool ok = t < M * 16 && n < N;
      float xn = 0.f;
      float* o = a.out_f32 + (long long)(r0 + m) * a.ldo + n;
      if (ok) {
        xn = (t0 == 0 ? pre_x : *o) + sum(m, 0, c);
        *o = xn;
      }
      const float g = t0 == 0 ? pre_g : (ok && a.y_out ? a.y_gain[n] : 0.f);
      ymax = fmaxf(ymax, resid_out_g<P>(a, r0 + m, n, xn, c, ok, g));
    }
    amax_flush(a.y_amax, ymax, lane);
  } else {
    const int nqk = (a.Hq + a.Hk) * a.hd;
    for (int t = threadIdx.x; t < M * gs * 16; t += blockDim.x) {
      const int m = t / (gs * 16), j = (t >> 4) % gs, c = t & 15;
      const int n = group_block(EPI, a.hd, gi, j) * 16 + c;
      if (n >= N) continue;
      const bool first = t == int(threadIdx.x);
      const float v = sum(m, j, c);
      const long long row = r0 + m;
      if constexpr (EPI == E_STORE) {
        a.out_f32[row * a.ldo + n] = v;
      } else {
        float partner = 0.f;
        if (n < nqk) partner = a.hd == 16 ? sum(m, 0, c ^ 8) : sum(m, 1 - j, c);
        if (first)
          emit_qkv_core(a, P == P_F32 ? P_F32 : P_BF16, int(row), n, v, partner, pre_rm, pre_cs);
        else
          emit_qkv_prec(a, P == P_F32 ? P_F32 : P_BF16, int(row), n, v, partner);
      }
    }
  }
}

// ---- attention ------------------------------------------------------------------------------
//
// Keys of a query's window [s(pos), pos] are cut into 64-key chunks at fixed absolute positions,
// chunks into quads of 4 (256 keys) and quads into groups of 4 (1,024 keys).  A chunk partial is
// one softmax pass over its 64 keys:
//   m = max score, p = 2^(score - m), l = sum p (fixed order), o = V^T P^T (chained MFMAs).
// Partials are combined by the left fold
//   (m, l, o) <- (M, l 2^(m - M) + l' 2^(m' - M), o 2^(m - M) + o' 2^(m' - M)),  M = max(m, m'),
// at three levels, each from the empty state (-inf, 0, 0) and in order: the chunks of a quad, the
// quads of a group, then the groups; the output is o / l.  Folding the empty state is exact in
// either operand, so chunks outside a column's window drop out and a column's result does not
// depend on the other columns of its launch, nor on which kernel computes it.
// S^T = K Q^T puts keys on MFMA rows and (query, head) pairs on columns, so the probabilities
// leave the QK MFMA in the B-operand layout of the P*V MFMA and no transpose is needed.  Within a
// chunk, MFMA row r of block b holds key 16 (r / 4) + 4 b + r % 4: a lane's P*V operand then
// covers 16 consecutive keys over the 4 blocks, so its V^T reads are contiguous.

constexpr int KCH = 64;      // keys per chunk
constexpr int QCH = 4;       // chunks per quad
constexpr int GQ = 4;        // quads per group
constexpr int MAXQ = 12;     // quads an item may span (window <= 2,048 keys + 15 query positions)
constexpr int HDMAX = 64;
constexpr int QSTATE = 2 + HDMAX / 4;  // floats per lane of a stored state: m, l, o[16]

__device__ __forceinline__ int window_start(int pos, int L, int C) {
  return pos < L ? 0 : C * (1 + (pos - L) / C);
}

// key offset within its chunk of MFMA row r of block b
__device__ __forceinline__ int chunk_key(int b, int r) { return (r >> 2) * 16 + b * 4 + (r & 3); }

struct AttnCol {
  bool valid;
  int pos, cs, row, head;
};

struct ChunkState {
  float m, l;
  v4f o[HDMAX / 16];  // o[hb][j]: hd index hb*16 + 4 (lane/16) + j of column lane%16
};

__device__ __forceinline__ void state_empty(ChunkState& a) {
  a.m = -INFINITY;
  a.l = 0.f;
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb) a.o[hb] = v4f{0.f, 0.f, 0.f, 0.f};
}

__device__ __forceinline__ void fold(ChunkState& a, const ChunkState& b, int nhb) {
  const float M = fmaxf(a.m, b.m);
  if (M == -INFINITY) return;
  const float e1 = exp2f(a.m - M), e2 = exp2f(b.m - M);
  a.l = a.l * e1 + b.l * e2;
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb)
    if (hb < nhb) a.o[hb] = a.o[hb] * e1 + b.o[hb] * e2;
  a.m = M;
}

// state of one lane <-> 18 floats (wave-interleaved: float i of lane l at i * 64 + l)
__device__ __forceinline__ void state_put(float* dst, const ChunkState& st, int lane) {
  dst[lane] = st.m;
  dst[64 + lane] = st.l;
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb)
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(2 + hb * 4 + j) * 64 + lane] = st.o[hb][j];
}
__device__ __forceinline__ void state_get(ChunkState& st, const float* src, int lane) {
  st.m = src[lane];
  st.l = src[64 + lane];
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb)
#pragma unroll
    for (int j = 0; j < 4; ++j) st.o[hb][j] = src[(2 + hb * 4 + j) * 64 + lane];
}

template <int PA>
struct QFrag {
  v8bf b[2];
  float f[HDMAX / 4];
};

template <int PA>
__device__ __forceinline__ void load_q(QFrag<PA>& q, const AttnArgs& a, const AttnCol& c,
                                       int grp) {
  const int hd = a.hd;
  const long long qbase = ((long long)c.row * a.Hq + c.head) * hd;
  // every load is issued (clamped into the row; c's row is valid even for an invalid column) and
  // the entries outside are zeroed afterwards, so that no branch makes the loads' count
  // path-dependent (a later wait would then drain every load in flight)
  if constexpr (PA == P_BF16) {
    const uint16_t* Q = static_cast<const uint16_t*>(a.q);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int k = s * 32 + grp * 8;
      const v4i v = *reinterpret_cast<const v4i*>(Q + qbase + min(k, hd - 8));
      q.b[s] = __builtin_bit_cast(v8bf, (c.valid && k < hd) ? v : v4i{0, 0, 0, 0});
    }
  } else {
    // step s, lane group g: hd entry 16 g + s (the same mapping is used for K)
    const float* Q = static_cast<const float*>(a.q);
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const int k = 16 * grp + 4 * qd;
      const v4f v = *reinterpret_cast<const v4f*>(Q + qbase + min(k, hd - 4));
#pragma unroll
      for (int e = 0; e < 4; ++e) q.f[4 * qd + e] = (c.valid && k < hd) ? v[e] : 0.f;
    }
  }
}

// Softmax of one chunk's masked scores st (in place: scores -> probabilities); returns (m, l).
__device__ __forceinline__ void chunk_softmax(v4f (&st)[4], const AttnArgs& a, const AttnCol& c,
                                              int key0, int grp, float& m, float& l) {
  float mx = -INFINITY;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int key = key0 + chunk_key(b, grp * 4 + j);
      const bool ok = c.valid && key >= c.cs && key <= c.pos;
      st[b][j] = ok ? st[b][j] * a.scale_log2 : -INFINITY;
      mx = fmaxf(mx, st[b][j]);
    }
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  float ls = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int j = 0; j < 4; ++j) st[b][j] = mx == -INFINITY ? 0.f : exp2f(st[b][j] - mx);
    ls += (st[b][0] + st[b][1]) + (st[b][2] + st[b][3]);
  }
  ls += __shfl_xor(ls, 16, 64);
  ls += __shfl_xor(ls, 32, 64);
  m = mx;
  l = ls;
}

// One chunk partial for the 16 columns of this wave.
template <int PA>
__device__ __forceinline__ ChunkState chunk_partial(const AttnArgs& a, const AttnItem& it,
                                                    const AttnCol& c, const QFrag<PA>& q,
                                                    int chunk, int col, int grp) {
  const int hd = a.hd, nhb = hd / 16;
  const long long sbase = (long long)it.stream * a.kv_stride + (long long)it.kvh * a.ring * hd;
  const int key0 = chunk * KCH;
  // ring slot of key key0 + off (0 <= off < 64 <= ring): one wave-uniform modulo per chunk
  const int base = key0 % a.ring;
  auto slot_of = [&](int off) {
    const int t = base + off;
    return t >= a.ring ? t - a.ring : t;
  };
  // V^T operand of this lane: keys key0 + 16 grp .. + 15 (never wrapping: ring % 16 == 0)
  const int vslot = slot_of(16 * grp);
  v4f st[4];
  ChunkState r;
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb) r.o[hb] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (PA == P_BF16) {
    const uint16_t* Kc = static_cast<const uint16_t*>(a.k_cache);
    const uint16_t* Vt = static_cast<const uint16_t*>(a.vt_cache);
    // K and V^T fragments of the 4 blocks, all loads in flight together
    v4i kf[4][2];
    v4i vf[HDMAX / 16][2];  // 16 keys per lane per hd block
    // (loads clamped into range and masked afterwards, as for q)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long ks = sbase + (long long)slot_of(chunk_key(b, col)) * hd;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k = s * 32 + grp * 8;
        const v4i v = *reinterpret_cast<const v4i*>(Kc + ks + min(k, hd - 8));
        kf[b][s] = k < hd ? v : v4i{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int hb = 0; hb < HDMAX / 16; ++hb)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int hc = min(hb, nhb - 1);
        const v4i v = *reinterpret_cast<const v4i*>(
            Vt + sbase + (long long)(hc * 16 + col) * a.ring + vslot + 8 * h);
        vf[hb][h] = hb < nhb ? v : v4i{0, 0, 0, 0};
      }
    __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first MFMA
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      st[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (s * 32 < hd)
          st[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, kf[b][s]),
                                                          q.b[s], st[b], 0, 0, 0);
    }
    chunk_softmax(st, a, c, key0, grp, r.m, r.l);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      v4s pb;
#pragma unroll
      for (int j = 0; j < 4; ++j) pb[j] = short(f2bf(st[b][j]));
#pragma unroll
      for (int hb = 0; hb < HDMAX / 16; ++hb)
        if (hb < nhb) {
          // keys 4 b .. 4 b + 3 of the lane's 16: dwords 2 (b % 2) .. + 1 of half b / 2
          const v4i w = vf[hb][b >> 1];
          const v4s va = __builtin_bit_cast(v4s, (b & 1) ? int2{w[2], w[3]} : int2{w[0], w[1]});
          r.o[hb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va, pb, r.o[hb], 0, 0, 0);
        }
    }
  } else {
    const float* Kc = static_cast<const float*>(a.k_cache);
    const float* Vt = static_cast<const float*>(a.vt_cache);
    // every K and V^T fragment of the chunk requested before the first MFMA
    v4f kf[4][4], vf[HDMAX / 16][4];
    // (loads clamped into range and masked afterwards, as for q)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long ks = sbase + (long long)slot_of(chunk_key(b, col)) * hd;
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        const int k = 16 * grp + 4 * qd;
        const v4f v = *reinterpret_cast<const v4f*>(Kc + ks + min(k, hd - 4));
        kf[b][qd] = k < hd ? v : v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int hb = 0; hb < HDMAX / 16; ++hb)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int hc = min(hb, nhb - 1);
        const v4f v = *reinterpret_cast<const v4f*>(
            Vt + sbase + (long long)(hc * 16 + col) * a.ring + vslot + 4 * b);
        vf[hb][b] = hb < nhb ? v : v4f{0.f, 0.f, 0.f, 0.f};
      }
    // every load above is issued before the first MFMA (the scheduler would otherwise sink the
    // V^T loads behind the score chains, adding a memory round trip)
    __builtin_amdgcn_sched_barrier(0);
    // the four blocks' MFMA chains interleaved step by step
#pragma unroll
    for (int b = 0; b < 4; ++b) st[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < HDMAX / 4; ++s)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        st[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kf[b][s >> 2][s & 3], q.f[s], st[b], 0, 0, 0);
    chunk_softmax(st, a, c, key0, grp, r.m, r.l);
    // the four hd blocks' P*V chains interleaved step by step (same order per chain)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int hb = 0; hb < HDMAX / 16; ++hb)
          if (hb < nhb)
            r.o[hb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vf[hb][b][j], st[b][j], r.o[hb], 0, 0, 0);
  }
  return r;
}

// Column col of an item; a column past ncols is invalid and takes the last valid column's row,
// head and position, so that every address derived from it stays inside the pass.
__device__ __forceinline__ AttnCol attn_col(const AttnArgs& a, const AttnItem& it, int col) {
  const int g = a.Hq / a.Hk;
  const int cc = it.c0 + min(col, it.ncols - 1);
  AttnCol c;
  c.valid = col < it.ncols;
  const int qo = cc / g;
  c.head = it.kvh * g + cc % g;
  c.pos = it.pos_base + qo;
  c.row = it.row_base + qo;
  c.cs = window_start(c.pos, a.ctx_len, a.slide);
  return c;
}

// absolute chunk range [c_lo, c_hi] of an item
__device__ __forceinline__ void item_chunks(const AttnArgs& a, const AttnItem& it, int& c_lo,
                                            int& c_hi) {
  const int g = a.Hq / a.Hk;
  const int kmin = window_start(it.pos_base + it.c0 / g, a.ctx_len, a.slide);
  const int kmax = it.pos_base + (it.c0 + it.ncols - 1) / g;
  c_lo = kmin / KCH;
  c_hi = kmax / KCH;
}

template <int PO>
__device__ __forceinline__ float attn_store(const AttnArgs& a, const AttnItem& it,
                                            const ChunkState& s, int col, int grp) {
  const int g = a.Hq / a.Hk, hd = a.hd, nhb = hd / 16;
  float omax = 0.f;
  if (col >= it.ncols) return omax;
  const int cc = it.c0 + col;
  const long long orow = it.row_base + cc / g;
  const int oh = it.kvh * g + cc % g;
  const float oinv = (PO == P_FP8) ? 1.0f / a.out_scale : 1.0f;
#pragma unroll
  for (int hb = 0; hb < HDMAX / 16; ++hb)
    if (hb < nhb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = hb * 16 + grp * 4 + j;
        const float o = s.o[hb][j] / s.l;
        const long long idx = orow * ((long long)a.Hq * hd) + (long long)oh * hd + d;
        omax = fmaxf(omax, fabsf(o));
        if constexpr (PO == P_F32)
          PT<P_F32>::store(a.out, idx, o, 1.f);
        else if constexpr (PO == P_BF16)
          PT<P_BF16>::store(a.out, idx, o, 1.f);
        else
          PT<P_FP8>::store(a.out, idx, o, oinv);
      }
  return omax;
}

// Many items (prefill): one wave per item, the three fold levels in registers.
template <int PA, int PO>
__global__ __launch_bounds__(256) void attention_seq_kernel(const AttnArgs a) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= a.n_items) return;
  const AttnItem it = a.items[item];
  const AttnCol c = attn_col(a, it, col);
  const int nhb = a.hd / 16;
  QFrag<PA> q;
  load_q<PA>(q, a, c, grp);
  int c_lo, c_hi;
  item_chunks(a, it, c_lo, c_hi);
  ChunkState run, gs, qs;
  state_empty(run);
  constexpr int GCH = QCH * GQ;
  for (int g0 = (c_lo / GCH) * GCH; g0 <= c_hi; g0 += GCH) {
    state_empty(gs);
    for (int q0 = g0; q0 < g0 + GCH; q0 += QCH) {
      if (q0 + QCH - 1 < c_lo || q0 > c_hi) continue;
      state_empty(qs);
      for (int ch = max(q0, c_lo); ch <= min(q0 + QCH - 1, c_hi); ++ch)
        fold(qs, chunk_partial<PA>(a, it, c, q, ch, col, grp), nhb);
      fold(gs, qs, nhb);
    }
    fold(run, gs, nhb);
  }
  float omax = attn_store<PO>(a, it, run, col, grp);
  if (a.out_amax) {
    omax = wave_max_f(omax);
    if (lane == 0) atomic_max_abs(a.out_amax, omax);
  }
}

// Few items (decode), first kernel: one 4-wave workgroup per (item, quad); wave w computes chunk
// 4 Q + w, wave 0 folds the quad in order and stores its state.  When several items share a
// stream's K/V (the column blocks of a multi-row pass, consecutive in the item list), work unit
// u = item + n_items * qi is placed by an XCD-aware bijection of the 1-D grid (dispatch is
// round-robin over the 8 XCDs): XCD x runs a contiguous range of units, so those items read the
// same K/V chunks from one L2.  Otherwise (one row per stream, where contiguous ranges would
// gather the empty units past short windows on a few XCDs) the units keep the round-robin order.
template <int PA>
__global__ __launch_bounds__(256) void attention_quad_kernel(const AttnArgs a) {
  __shared__ float part[QCH][QSTATE * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int nu = gridDim.x;
  int item = blockIdx.x % a.n_items, qi = blockIdx.x / a.n_items;
  if (a.xcd_place) {
    const int q8 = nu / 8, r8 = nu % 8, xcd = blockIdx.x % 8;
    const int u = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
    item = u % a.n_items;
    qi = u / a.n_items;
  }
  const AttnItem it = a.items[item];
  int c_lo, c_hi;
  item_chunks(a, it, c_lo, c_hi);
  const int q0 = (c_lo / QCH + qi) * QCH;
  if (q0 > c_hi) return;  // beyond the item: its fold never reads this quad
  const AttnCol c = attn_col(a, it, col);
  const int nhb = a.hd / 16;
  const int ch = q0 + wave;
  if (ch >= c_lo && ch <= c_hi) {
    QFrag<PA> q;
    load_q<PA>(q, a, c, grp);
    state_put(part[wave], chunk_partial<PA>(a, it, c, q, ch, col, grp), lane);
  }
  __syncthreads();
  if (wave != 0) return;
  ChunkState qs, p;
  state_empty(qs);
  for (int w = 0; w < QCH; ++w) {
    if (q0 + w < c_lo || q0 + w > c_hi) continue;
    state_get(p, part[w], lane);
    fold(qs, p, nhb);
  }
  state_put(a.ws + ((long long)item * MAXQ + qi) * QSTATE * 64, qs, lane);
}

// Few items, second kernel: quads -> groups -> output, one workgroup per (item, head-dimension
// block hb): a state's m and l and its block hb fold on their own (the other blocks only scale
// alike), so the four blocks' folds run side by side.  Wave w folds the quads of the item's w-th
// group (their states loaded together) and leaves the group state in LDS; wave 0 then folds the
// groups in order.  The folds are the sequential kernel's, in the same order, so the output is
// the same.
constexpr int FOLD_WAVES = (MAXQ + GQ - 2) / GQ + 1;  // groups an item may span
constexpr int BSTATE = 2 + 4;                         // floats per lane of a one-block state
template <int PO>
__global__ __launch_bounds__(64 * FOLD_WAVES) void attention_fold_kernel(const AttnArgs a) {
  __shared__ float gst[FOLD_WAVES][BSTATE * 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  const int item = blockIdx.x, hb = blockIdx.y;
  const AttnItem it = a.items[item];
  int c_lo, c_hi;
  item_chunks(a, it, c_lo, c_hi);
  const int qlo = c_lo / QCH, qhi = c_hi / QCH;
  const int gfirst = (qlo / GQ) * GQ;
  const int ng = (qhi - gfirst) / GQ + 1;  // <= FOLD_WAVES: qhi - qlo < MAXQ
  const float* src = a.ws + (long long)item * MAXQ * QSTATE * 64;
  // m, l and block hb of a quad state (state_put layout) as a one-block state
  auto get_block = [&](ChunkState& st, const float* q) {
    st.m = q[lane];
    st.l = q[64 + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j) st.o[0][j] = q[(2 + hb * 4 + j) * 64 + lane];
  };
  if (w < ng) {
    const int g0 = gfirst + w * GQ;
    ChunkState gs, p[GQ];
#pragma unroll
    for (int u = 0; u < GQ; ++u)
      if (g0 + u >= qlo && g0 + u <= qhi) get_block(p[u], src + (g0 + u - qlo) * QSTATE * 64);
    state_empty(gs);
#pragma unroll
    for (int u = 0; u < GQ; ++u)
      if (g0 + u >= qlo && g0 + u <= qhi) fold(gs, p[u], 1);
    gst[w][lane] = gs.m;
    gst[w][64 + lane] = gs.l;
#pragma unroll
    for (int j = 0; j < 4; ++j) gst[w][(2 + j) * 64 + lane] = gs.o[0][j];
  }
  __syncthreads();
  if (w != 0) return;
  ChunkState run, gs;
  state_empty(run);
  state_empty(gs);
  for (int k = 0; k < ng; ++k) {
    gs.m = gst[k][lane];
    gs.l = gst[k][64 + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j) gs.o[0][j] = gst[k][(2 + j) * 64 + lane];
    fold(run, gs, 1);
  }
  // output block hb of the lane's column: attn_store's arithmetic for one block
  float omax = 0.f;
  if (col < it.ncols) {
    const int g = a.Hq / a.Hk, hd = a.hd;
    const int cc = it.c0 + col;
    const long long orow = it.row_base + cc / g;
    const int oh = it.kvh * g + cc % g;
    const float oinv = (PO == P_FP8) ? 1.0f / a.out_scale : 1.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = hb * 16 + grp * 4 + j;
      const float o = run.o[0][j] / run.l;
      const long long idx = orow * ((long long)a.Hq * hd) + (long long)oh * hd + d;
      omax = fmaxf(omax, fabsf(o));
      if constexpr (PO == P_F32)
        PT<P_F32>::store(a.out, idx, o, 1.f);
      else if constexpr (PO == P_BF16)
        PT<P_BF16>::store(a.out, idx, o, 1.f);
      else
        PT<P_FP8>::store(a.out, idx, o, oinv);
    }
  }
  if (a.out_amax) {
    omax = wave_max_f(omax);
    if (lane == 0) atomic_max_abs(a.out_amax, omax);
  }
}

// ---- small kernels ------------------------------------------------------------------------

// x[r] = E[tok]; one wave per row, which also writes the row's inverse RMS (row_inv_rms order).
// x[r] = E[tok], the block sums of squares of the row, and y[r] = quantise(x[r] * gain)
// Few items, FP32 (decode): the quad kernel's work spread over four workgroups per quad, so that
// each chunk's MFMA chains run on four SIMDs instead of one.  Workgroup (item, quad, chunk):
// wave w runs the score chain of key block w, the four blocks' scores meet in LDS, every wave
// takes the chunk's softmax (the same code, the same bits), and wave w runs the P*V chain of
// head-dimension block w.  The chunk state is published at device scope: each store is written
// through to the device's coherence point, every wave waits until its stores are acknowledged
// (s_waitcnt 0), and after a barrier one thread counts the chunk in with a device-scope atomic.
// The workgroup that brings the count to the quad's number of chunks reads the quad's chunk
// states from that point, folds them in order (as the quad kernel does, hd block w in wave w),
// stores the quad state for the fold kernel and resets the count to zero for the next launch.
// No thread waits for another workgroup, so the launch always drains.
constexpr int kChunkItems = 24;  // largest item count of the chunk-parallel path
constexpr int CST = 6;           // floats per lane of one wave's chunk state: m, l, o[4]

__device__ __forceinline__ float* chunk_slot(const AttnArgs& a, int item, int qi, int cw, int w) {
  float* base = a.ws + (size_t)a.n_items * MAXQ * QSTATE * 64;  // after the quad states
  return base + ((((size_t)item * MAXQ + qi) * QCH + cw) * 4 + w) * CST * 64;
}

__global__ __launch_bounds__(256) void attention_chunk_kernel(const AttnArgs a) {
  __shared__ float s_st[4][4][64];  // scores [key block][element][lane]
  __shared__ int s_last;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int cw = blockIdx.x % QCH, rest = blockIdx.x / QCH;
  const int item = rest % a.n_items, qi = rest / a.n_items;
  const AttnItem it = a.items[item];
  int c_lo, c_hi;
  item_chunks(a, it, c_lo, c_hi);
  const int q0 = (c_lo / QCH + qi) * QCH, ch = q0 + cw;
  if (ch < c_lo || ch > c_hi) return;  // not a chunk of the item (never counted)
  const AttnCol c = attn_col(a, it, col);
  const int hd = a.hd, nhb = hd / 16;
  QFrag<P_F32> q;
  load_q<P_F32>(q, a, c, grp);
  const float* Kc = static_cast<const float*>(a.k_cache);
  const float* Vt = static_cast<const float*>(a.vt_cache);
  const long long sbase = (long long)it.stream * a.kv_stride + (long long)it.kvh * a.ring * hd;
  const int key0 = ch * KCH;
  const int base = key0 % a.ring;
  auto slot_of = [&](int off) {
    const int t = base + off;
    return t >= a.ring ? t - a.ring : t;
  };
  const int vslot = slot_of(16 * grp);
  // key block w's K fragment and head-dimension block w's V^T fragment (loads clamped into
  // range and masked afterwards, as in chunk_partial)
  v4f kf[4], vf[4];
  {
    const long long ks = sbase + (long long)slot_of(chunk_key(w, col)) * hd;
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const int k = 16 * grp + 4 * qd;
      const v4f v = *reinterpret_cast<const v4f*>(Kc + ks + min(k, hd - 4));
      kf[qd] = k < hd ? v : v4f{0.f, 0.f, 0.f, 0.f};
    }
    const int hc = min(w, nhb - 1);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const v4f v = *reinterpret_cast<const v4f*>(Vt + sbase + (long long)(hc * 16 + col) * a.ring +
                                                  vslot + 4 * b);
      vf[b] = w < nhb ? v : v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first MFMA
  v4f sw = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < HDMAX / 4; ++s)
    sw = __builtin_amdgcn_mfma_f32_16x16x4f32(kf[s >> 2][s & 3], q.f[s], sw, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) s_st[w][j][lane] = sw[j];
  __syncthreads();
  v4f st[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) st[b][j] = s_st[b][j][lane];
  ChunkState r;
  state_empty(r);
  chunk_softmax(st, a, c, key0, grp, r.m, r.l);
  if (w < nhb) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        r.o[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(vf[b][j], st[b][j], r.o[0], 0, 0, 0);
  }
  // publish this wave's part of the chunk state
  {
    float* dst = chunk_slot(a, item, qi, cw, w);
    auto put = [&](int i, float v) {
      __hip_atomic_store(dst + i * 64 + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    put(0, r.m);
    put(1, r.l);
#pragma unroll
    for (int j = 0; j < 4; ++j) put(2 + j, r.o[0][j]);
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wave's device-scope stores are acknowledged
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nv = min(q0 + QCH - 1, c_hi) - max(q0, c_lo) + 1;  // the quad's chunks
    const int old = __hip_atomic_fetch_add(a.ctr + item * MAXQ + qi, 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_last = old == nv - 1;
  }
  __syncthreads();
  if (!s_last) return;
  if (threadIdx.x == 0)
    __hip_atomic_store(a.ctr + item * MAXQ + qi, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the quad state: its chunks folded in order from the empty state (hd block w in wave w)
  ChunkState qs, p;
  state_empty(qs);
  state_empty(p);
  for (int k = 0; k < QCH; ++k) {
    if (q0 + k < c_lo || q0 + k > c_hi) continue;
    const float* src = chunk_slot(a, item, qi, k, w);
    auto get = [&](int i) {
      return __hip_atomic_load(src + i * 64 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    p.m = get(0);
    p.l = get(1);
#pragma unroll
    for (int j = 0; j < 4; ++j) p.o[0][j] = get(2 + j);
    fold(qs, p, 1);
  }
  // the fold kernel's layout (state_put): m, l, then o[hb][j] at 2 + 4 hb + j
  float* qd = a.ws + ((long long)item * MAXQ + qi) * QSTATE * 64;
  if (w == 0) {
    qd[lane] = qs.m;
    qd[64 + lane] = qs.l;
  }
  if (w < nhb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) qd[(2 + w * 4 + j) * 64 + lane] = qs.o[0][j];
  }
}

template <int P>
__global__ void embed_kernel(const float* __restrict__ E, const RowMeta* __restrict__ rows, int n,
                             int d, float* __restrict__ x, float* __restrict__ ssq, void* y,
                             const float* __restrict__ gain, float inv_scale, float* y_amax) {
  const int r = blockIdx.x;
  if (r >= n) return;
  const int lane = threadIdx.x, c = lane & 15, q = lane >> 4;
  const int nb = d / 16;
  const long long t = rows[r].tok;
  float ymax = 0.f;
  for (int b0 = 0; b0 < nb; b0 += 4) {
    const int b = b0 + q;
    const bool ok = b < nb;
    const int k = 16 * b + c;
    const float v = ok ? E[t * d + k] : 0.f;
    const float sq = block_ssq16(v);
    if (ok) {
      x[(long long)r * d + k] = v;
      if (c == 0) ssq[(long long)r * nb + b] = sq;
      const float yv = v * gain[k];
      PT<P>::store(y, (long long)r * d + k, yv, inv_scale);
      ymax = fmaxf(ymax, fabsf(yv));
    }
  }
  amax_flush(y_amax, ymax, lane);
}

template <int P>
__global__ void convert_kernel(const float* __restrict__ src, void* __restrict__ dst, long long n,
                               float inv_scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    PT<P>::store(dst, i, src[i], inv_scale);
}

// ---- launchers ------------------------------------------------------------------------------

template <int P, int AM, int EPI, int WM, int WN, int WVM, int WVN>
static void gemm_go(const GemmArgs& a, hipStream_t s) {
  constexpr int BM = WM * WVM, BN = WN * WVN;
  const dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM);
  hipLaunchKernelGGL((gemm_kernel<P, AM, EPI, WM, WN, WVM, WVN>), grid, dim3(64 * WVM * WVN), 0, s,
                     a);
}

constexpr size_t kSplitLdsMax = 144 * 1024;  // of the 160 KiB LDS of a gfx950 CU

template <int P, int AM, int EPI, int MB>
static void launch_split(dim3 grid, dim3 block, size_t lds, const GemmArgs& a, hipStream_t s) {
  static bool raised = false;  // allow more than the default 64 KiB of dynamic LDS, once
  if (!raised) {
    NC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_split_kernel<P, AM, EPI, MB>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(kSplitLdsMax)));
    raised = true;
  }
  hipLaunchKernelGGL((gemm_split_kernel<P, AM, EPI, MB>), grid, block, lds, s, a);
}

// Row blocks (16 rows each) per workgroup: GEMMs with few column groups cut M finer, so that
// more workgroups share the work and each one's chain of loads, MFMAs and epilogue is shorter.
static int split_mb(const GemmArgs& a, int epi) {
  const int nblk = (a.N + 15) / 16, gs = group_size(epi, a.hd);
  const int ngroups = (nblk + gs - 1) / gs;
  const int cap = ngroups < 64 ? 1 : ngroups < 128 ? 2 : SPLIT_ROWS / 16;
  return std::min((a.M + 15) / 16, cap);
}

static int split_parts(const GemmArgs& a) { return (a.K + KP - 1) / KP; }

static size_t split_lds(const GemmArgs& a, int epi, int mb) {
  const int nb16 = a.K / 16;
  const size_t ssq = (epi != E_RESID && nb16 <= kSsqStage) ? size_t(mb) * 16 * nb16 : 0;
  return (size_t(split_parts(a)) * group_size(epi, a.hd) * mb * 256 + SPLIT_ROWS + ssq) *
         sizeof(float);
}

template <int P, int AM, int EPI>
static void gemm_split(const GemmArgs& a, hipStream_t s, int mb, int waves) {
  const int nblk = (a.N + 15) / 16;
  const int gs = group_size(EPI, a.hd);
  const int ngroups = (nblk + gs - 1) / gs;
  const dim3 grid(ngroups, (a.M + 16 * mb - 1) / (16 * mb)), block(64 * waves);
  const size_t lds = split_lds(a, EPI, mb);
  switch (mb) {
    case 1: launch_split<P, AM, EPI, 1>(grid, block, lds, a, s); break;
    case 2: launch_split<P, AM, EPI, 2>(grid, block, lds, a, s); break;
    case 3: launch_split<P, AM, EPI, 3>(grid, block, lds, a, s); break;
    default: launch_split<P, AM, EPI, 4>(grid, block, lds, a, s); break;
  }
}

void launch_row_rms(const GemmArgs& a, float* inv, hipStream_t s) {
  if (a.M <= 0) return;
  hipLaunchKernelGGL(row_rms_kernel, dim3((a.M + 255) / 256), dim3(256), 0, s, a, inv);
  NC_HIP(hipGetLastError());
}

static bool wide_ok(int prec, int epi, const GemmArgs& a) {
  return prec != P_F32 && (epi != E_QKV || a.hd == 32 || a.hd == 64);
}

static bool tile_valid(int prec, int epi, const GemmArgs& a, const GemmTile& t) {
  switch (t.kind) {
    case T_AUTO: return true;
    case T_SPLIT:
      return t.mb >= 1 && t.mb <= SPLIT_ROWS / 16 && t.waves >= 1 && t.waves <= SPLIT_WAVES &&
             split_lds(a, epi, t.mb) <= kSplitLdsMax;
    case T_TILE_S:
    case T_TILE_M: return true;
    case T_WIDE: return wide_ok(prec, epi, a);
    default: return false;
  }
}

// The fixed rule used when no measured choice is given.
static GemmTile default_tile(int prec, int epi, const GemmArgs& a) {
  const int S = split_parts(a);
  const GemmTile sp{T_SPLIT, split_mb(a, epi), S < SPLIT_WAVES ? S : SPLIT_WAVES};
  if (a.M < SKINNY_ROWS && split_lds(a, epi, sp.mb) <= kSplitLdsMax) return sp;
  if (a.M >= WIDE_ROWS && wide_ok(prec, epi, a)) return GemmTile{T_WIDE, 0, 0};
  return GemmTile{a.M <= 64 ? T_TILE_S : T_TILE_M, 0, 0};
}

bool gemm_tile_fits(int prec, int epi, const GemmArgs& a, const GemmTile& t) {
  return tile_valid(prec, epi, a, t);
}

std::vector<GemmTile> gemm_candidates(int prec, int epi, const GemmArgs& a) {
  std::vector<GemmTile> out;
  const int S = split_parts(a);
  const int wmax = S < SPLIT_WAVES ? S : SPLIT_WAVES;
  if (a.M <= 1024) {
    const int mbmax = std::min((a.M + 15) / 16, SPLIT_ROWS / 16);
    for (int mb = 1; mb <= mbmax; ++mb) {
      int prev = 0;
      for (int div = 1; div <= 4; div *= 2) {
        const int w = (wmax + div - 1) / div;
        const GemmTile t{T_SPLIT, mb, w};
        if (w != prev && tile_valid(prec, epi, a, t)) out.push_back(t);
        prev = w;
      }
    }
  }
  out.push_back(GemmTile{T_TILE_S, 0, 0});
  out.push_back(GemmTile{T_TILE_M, 0, 0});
  if (wide_ok(prec, epi, a)) out.push_back(GemmTile{T_WIDE, 0, 0});
  return out;
}

template <int P, int AM, int EPI>
static void gemm_shape(const GemmArgs& a, hipStream_t s, GemmTile t) {
  if (t.kind == T_AUTO) t = default_tile(P, EPI, a);
  if (t.kind == T_SPLIT) return gemm_split<P, AM, EPI>(a, s, t.mb, t.waves);
  if constexpr (P != P_F32) {
    if (t.kind == T_WIDE) return gemm_wide<P, AM, EPI>(a, s);
  }
  if constexpr (EPI == E_GLU) {
    if (t.kind == T_TILE_S)
      gemm_go<P, AM, EPI, 16, 32, 1, 2>(a, s);
    else
      gemm_go<P, AM, EPI, 32, 32, 2, 2>(a, s);
  } else {
    if (t.kind == T_TILE_S)
      gemm_go<P, AM, EPI, 16, 16, 1, 4>(a, s);
    else
      gemm_go<P, AM, EPI, 32, 32, 2, 2>(a, s);
  }
}

template <int P>
static void gemm_prec(int amode, int epi, const GemmArgs& a, hipStream_t s, GemmTile t) {
  if (amode == A_NORM) {
    switch (epi) {
      case E_STORE: return gemm_shape<P, A_NORM, E_STORE>(a, s, t);
      case E_GLU: return gemm_shape<P, A_NORM, E_GLU>(a, s, t);
      case E_QKV: return gemm_shape<P, A_NORM, E_QKV>(a, s, t);
      default: break;
    }
  } else if (epi == E_RESID) {
    return gemm_shape<P, A_DIRECT, E_RESID>(a, s, t);
  }
  fail(NC_E_INVALID, "unsupported GEMM variant");
}

void launch_gemm(int prec, int amode, int epi, const GemmArgs& a, hipStream_t s, GemmTile t) {
  if (a.M <= 0) return;
  NC_CHECK(a.K % 16 == 0, NC_E_INVALID, "GEMM K must be a multiple of 16");
  if (epi == E_QKV) NC_CHECK(64 % a.hd == 0, NC_E_INVALID, "head_dim must divide 64");
  if (epi == E_GLU) NC_CHECK(a.N % 32 == 0, NC_E_INVALID, "d_ffn must be a multiple of 16");
  if (amode == A_NORM) NC_CHECK(a.ssq || a.inv, NC_E_INVALID, "normed GEMM needs row statistics");
  NC_CHECK(!a.a_rows || epi == E_STORE, NC_E_INVALID, "only the output layer gathers A rows");
  if (epi == E_RESID)
    NC_CHECK(a.N % 16 == 0 && (!a.y_out || a.y_gain), NC_E_INVALID, "bad residual epilogue");
  NC_CHECK(tile_valid(prec, epi, a, t), NC_E_INVALID, "GEMM launch shape does not fit this GEMM");
  if (prec == P_F32)
    gemm_prec<P_F32>(amode, epi, a, s, t);
  else if (prec == P_BF16)
    gemm_prec<P_BF16>(amode, epi, a, s, t);
  else
    gemm_prec<P_FP8>(amode, epi, a, s, t);
  NC_HIP(hipGetLastError());
}

// Quads an item can span: its keys run from the window start of its first query to its last
// query, at most ctx_len + 15 keys (a window holds at most ctx_len keys, an item at most 16
// query positions), i.e. at most nch chunks at any alignment.
static int attention_quads(int ctx_len) {
  const int nch = (ctx_len + 15 + KCH - 1) / KCH + 1;
  return (nch - 1 + QCH - 1) / QCH + 1;
}

template <int PA, int PO>
static void attn_go(const AttnArgs& a, bool parallel, hipStream_t s) {
  if (parallel) {
    const int nq = attention_quads(a.ctx_len);
    if (PA == P_F32 && a.ctr && a.n_items <= kChunkItems) {
      hipLaunchKernelGGL(attention_chunk_kernel, dim3(a.n_items * nq * QCH), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL((attention_quad_kernel<PA>), dim3(a.n_items * nq), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((attention_fold_kernel<PO>), dim3(a.n_items, a.hd / 16),
                       dim3(64 * FOLD_WAVES), 0, s, a);
  } else {
    hipLaunchKernelGGL((attention_seq_kernel<PA, PO>), dim3((a.n_items + 3) / 4), dim3(256), 0, s,
                       a);
  }
}

size_t attention_ws_bytes(int n_items) {
  const size_t quads = size_t(n_items) * MAXQ * QSTATE * 64;
  const size_t chunks = n_items <= kChunkItems ? size_t(n_items) * MAXQ * QCH * 4 * CST * 64 : 0;
  return (quads + chunks) * sizeof(float);
}

size_t attention_counters(int n_items) { return size_t(n_items) * MAXQ; }

// parallel: a workgroup per (item, quad of chunks) and a fold kernel (few items, decode);
// otherwise one wave per item (prefill).  Both produce the same bits.
void launch_attention(int prec_att, int prec_out, const AttnArgs& a, bool parallel,
                      hipStream_t s) {
  if (a.n_items <= 0) return;
  NC_CHECK(a.hd % 16 == 0 && a.hd <= HDMAX, NC_E_INVALID, "head_dim must be 16..64, x16");
  NC_CHECK(attention_quads(a.ctx_len) <= MAXQ, NC_E_INVALID, "context window too large");
  NC_CHECK(a.ring % 16 == 0, NC_E_INVALID, "ring must be a multiple of 16");
  if (parallel)
    NC_CHECK(a.ws && a.ws_bytes >= attention_ws_bytes(a.n_items), NC_E_INVALID,
             "attention workspace too small");
  if (prec_att == P_F32) {
    NC_CHECK(prec_out == P_F32, NC_E_INVALID, "fp32 attention feeds fp32 GEMMs");
    attn_go<P_F32, P_F32>(a, parallel, s);
  } else if (prec_out == P_BF16) {
    attn_go<P_BF16, P_BF16>(a, parallel, s);
  } else {
    attn_go<P_BF16, P_FP8>(a, parallel, s);
  }
  NC_HIP(hipGetLastError());
}

void launch_embed(const float* E, const RowMeta* rows, int n, int d, float* x, float* ssq,
                  void* y, const float* gain, int prec, float inv_scale, float* y_amax,
                  hipStream_t s) {
  if (n <= 0) return;
  NC_CHECK(d % 16 == 0, NC_E_INVALID, "d_model must be a multiple of 16");
  if (prec == P_F32)
    hipLaunchKernelGGL(embed_kernel<P_F32>, dim3(n), dim3(64), 0, s, E, rows, n, d, x, ssq, y,
                       gain, inv_scale, y_amax);
  else if (prec == P_BF16)
    hipLaunchKernelGGL(embed_kernel<P_BF16>, dim3(n), dim3(64), 0, s, E, rows, n, d, x, ssq, y,
                       gain, inv_scale, y_amax);
  else
    hipLaunchKernelGGL(embed_kernel<P_FP8>, dim3(n), dim3(64), 0, s, E, rows, n, d, x, ssq, y,
                       gain, inv_scale, y_amax);
  NC_HIP(hipGetLastError());
}

void launch_convert(const float* src, void* dst, long long n, int prec, float inv_scale,
                    hipStream_t s) {
  const int blocks = int(std::min<long long>((n + 255) / 256, 65536));
  if (prec == P_F32)
    hipLaunchKernelGGL(convert_kernel<P_F32>, dim3(blocks), dim3(256), 0, s, src, dst, n, inv_scale);
  else if (prec == P_BF16)
    hipLaunchKernelGGL(convert_kernel<P_BF16>, dim3(blocks), dim3(256), 0, s, src, dst, n,
                       inv_scale);
  else
    hipLaunchKernelGGL(convert_kernel<P_FP8>, dim3(blocks), dim3(256), 0, s, src, dst, n,
                       inv_scale);
  NC_HIP(hipGetLastError());
}

}  // namespace nc
