// Transformer kernels of the 135M-shape decoder (paper section 3.2 Eq. (lm), section 3.10):
// MFMA GEMMs with a fused RMSNorm prologue and fused epilogues (RoPE + KV-ring write, residual
// add, SiLU-gated MLP, logits), GQA attention over the sliding window, embedding gather and
// precision conversion.
//
// Batch invariance.  Every output element of a GEMM is the sum over K in chunks of 32 taken in
// increasing order, each chunk by the same MFMA instruction (f32 16x16x4, bf16 16x16x32, fp8
// 16x16x32), whatever the tile shape or the number of rows M.  Attention splits the keys into
// 256-key chunks at fixed absolute positions and combines the chunk partials with one fixed
// formula.  A token's logits are therefore bitwise the same whether it is evaluated in a
// 32,768-row prefill or in a one-row decode step, which the coder relies on.
#include "cdf_dev.hpp"
#include "common.hpp"
#include "llm_dev.hpp"

#include <algorithm>

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

constexpr int BK = 32;

template <int P, int AM, int EPI, int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_kernel(const GemmArgs a) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = WM * WAVES_M, BN = WN * WAVES_N;
  constexpr int ES = PT<P>::ES;
  constexpr int ROWB = BK * ES + 16;  // padded LDS row (bytes)
  constexpr int RB = WM / 16, CB = WN / 16;
  constexpr int CPR = BK * ES / 16;  // 16-byte chunks per LDS row
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
  if constexpr (AM == A_NORM) {
    // inverse RMS of each A row, one wave per row, lanes striding over K in a fixed order
    const float* X = static_cast<const float*>(a.A);
    for (int r = wave; r < BM; r += NT / 64) {
      const int ar = s_arow[r];
      float ss = 0.f;
      if (ar >= 0)
        for (int k = lane; k < K; k += 64) {
          const float v = X[(long long)ar * K + k];
          ss += v * v;
        }
      ss = wave_sum_f(ss);
      if (lane == 0) s_inv[r] = 1.0f / sqrtf(ss / float(K) + a.eps);
    }
    __syncthreads();
  }

  v4f acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float amax = 0.f;
  const float a_inv = (P == P_FP8) ? 1.0f / a.a_scale : 1.0f;

  for (int k0 = 0; k0 < K; k0 += BK) {
    // ---- global -> LDS ----
    if constexpr (AM == A_NORM) {
      const float* X = static_cast<const float*>(a.A);
      for (int c = tid; c < BM * (BK / 4); c += NT) {
        const int r = c / (BK / 4), kc = c % (BK / 4);
        const int k = k0 + kc * 4;
        const int ar = s_arow[r];
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (ar >= 0 && k < K) {
          const v4f x = *reinterpret_cast<const v4f*>(X + (long long)ar * K + k);
          const float inv = s_inv[r];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            v[i] = x[i] * inv * a.gain[k + i];
            amax = fmaxf(amax, fabsf(v[i]));
          }
        }
        PT<P>::put4(lds_a + r * ROWB + kc * 4 * ES, v, a_inv);
      }
    } else {
      const uint8_t* A8 = static_cast<const uint8_t*>(a.A);
      for (int c = tid; c < BM * CPR; c += NT) {
        const int r = c / CPR, kc = c % CPR;
        const int k = k0 + kc * (16 / ES);
        const int ar = s_arow[r];
        v4i v = {0, 0, 0, 0};
        if (ar >= 0 && k < K) v = *reinterpret_cast<const v4i*>(A8 + ((long long)ar * K + k) * ES);
        *reinterpret_cast<v4i*>(lds_a + r * ROWB + kc * 16) = v;
      }
    }
    {
      const uint8_t* W8 = static_cast<const uint8_t*>(a.W);
      for (int c = tid; c < BN * CPR; c += NT) {
        const int r = c / CPR, kc = c % CPR;
        const int k = k0 + kc * (16 / ES);
        const int n = n0 + r;
        v4i v = {0, 0, 0, 0};
        if (n < a.N && k < K) v = *reinterpret_cast<const v4i*>(W8 + ((long long)n * K + k) * ES);
        *reinterpret_cast<v4i*>(lds_b + r * ROWB + kc * 16) = v;
      }
    }
    __syncthreads();
    // ---- MFMA ----
    const int fr = lane & 15, fg = lane >> 4;
    if constexpr (P == P_BF16) {
      v8bf af[RB], bf[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
        af[i] = __builtin_bit_cast(
            v8bf, *reinterpret_cast<const v4i*>(lds_a + (wm * WM + i * 16 + fr) * ROWB + fg * 16));
#pragma unroll
      for (int j = 0; j < CB; ++j)
        bf[j] = __builtin_bit_cast(
            v8bf, *reinterpret_cast<const v4i*>(lds_b + (wn * WN + j * 16 + fr) * ROWB + fg * 16));
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    } else if constexpr (P == P_FP8) {
      long af[RB], bf[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
        af[i] = *reinterpret_cast<const long*>(lds_a + (wm * WM + i * 16 + fr) * ROWB + fg * 8);
#pragma unroll
      for (int j = 0; j < CB; ++j)
        bf[j] = *reinterpret_cast<const long*>(lds_b + (wn * WN + j * 16 + fr) * ROWB + fg * 8);
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(af[i], bf[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[RB], bf[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i)
          af[i] = *reinterpret_cast<const float*>(lds_a + (wm * WM + i * 16 + fr) * ROWB +
                                                  (kk * 4 + fg) * 4);
#pragma unroll
        for (int j = 0; j < CB; ++j)
          bf[j] = *reinterpret_cast<const float*>(lds_b + (wn * WN + j * 16 + fr) * ROWB +
                                                  (kk * 4 + fg) * 4);
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (a.a_amax) {
    amax = wave_max_f(amax);
    if (lane == 0) atomic_max_abs(a.a_amax, amax);
  }

  const float deq = (P == P_FP8) ? a.a_scale * a.w_scale : 1.0f;
  const int fr = lane & 15, fg = lane >> 4;

  if constexpr (EPI == E_STORE || EPI == E_RESID) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = m0 + wm * WM + i * 16 + fg * 4 + e;
          const int n = n0 + wn * WN + j * 16 + fr;
          if (m < a.M && n < a.N) {
            const float v = acc[i][j][e] * deq;
            float* o = a.out_f32 + (long long)m * a.ldo + n;
            if constexpr (EPI == E_RESID)
              *o += v;
            else
              *o = v;
          }
        }
  } else if constexpr (EPI == E_GLU) {
    // W rows are interleaved in 16-row groups (gate block, up block, gate block, ...), so the
    // even column block j holds gates and block j + 1 the matching up projections.
    float omax = 0.f;
    const float oinv = (P == P_FP8) ? 1.0f / a.out_scale : 1.0f;
    const int half = a.N / 2;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; j += 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = m0 + wm * WM + i * 16 + fg * 4 + e;
          const int nb = n0 + wn * WN + j * 16;  // first column of the gate block
          const int col = (nb / 32) * 16 + fr;
          if (m < a.M && col < half) {
            const float g = acc[i][j][e] * deq, u = acc[i][j + 1][e] * deq;
            const float h = g / (1.0f + expf(-g)) * u;
            omax = fmaxf(omax, fabsf(h));
            PT<P>::store(a.out_p, (long long)m * half + col, h, oinv);
          }
        }
    if (a.out_amax) {
      omax = wave_max_f(omax);
      if (lane == 0) atomic_max_abs(a.out_amax, omax);
    }
  } else if constexpr (EPI == E_QKV) {
    // stage the tile in LDS, then rotate q and k pairs (i, i + hd/2) and scatter q, k, v.
    __shared__ float ct[BM][BN + 1];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ct[wm * WM + i * 16 + fg * 4 + e][wn * WN + j * 16 + fr] = acc[i][j][e] * deq;
    __syncthreads();
    const int hd = a.hd, h2 = hd / 2;
    const int nq = a.Hq * hd, nk = a.Hk * hd;
    for (int c = tid; c < BM * BN; c += NT) {
      const int r = c / BN, cn = c % BN;
      const int m = m0 + r, n = n0 + cn;
      if (m >= a.M || n >= a.N) continue;
      const RowMeta rm = a.rows[m];
      const int within = n % hd;
      float v = ct[r][cn];
      if (n < nq + nk) {
        const int i = within < h2 ? within : within - h2;
        const float cs = a.rope[((long long)rm.pos * h2 + i) * 2 + 0];
        const float sn = a.rope[((long long)rm.pos * h2 + i) * 2 + 1];
        const float other = within < h2 ? ct[r][cn + h2] : ct[r][cn - h2];
        v = within < h2 ? v * cs - other * sn : v * cs + other * sn;
      }
      if (n < nq) {
        if constexpr (P == P_F32)
          PT<P_F32>::store(a.q_out, (long long)m * nq + n, v, 1.f);
        else
          PT<P_BF16>::store(a.q_out, (long long)m * nq + n, v, 1.f);
      } else {
        const int kv = n < nq + nk ? n - nq : n - nq - nk;
        const int kvh = kv / hd;
        const long long slot = rm.pos % a.ring;
        const long long sb = (long long)rm.stream * a.kv_stride + (long long)kvh * a.ring * hd;
        if (n < nq + nk) {
          const long long idx = sb + slot * hd + within;
          if constexpr (P == P_F32)
            PT<P_F32>::store(a.k_cache, idx, v, 1.f);
          else
            PT<P_BF16>::store(a.k_cache, idx, v, 1.f);
        } else {
          const long long idx = sb + (long long)within * a.ring + slot;
          if constexpr (P == P_F32)
            PT<P_F32>::store(a.vt_cache, idx, v, 1.f);
          else
            PT<P_BF16>::store(a.vt_cache, idx, v, 1.f);
        }
      }
    }
  }
}

// ---- attention ------------------------------------------------------------------------------

constexpr int KCH = 256;   // keys per chunk; chunks start at multiples of 256 (absolute positions)
constexpr int MAXCH = 12;  // chunks per item: covers a window of ctx_len + slide <= 2,816 keys
constexpr int HDMAX = 64;

__device__ __forceinline__ int window_start(int pos, int L, int C) {
  return pos < L ? 0 : C * (1 + (pos - L) / C);
}

// One workgroup per item; wave w handles chunks w, w + NW, ...  Per chunk and column: online
// softmax over 16-key blocks with S^T = K Q^T (keys are MFMA rows, columns are (query, head)
// pairs), so the probabilities come out of the QK MFMA already in the B-operand layout of the
// 16x16x16 P*V MFMA (lane: column l%16, keys 4(l/16)..+3).  Partials (m, l, o) go to LDS and are
// combined over chunks in increasing order by one fixed formula.
template <int PA, int PO, int NW>
__global__ __launch_bounds__(64 * NW) void attention_kernel(const AttnArgs a) {
  __shared__ float pm[MAXCH][16], pl[MAXCH][16];
  __shared__ float po[MAXCH][16][HDMAX + 1];
  const AttnItem it = a.items[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = a.Hq / a.Hk, hd = a.hd, L = a.ctx_len, C = a.slide;
  const int col = lane & 15, grp = lane >> 4;

  // this lane's column
  const int cc = it.c0 + col;
  const bool cvalid = col < it.ncols;
  const int qo = cc / g;
  const int head = it.kvh * g + cc % g;
  const int pos = it.pos_base + qo;
  const int row = it.row_base + qo;
  const int cs = window_start(pos, L, C);
  // item key range: first column has the smallest position
  const int kmin = window_start(it.pos_base + it.c0 / g, L, C);
  const int kmax = it.pos_base + (it.c0 + it.ncols - 1) / g;
  const int ch0 = kmin / KCH, nch = kmax / KCH - ch0 + 1;

  const long long sbase = (long long)it.stream * a.kv_stride + (long long)it.kvh * a.ring * hd;
  const int nkstep = PA == P_BF16 ? (hd + 31) / 32 : hd / 4;
  const int nhb = hd / 16;

  // Q^T operand (B of the QK MFMA): column col, hd entries
  v8bf qb[2];
  float qf[HDMAX / 4];
  {
    const long long qbase = ((long long)row * a.Hq + head) * hd;
    if constexpr (PA == P_BF16) {
      const uint16_t* Q = static_cast<const uint16_t*>(a.q);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        uint16_t t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k = s * 32 + grp * 8 + i;
          t[i] = (cvalid && s < nkstep && k < hd) ? Q[qbase + k] : uint16_t(0);
        }
        qb[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<v4i*>(t));
      }
    } else {
      const float* Q = static_cast<const float*>(a.q);
#pragma unroll
      for (int s = 0; s < HDMAX / 4; ++s) {
        const int k = s * 4 + grp;
        qf[s] = (cvalid && s < nkstep) ? Q[qbase + k] : 0.f;
      }
    }
  }

  for (int ci = wave; ci < nch; ci += NW) {
    const int kc0 = (ch0 + ci) * KCH;
    const int b0 = max(kc0, kmin) / 16, b1 = min(kc0 + KCH - 1, kmax) / 16;
    float m = -INFINITY, l = 0.f;
    v4f acc[HDMAX / 16];
#pragma unroll
    for (int hb = 0; hb < HDMAX / 16; ++hb) acc[hb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kb = b0; kb <= b1; ++kb) {
      const int key0 = kb * 16;
      // S^T block: rows = keys key0 + l%16 (A operand), columns = (query, head)
      v4f st = {0.f, 0.f, 0.f, 0.f};
      {
        const long long ks = sbase + (long long)((key0 + col) % a.ring) * hd;
        if constexpr (PA == P_BF16) {
          const uint16_t* Kc = static_cast<const uint16_t*>(a.k_cache);
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            if (s < nkstep) {
              v4i raw = {0, 0, 0, 0};
              const int k = s * 32 + grp * 8;
              if (k < hd) raw = *reinterpret_cast<const v4i*>(Kc + ks + k);
              st = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, raw), qb[s],
                                                           st, 0, 0, 0);
            }
          }
        } else {
          const float* Kc = static_cast<const float*>(a.k_cache);
#pragma unroll
          for (int s = 0; s < HDMAX / 4; ++s)
            if (s < nkstep)
              st = __builtin_amdgcn_mfma_f32_16x16x4f32(Kc[ks + s * 4 + grp], qf[s], st, 0, 0, 0);
        }
      }
      // mask and scale; lane holds keys key0 + 4 grp + j of column col
      float p[4];
      float mx = -INFINITY;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int key = key0 + grp * 4 + j;
        const bool ok = cvalid && key >= cs && key <= pos;
        p[j] = ok ? st[j] * a.scale_log2 : -INFINITY;
        mx = fmaxf(mx, p[j]);
      }
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      const float mn = fmaxf(m, mx);
      float alpha;
      if (mn == -INFINITY) {
        alpha = 1.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] = 0.f;
      } else {
        alpha = exp2f(m - mn);
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] = exp2f(p[j] - mn);
      }
      float rs = (p[0] + p[1]) + (p[2] + p[3]);
      rs += __shfl_xor(rs, 16, 64);
      rs += __shfl_xor(rs, 32, 64);
      l = l * alpha + rs;
      m = mn;
#pragma unroll
      for (int hb = 0; hb < HDMAX / 16; ++hb) acc[hb] *= alpha;
      // O^T += V^T P^T; A = V^T rows (hd), k = keys key0 + 4 grp + j
      const int slot = (key0 + grp * 4) % a.ring;
      if constexpr (PA == P_BF16) {
        const uint16_t* Vt = static_cast<const uint16_t*>(a.vt_cache);
        v4s pb;
#pragma unroll
        for (int j = 0; j < 4; ++j) pb[j] = short(f2bf(p[j]));
#pragma unroll
        for (int hb = 0; hb < HDMAX / 16; ++hb)
          if (hb < nhb) {
            const v4s vv = *reinterpret_cast<const v4s*>(
                Vt + sbase + (long long)(hb * 16 + col) * a.ring + slot);
            acc[hb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vv, pb, acc[hb], 0, 0, 0);
          }
      } else {
        const float* Vt = static_cast<const float*>(a.vt_cache);
#pragma unroll
        for (int hb = 0; hb < HDMAX / 16; ++hb)
          if (hb < nhb) {
            const float* vp = Vt + sbase + (long long)(hb * 16 + col) * a.ring + slot;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[hb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vp[j], p[j], acc[hb], 0, 0, 0);
          }
      }
    }
    // chunk partial: lane holds o[hd = hb*16 + 4 grp + j][column col]
    if (grp == 0) {
      pm[ci][col] = m;
      pl[ci][col] = l;
    }
#pragma unroll
    for (int hb = 0; hb < HDMAX / 16; ++hb)
      if (hb < nhb)
#pragma unroll
        for (int j = 0; j < 4; ++j) po[ci][col][hb * 16 + grp * 4 + j] = acc[hb][j];
  }
  __syncthreads();
  // combine the chunks of each column in increasing order
  const float oinv = (PO == P_FP8) ? 1.0f / a.out_scale : 1.0f;
  float omax = 0.f;
  for (int t = threadIdx.x; t < 16 * hd; t += 64 * NW) {
    const int c = t / hd, d = t % hd;
    if (c >= it.ncols) continue;
    float M = -INFINITY;
    for (int k = 0; k < nch; ++k) M = fmaxf(M, pm[k][c]);
    float Lsum = 0.f, o = 0.f;
    for (int k = 0; k < nch; ++k) {
      const float e = exp2f(pm[k][c] - M);
      Lsum += pl[k][c] * e;
      o += po[k][c][d] * e;
    }
    o = o / Lsum;
    const int ccc = it.c0 + c;
    const long long orow = it.row_base + ccc / g;
    const int oh = it.kvh * g + ccc % g;
    const long long idx = orow * ((long long)a.Hq * hd) + (long long)oh * hd + d;
    omax = fmaxf(omax, fabsf(o));
    if constexpr (PO == P_F32)
      PT<P_F32>::store(a.out, idx, o, 1.f);
    else if constexpr (PO == P_BF16)
      PT<P_BF16>::store(a.out, idx, o, 1.f);
    else
      PT<P_FP8>::store(a.out, idx, o, oinv);
  }
  if (a.out_amax) {
    omax = wave_max_f(omax);
    if (lane == 0) atomic_max_abs(a.out_amax, omax);
  }
}

// ---- small kernels ------------------------------------------------------------------------

__global__ void embed_kernel(const float* __restrict__ E, const RowMeta* __restrict__ rows, int n,
                             int d, float* __restrict__ x) {
  const int r = blockIdx.x;
  if (r >= n) return;
  const long long t = rows[r].tok;
  for (int k = threadIdx.x; k < d; k += blockDim.x) x[(long long)r * d + k] = E[t * d + k];
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

template <int P, int AM, int EPI>
static void gemm_shape(const GemmArgs& a, bool small_m, hipStream_t s) {
  if constexpr (EPI == E_GLU) {
    if (small_m)
      gemm_go<P, AM, EPI, 16, 32, 1, 2>(a, s);
    else
      gemm_go<P, AM, EPI, 32, 32, 2, 2>(a, s);
  } else {
    if (small_m)
      gemm_go<P, AM, EPI, 16, 16, 1, 4>(a, s);
    else
      gemm_go<P, AM, EPI, 32, 32, 2, 2>(a, s);
  }
}

template <int P>
static void gemm_prec(int amode, int epi, const GemmArgs& a, bool small_m, hipStream_t s) {
  if (amode == A_NORM) {
    switch (epi) {
      case E_STORE: return gemm_shape<P, A_NORM, E_STORE>(a, small_m, s);
      case E_GLU: return gemm_shape<P, A_NORM, E_GLU>(a, small_m, s);
      case E_QKV: return gemm_shape<P, A_NORM, E_QKV>(a, small_m, s);
      default: break;
    }
  } else if (epi == E_RESID) {
    return gemm_shape<P, A_DIRECT, E_RESID>(a, small_m, s);
  }
  fail(NC_E_INVALID, "unsupported GEMM variant");
}

void launch_gemm(int prec, int amode, int epi, const GemmArgs& a, bool small_m, hipStream_t s) {
  if (a.M <= 0) return;
  NC_CHECK(a.K % 16 == 0, NC_E_INVALID, "GEMM K must be a multiple of 16");
  if (epi == E_QKV) NC_CHECK(64 % a.hd == 0, NC_E_INVALID, "head_dim must divide 64");
  if (epi == E_GLU) NC_CHECK(a.N % 32 == 0, NC_E_INVALID, "d_ffn must be a multiple of 16");
  if (prec == P_F32)
    gemm_prec<P_F32>(amode, epi, a, small_m, s);
  else if (prec == P_BF16)
    gemm_prec<P_BF16>(amode, epi, a, small_m, s);
  else
    gemm_prec<P_FP8>(amode, epi, a, small_m, s);
  NC_HIP(hipGetLastError());
}

template <int PA, int PO>
static void attn_go(const AttnArgs& a, int waves, hipStream_t s) {
  if (waves >= 8)
    hipLaunchKernelGGL((attention_kernel<PA, PO, 8>), dim3(a.n_items), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((attention_kernel<PA, PO, 4>), dim3(a.n_items), dim3(256), 0, s, a);
}

void launch_attention(int prec_att, int prec_out, const AttnArgs& a, int waves, hipStream_t s) {
  if (a.n_items <= 0) return;
  NC_CHECK(a.hd % 16 == 0 && a.hd <= HDMAX, NC_E_INVALID, "head_dim must be 16..64, x16");
  NC_CHECK((a.ctx_len + a.slide) <= (MAXCH - 1) * KCH, NC_E_INVALID, "window too large");
  NC_CHECK(a.ring % 16 == 0, NC_E_INVALID, "ring must be a multiple of 16");
  if (prec_att == P_F32) {
    NC_CHECK(prec_out == P_F32, NC_E_INVALID, "fp32 attention feeds fp32 GEMMs");
    attn_go<P_F32, P_F32>(a, waves, s);
  } else if (prec_out == P_BF16) {
    attn_go<P_BF16, P_BF16>(a, waves, s);
  } else {
    attn_go<P_BF16, P_FP8>(a, waves, s);
  }
  NC_HIP(hipGetLastError());
}

void launch_embed(const float* E, const RowMeta* rows, int n, int d, float* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(embed_kernel, dim3(n), dim3(256), 0, s, E, rows, n, d, x);
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
