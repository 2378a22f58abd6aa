// Per-token vocabulary chain over a batch of streams (one row per stream and step):
//   softmax of z + b (paper section 3.3 with the section 3.7 bias, temperature 1),
//   coding distribution: bias head alone (warmup), n-gram alone (section 3.8 skip), the linear
//   mix of section 3.6, or the softmax-gated ensemble,
//   CDF-24 quantisation and scan (section 3.4) with the interval gather (encode) or the target
//   search (decode) of section 3.9,
//   online updates: bias head SGD (section 3.7), exponential-weights mixer (section 3.6), n-gram
//   counts with the 64-slot cap (section 3.5), ensemble backward + SGD,
//   n-gram prediction of the next position, its entropy and the skip decision (section 3.8).
//
// Rows are cut into 4096-entry segments, one 256-thread workgroup per (segment, row), and every
// cross-segment combination runs in segment order, so each row's result is independent of the
// launch shape and of the other rows.  No float atomics are used.
#include "cdf_dev.hpp"
#include "common.hpp"
#include "vocab_dev.hpp"

// The same probability must come out of the counting pass and the scanning pass bit for bit, so
// no multiply-add contraction is allowed to differ between them: contraction is off here.
#pragma clang fp contract(off)

namespace nc {

// ---- shared row arithmetic -----------------------------------------------------------------

__device__ __forceinline__ LsePart lse_merge(LsePart a, LsePart b) {
  const float M = fmaxf(a.m, b.m);
  if (M == -INFINITY) return LsePart{-INFINITY, 0.f};
  return LsePart{M, a.s * expf(a.m - M) + b.s * expf(b.m - M)};
}

// logsumexp of the row from its segment partials, combined in segment order; the partials are
// read 16 at a time before they are merged, so their loads overlap
__device__ __forceinline__ float row_lse(const LsePart* parts, int nseg) {
  LsePart acc{-INFINITY, 0.f};
  for (int k0 = 0; k0 < nseg; k0 += 16) {
    LsePart buf[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) buf[u] = k0 + u < nseg ? parts[k0 + u] : LsePart{-INFINITY, 0.f};
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (k0 + u < nseg) acc = k0 + u == 0 ? buf[u] : lse_merge(acc, buf[u]);
  }
  return acc.m + logf(acc.s);
}

struct RowIn {
  const float* z;   // logits of the row (modes that use the LLM)
  const float* b;   // bias vector of the stream
  const float* png; // n-gram distribution of the stream
  const float* pk;  // P_1..P_K (ensemble)
  float lse;
  int mode, use_head, K, V;
  float w[kMaxExperts];
};

// Mixture / gate weights of a stream: mixer w = exp(log w); ensemble w = softmax(theta).
__device__ __forceinline__ void row_weights(const VocabParams& P, const float* lw, float* w) {
  if (P.ensemble) {
    // every one of the kMaxOrder + 1 slots is read and written unconditionally (entries past n
    // masked by selects), so that w stays in registers; the kept terms are combined in order
    const int n = P.K + 1;
    float l[kMaxOrder + 1];
#pragma unroll
    for (int j = 0; j <= kMaxOrder; ++j) l[j] = lw[j];
    float mx = l[0];
#pragma unroll
    for (int j = 1; j <= kMaxOrder; ++j) mx = j < n ? fmaxf(mx, l[j]) : mx;
    float s = 0.f;
#pragma unroll
    for (int j = 0; j <= kMaxOrder; ++j) {
      const float e = expf(l[j] - mx);
      s = j < n ? s + e : s;
    }
#pragma unroll
    for (int j = 0; j <= kMaxOrder; ++j) w[j] = j < n ? expf(l[j] - mx) / s : 0.f;
  } else {
    // (the same slots written as by the ensemble branch, so that the two merge by value)
    w[0] = expf(lw[0]);
    w[1] = expf(lw[1]);
#pragma unroll
    for (int j = 2; j <= kMaxOrder; ++j) w[j] = 0.f;
  }
}

__device__ __forceinline__ bool uses_llm(int mode) { return mode != M_SKIP; }

// ---- the per-segment steps ------------------------------------------------------------------
//
// Each step is a device function of (segment, row, thread index within a 256-thread segment
// group), run by one workgroup per (segment, row).  Steps that contain barriers take an `active`
// flag: an inactive group passes through the barriers and touches nothing, so several groups of
// one workgroup could share them.

// V1: logsumexp partial of z + b over one segment
__device__ __forceinline__ void v1_seg(const VocabParams& P, const StreamState& S,
                                       const StepArgs& A, int seg, int r, int nseg, int tid,
                                       bool active, LsePart* wl) {
  const int lane = tid & 63, w = tid >> 6;
  const int V = P.V;
  const int s = A.rows[r];
  LsePart part{-INFINITY, 0.f};
  if (active && uses_llm(S.mode[s])) {
    const float* z = A.z + (size_t)r * V;
    const float* b = S.b + (size_t)s * V;
    float u[4][4];
    float m = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
      if (t0 + 3 < uint32_t(V)) {
        const f4v zz = *reinterpret_cast<const f4v*>(z + t0);
        const f4v bb = P.use_head ? *reinterpret_cast<const f4v*>(b + t0) : f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) u[j][i] = P.use_head ? zz[i] + bb[i] : zz[i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t t = t0 + i;
          u[j][i] = t < uint32_t(V) ? (P.use_head ? z[t] + b[t] : z[t]) : -INFINITY;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) m = fmaxf(m, u[j][i]);
    }
    float sum = 0.f;
    if (m != -INFINITY)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) sum += expf(u[j][i] - m);
    part = LsePart{m, sum};
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const LsePart o{__shfl_xor(part.m, d, 64), __shfl_xor(part.s, d, 64)};
    part = (lane & d) ? lse_merge(o, part) : lse_merge(part, o);
  }
  if (lane == 0) wl[w] = part;
  __syncthreads();
  if (active && tid == 0) {
    LsePart acc = wl[0];
    for (int k = 1; k < kSegWaves; ++k) acc = lse_merge(acc, wl[k]);
    A.lse_parts[(size_t)r * nseg + seg] = acc;
  }
  __syncthreads();  // wl is reused by the next call
}

// Row setup shared by V2 and V3 (identical code, identical results).
__device__ __forceinline__ RowIn make_row(const VocabParams& P, const StreamState& S,
                                          const StepArgs& A, int r, int s, int nseg) {
  RowIn R;
  R.V = P.V;
  R.K = P.K;
  R.mode = S.mode[s];
  R.use_head = P.use_head;
  R.z = A.z + (size_t)r * P.V;
  R.b = S.b + (size_t)s * P.V;
  R.png = S.png + (size_t)s * P.V;
  R.pk = S.pk ? S.pk + (size_t)s * P.K * P.V : nullptr;
  R.lse = uses_llm(R.mode) ? row_lse(A.lse_parts + (size_t)r * nseg, nseg) : 0.f;
  for (int j = 0; j < kMaxExperts; ++j) R.w[j] = 0.f;
  row_weights(P, S.lw + (size_t)s * kMaxExperts, R.w);
  return R;
}

// This thread's 16 entries of segment seg (4 contiguous per quarter) of the row's logits, bias and
// n-gram probabilities, loaded as vectors before the row's mode is known (the mode only selects
// among them), so that these loads overlap the row-metadata loads.  V % 4 == 0: a group of four
// is whole or past the end (zero).
struct RowVec {
  f4v z[4], b[4], g[4];
};
__device__ __forceinline__ void row_fetch(const VocabParams& P, const StreamState& S,
                                          const StepArgs& A, int r, int s, uint32_t seg, int tid,
                                          RowVec& v) {
  const float* z = A.z + (size_t)r * P.V;
  const float* b = S.b + (size_t)s * P.V;
  const float* g = S.png + (size_t)s * P.V;
  const f4v zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t t0 = seg_index(seg, j, tid, 0);
    const bool in = t0 < uint32_t(P.V);
    v.z[j] = in ? *reinterpret_cast<const f4v*>(z + t0) : zero4;
    v.b[j] = in && P.use_head ? *reinterpret_cast<const f4v*>(b + t0) : zero4;
    v.g[j] = in ? *reinterpret_cast<const f4v*>(g + t0) : zero4;
  }
}

// Probabilities of this thread's 16 entries of segment seg from the fetched vectors, zero at or
// beyond V.
__device__ __forceinline__ void row_probs(const RowIn& R, const RowVec& v, uint32_t seg, int tid,
                                          float (&p)[4][4], float (&pt)[4][4]) {
  if (R.mode == M_ENS) {
    // The ensemble also reads P_1..P_K at the thread's 16 entries: every vector is requested
    // (clamped into the row, masked after) before the first is used, rather than one dependent
    // load per entry and order.  p = w0 q + w1 P_1 + ... + wK P_K, added in that order.
    f4v pk[4][kMaxOrder];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
      const uint32_t tc = t0 < uint32_t(R.V) ? t0 : 0u;
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k)
        pk[j][k] = *reinterpret_cast<const f4v*>(R.pk + (size_t)min(k, R.K - 1) * R.V + tc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (t0 >= uint32_t(R.V)) {
          p[j][i] = pt[j][i] = 0.f;
          continue;
        }
        const float q = expf((R.use_head ? v.z[j][i] + v.b[j][i] : v.z[j][i]) - R.lse);
        pt[j][i] = q;
        float pv = R.w[0] * q;
#pragma unroll
        for (int k = 1; k <= kMaxOrder; ++k)
          if (k <= R.K) pv = pv + R.w[k] * pk[j][k - 1][i];
        p[j][i] = pv;
      }
    }
    return;
  }
  // The other forms, one loop per form (the mode is the row's, uniform over the workgroup):
  // SKIP p = g; LLM p = q; MIX p = w0 q + w1 g; with q = exp(z (+ b) - lse) the bias-head
  // probability, returned in pt (0 for SKIP).
  if (R.mode == M_SKIP) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool in = seg_index(seg, j, tid, 0) < uint32_t(R.V);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        p[j][i] = in ? v.g[j][i] : 0.f;
        pt[j][i] = 0.f;
      }
    }
    return;
  }
  const bool mix = R.mode == M_MIX;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool in = seg_index(seg, j, tid, 0) < uint32_t(R.V);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float q = expf((R.use_head ? v.z[j][i] + v.b[j][i] : v.z[j][i]) - R.lse);
      pt[j][i] = in ? q : 0.f;
      p[j][i] = in ? (mix ? R.w[0] * q + R.w[1] * v.g[j][i] : q) : 0.f;
    }
  }
}

// V2: count partial of one segment
__device__ __forceinline__ void v2_seg(const VocabParams& P, const StreamState& S,
                                       const StepArgs& A, int seg, int r, int nseg, int tid,
                                       bool active, SegLds& L) {
  float p[4][4], pt[4][4];
  RowIn R;
  if (active) {
    const int s = A.rows[r];
    RowVec v;
    row_fetch(P, S, A, r, s, seg, tid, v);
    R = make_row(P, S, A, r, s, nseg);
    row_probs(R, v, seg, tid, p, pt);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) p[j][i] = 0.f;
  }
  const SegPartial sp = seg_reduce(p, seg, P.V, P.total - P.V, L, tid);
  if (active && tid == 0) static_cast<SegPartial*>(A.seg_parts)[(size_t)r * nseg + seg] = sp;
  __syncthreads();  // L is reused by the next call
}

// V3: scan of one segment, the interval (encode) or the target search (decode), the outcome and
// the bias-head step on the segment's entries
__device__ __forceinline__ void v3_seg(const VocabParams& P, const StreamState& S,
                                       const StepArgs& A, int seg, int r, int nseg, int tid,
                                       bool active, SegLds& L, int* s_sym) {
  const int V = P.V;
  const int s = A.rows[r];
  // Issue order: the count partials of the row's segments (into registers; an LDS store right
  // after the load would wait for it before anything else is issued), the row's vectors and
  // metadata, then the key (decode: the host's target; encode: the token at the stream's next
  // position, behind the committed count), all before the scan needs any of them.
  SegPartial part{};
  if (active)
    part = static_cast<const SegPartial*>(A.seg_parts)[(size_t)r * nseg + min(tid, nseg - 1)];
  RowIn R;
  RowVec v;
  float p[4][4], pt[4][4];
  if (active) {
    row_fetch(P, S, A, r, s, seg, tid, v);
    R = make_row(P, S, A, r, s, nseg);
  }
  const int i_pos = !active ? 0 : (A.pos >= 0 ? A.pos + (A.pos_base ? *A.pos_base : 0)
                                               : S.ncommit[s]);
  const uint32_t key =
      !active ? 0u
              : (A.decode ? (A.targets ? A.targets[r] : A.targets_in[r])
                          : uint32_t(S.hist[(size_t)s * S.maxT + i_pos]));
  if (active && tid < nseg) L.parts[tid] = part;
  if (tid == 0) *s_sym = -1;
  if (active) {
    row_probs(R, v, seg, tid, p, pt);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) p[j][i] = pt[j][i] = 0.f;
  }
  __syncthreads();
  RowQuant q{};
  if (active) q = seg_combine(L.parts, nseg, seg, V, P.total);
  uint32_t base[4], cnt[4][4];
  seg_scan(p, seg, V, q, base, cnt, L, tid);
  int found = -1;
  uint32_t fcl = 0, fch = 0;
  float fp = 0.f, fpt = 0.f, fpng = 0.f;
  if (active) {
    // the entry whose interval holds the key (decode) or the key's entry (encode), by selects
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t run = base[j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t t = seg_index(seg, j, tid, i);
        const uint32_t c = cnt[j][i];
        const bool hit = t < uint32_t(V) &&
                         (A.decode ? (key >= run && key - run < c) : (t == key));
        found = hit ? int(t) : found;
        fcl = hit ? run : fcl;
        fch = hit ? run + c : fch;
        fp = hit ? p[j][i] : fp;
        fpt = hit ? pt[j][i] : fpt;
        fpng = hit ? v.g[j][i] : fpng;  // the row's p_ng at t, fetched with the row
        run += c;
      }
    }
    // full-row diagnostics (single-row probes)
    if (A.dbg_cdf || A.dbg_p || A.dbg_pt) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t run = base[j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t t = seg_index(seg, j, tid, i);
          run += cnt[j][i];
          if (t >= uint32_t(V)) continue;
          if (A.dbg_cdf) A.dbg_cdf[(size_t)r * (V + 1) + t + 1] = run;
          if (A.dbg_p) A.dbg_p[(size_t)r * V + t] = p[j][i];
          if (A.dbg_pt) A.dbg_pt[(size_t)r * V + t] = pt[j][i];
        }
      }
    }
    if (A.dbg_cdf && seg == 0 && tid == 0) A.dbg_cdf[(size_t)r * (V + 1)] = 0;
    if (found >= 0 && !A.no_update) {
      *s_sym = found;
      Outcome o;
      o.sym = q.status ? -1 : found;
      o.cl = fcl;
      o.ch = fch;
      o.mode = R.mode;
      o.p = fp;
      o.pt = fpt;
      o.png = fpng;
      o.lse = R.lse;
      for (int k = 0; k < kMaxOrder; ++k)
        o.pk[k] = (R.pk && k < P.K) ? R.pk[(size_t)k * V + found] : 0.f;
      for (int k = 0; k < kMaxExperts; ++k) o.r[k] = 0.f;
      if (R.mode == M_ENS) {
        o.r[0] = R.w[0] * fpt / fp;
#pragma unroll
        for (int k = 1; k <= kMaxOrder; ++k)
          if (k <= P.K) o.r[k] = R.w[k] * o.pk[k - 1] / fp;
      }
      A.out[r] = o;
      if (A.iv) {
        A.iv[((size_t)s * S.maxT + i_pos) * 2 + 0] = fcl;
        A.iv[((size_t)s * S.maxT + i_pos) * 2 + 1] = fch;
      }
      if (A.ptok) A.ptok[(size_t)s * S.maxT + i_pos] = fp;
    }
    if (found >= 0 && A.no_update) *s_sym = found;
    if (q.status && seg == 0 && tid == 0) {
      // invalid distribution: report through the outcome; no symbol can be coded
      Outcome o{};
      o.sym = -1;
      o.mode = R.mode;
      A.out[r] = o;
    }
  }
  // bias-head SGD step on -log ptilde(t*), section 3.7 (entries of this segment only)
  __syncthreads();
  if (active && P.use_head && !P.ensemble && (R.mode == M_LLM || R.mode == M_MIX) && !q.status &&
      !A.no_update) {
    const int sym = A.decode ? *s_sym : int(key);
    float* b = S.b + (size_t)s * V;
    // b was fetched with the row (use_head) and only this workgroup writes these entries
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
      if (t0 >= uint32_t(V)) continue;
      f4v nb;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float ind = int(t0) + i == sym ? 1.f : 0.f;
        nb[i] = v.b[j][i] - P.head_lr * (pt[j][i] - ind);
      }
      *reinterpret_cast<f4v*>(b + t0) = nb;
    }
  }
  __syncthreads();  // L and s_sym are reused by the next call
}

// V4: ensemble backward + SGD on b over one segment (no barriers)
__device__ __forceinline__ void v4_seg(const VocabParams& P, const StreamState& S,
                                       const StepArgs& A, int seg, int r, int tid) {
  const int s = A.rows[r];
  const Outcome o = A.out[r];
  if (o.sym < 0 || o.mode != M_ENS) return;
  const int V = P.V;
  const float* z = A.z + (size_t)r * V;
  float* b = S.b + (size_t)s * V;
  const float r0 = o.r[0];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = seg_index(seg, j, tid, i);
      if (t < uint32_t(V)) {
        const float q0 = expf(z[t] + b[t] - o.lse);
        const float ind = int(t) == o.sym ? 1.f : 0.f;
        b[t] = b[t] - P.head_lr * (r0 * (q0 - ind));
      }
    }
}

// ---- V5: n-gram + mixer / gate update with the coded symbol --------------------------------

// A context of up to kMaxOrder tokens.  Held by value and walked by loops unrolled to the
// compile-time bound (with the order k as a guard), so that it stays in registers.
struct Ctx {
  int32_t v[kMaxOrder];
};

__device__ __forceinline__ uint32_t ctx_hash(const Ctx& c, int k) {
  uint64_t h = 0x9E3779B97F4A7C15ull * uint64_t(k + 1);
#pragma unroll
  for (int i = 0; i < kMaxOrder; ++i)
    if (i < k) {
      h ^= uint64_t(uint32_t(c.v[i])) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
      h *= 0xBF58476D1CE4E5B9ull;
    }
  h ^= h >> 31;
  return uint32_t(h);
}

// Probe the order-k table t for the context c.v[0..k); returns the pool index or -1, and the
// empty table slot where it would go in *ins.
__device__ __forceinline__ int ctx_find(const StreamState& S, size_t t, const Ctx& c, int k,
                                         int* ins) {
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  static_assert(kMaxOrder == 4, "a table key is one 16-byte vector");
  const i4* keys = reinterpret_cast<const i4*>(S.keys + t * S.cap * 4);
  const int32_t* kidx = S.kidx + t * S.cap;
  uint32_t h = ctx_hash(c, k) & uint32_t(S.cap - 1);
  for (int probe = 0; probe < S.cap; ++probe) {
    // the slot's pool index and key are requested together (the key is read whether or not the
    // slot is in use)
    const int id = kidx[h];
    const i4 kk = keys[h];
    bool eq = true;
#pragma unroll
    for (int i = 0; i < kMaxOrder; ++i)
      if (i < k) eq = eq && kk[i] == c.v[i];
    if (id < 0) {
      *ins = int(h);
      return -1;
    }
    if (eq) return id;
    h = (h + 1) & uint32_t(S.cap - 1);
  }
  *ins = -1;
  return -1;
}

// thread k of the row's update (k = 0: unigram, history, mixer / gate; k = 1..K: order-k table);
// k < 0 does nothing but pass the barriers
__device__ __forceinline__ void v5_row(const VocabParams& P, const StreamState& S,
                                       const StepArgs& A, int r, int k) {
  const int s = A.rows[r];
  const int32_t* hist = S.hist + (size_t)s * S.maxT;
  // With the position given (batched encode) the committed token is the known one in hist, so the
  // count updates need not wait for this step's outcome; the mixer update always reads it.
  const bool given = A.pos >= 0 && !A.decode;
  const bool counts = (A.upd & kUpdCounts) != 0, mixer = (A.upd & kUpdMixer) != 0;
  const Outcome o = (mixer || !given) ? A.out[r] : Outcome{};
  const int i = k < 0 ? 0 : (A.pos >= 0 ? A.pos + (A.pos_base ? *A.pos_base : 0) : S.ncommit[s]);
  const int sym = given ? hist[i] : o.sym;
  const bool on = k >= 0 && sym >= 0 && (given || o.sym >= 0);
  __syncthreads();
  if (on && k == 0 && counts) {
    if (A.decode) S.hist[(size_t)s * S.maxT + i] = sym;
    if (P.use_ngram || P.ensemble) {
      S.uni[(size_t)s * P.V + sym] += 1;
      S.nseen[s] += 1;
    }
  }
  if (on && k == 0 && mixer && o.sym >= 0) {
    float* lw = S.lw + (size_t)s * kMaxExperts;
    if (o.mode == M_MIX) {
      // exponential weights (section 3.6): log w_j += eta log p_j(t*), then renormalise
      lw[0] = lw[0] + P.mix_eta * logf(o.pt);
      lw[1] = lw[1] + P.mix_eta * logf(o.png);
      const float mx = fmaxf(lw[0], lw[1]);
      const float ls = mx + logf(expf(lw[0] - mx) + expf(lw[1] - mx));
      lw[0] = lw[0] - ls;
      lw[1] = lw[1] - ls;
    } else if (o.mode == M_ENS) {
      float w[kMaxExperts];
      row_weights(P, lw, w);
#pragma unroll
      for (int j = 0; j <= kMaxOrder; ++j)
        if (j <= P.K) lw[j] = lw[j] - P.head_lr * (w[j] - o.r[j]);
    }
  }
  if (on && counts && (P.use_ngram || P.ensemble) && k >= 1 && k <= P.K) {
    const size_t t = (size_t)s * P.K + (k - 1);
    Ctx ctx{};
    // insert t* as a continuation of the order-k context ending at t_{i-1}
    if (i >= k) {
#pragma unroll
      for (int q = 0; q < kMaxOrder; ++q)
        if (q < k) ctx.v[q] = hist[i - k + q];
      int ins = -1;
      int id = ctx_find(S, t, ctx, k, &ins);
      if (id < 0) {
        if (ins >= 0 && S.nctx[t] < min(S.maxctx, P.ngram_max_contexts)) {
          id = S.nctx[t]++;
#pragma unroll
          for (int q = 0; q < 4; ++q) S.keys[(t * S.cap + ins) * 4 + q] = q < k ? ctx.v[q] : -1;
          S.kidx[t * S.cap + ins] = id;
          int32_t* sl = S.pool + (t * S.maxctx + id) * kSlots * 2;
          sl[0] = sym;
          sl[1] = 1;
          S.pool_n[t * S.maxctx + id] = 1;
          S.pool_sum[t * S.maxctx + id] = 1;
        }
      } else {
        int32_t* sl = S.pool + (t * S.maxctx + id) * kSlots * 2;
        const int n = S.pool_n[t * S.maxctx + id];
        // first slot holding t*, or n: eight slots per round of loads rather than one dependent
        // load per slot (kSlots is a multiple of 8, so a round stays inside the pool)
        static_assert(kSlots % 8 == 0, "slot rounds of eight");
        int j = n;
        for (int j0 = 0; j0 < n; j0 += 8) {
          typedef int32_t i4 __attribute__((ext_vector_type(4)));
          const i4* q4 = reinterpret_cast<const i4*>(sl + 2 * j0);
          const i4 a0 = q4[0], a1 = q4[1], a2 = q4[2], a3 = q4[3];
          const int32_t tk[8] = {a0.x, a0.z, a1.x, a1.z, a2.x, a2.z, a3.x, a3.z};
          int hit = -1;
#pragma unroll
          for (int u = 7; u >= 0; --u)
            if (j0 + u < n && tk[u] == sym) hit = j0 + u;
          if (hit >= 0) {
            j = hit;
            break;
          }
        }
        if (j < n) {
          sl[2 * j + 1] += 1;
          S.pool_sum[t * S.maxctx + id] += 1;
        } else if (n < kSlots) {
          sl[2 * n] = sym;
          sl[2 * n + 1] = 1;
          S.pool_n[t * S.maxctx + id] = n + 1;
          S.pool_sum[t * S.maxctx + id] += 1;
        } else {
          int ev = 0;  // lowest count, lowest slot index on ties
          for (int q = 1; q < kSlots; ++q)
            if (sl[2 * q + 1] < sl[2 * ev + 1]) ev = q;
          S.pool_sum[t * S.maxctx + id] += 1 - sl[2 * ev + 1];
          sl[2 * ev] = sym;
          sl[2 * ev + 1] = 1;
        }
      }
    }
    // context of the next position: t_{i-k+1} .. t_i (= t*)
    int nid = -1;
    if (i + 1 >= k) {
#pragma unroll
      for (int q = 0; q < kMaxOrder; ++q) {
        if (q < k - 1) ctx.v[q] = hist[i - k + 1 + q];
        if (q == k - 1) ctx.v[q] = sym;
      }
      int ins;
      nid = ctx_find(S, t, ctx, k, &ins);
    }
    S.next_ctx[(size_t)s * kMaxOrder + (k - 1)] = nid;
  }
  __syncthreads();
  if (on && k == 0 && counts) S.ncommit[s] = i + 1;
}

// ---- V6: dense n-gram prediction of the current position ------------------------------------

struct NgRow {
  float lam[kMaxOrder];
  int present[kMaxOrder];
  int id[kMaxOrder];  // pool index of the order-k context of the next position, or -1
  int n[kMaxOrder];   // its total count n_k
  float inv_norm;     // 1 / (N + V)
};

// The row's n-gram weights.  Lane q (mod kMaxOrder) of each wave fetches order q's context index
// and then that context's total count, and every lane reads the four orders' values from those
// lanes: two vector loads per row.  (Per-order scalar loads of the same values were issued one
// after the other, each behind the previous one's wait.)  Must be called by whole waves.
__device__ __forceinline__ NgRow ng_row(const VocabParams& P, const StreamState& S, int s) {
  static_assert((kMaxOrder & (kMaxOrder - 1)) == 0, "kMaxOrder must be a power of two");
  NgRow g;
  const int q = threadIdx.x & (kMaxOrder - 1);
  const int raw = S.next_ctx[(size_t)s * kMaxOrder + q];
  const int seen = S.nseen[s];
  const int idq = q < P.K ? raw : -1;
  // (indices clamped into the tables; a missing context's count is masked)
  const int nraw = S.pool_sum[((size_t)s * P.K + min(q, P.K - 1)) * S.maxctx + max(idq, 0)];
  const int nq = idq >= 0 ? nraw : 0;
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    g.id[k] = __shfl(idq, k, 64);
    g.n[k] = __shfl(nq, k, 64);
  }
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    g.present[k] = g.n[k] > 0 ? 1 : 0;
    g.lam[k] = g.present[k] ? float(g.n[k]) / (float(g.n[k]) + P.ngram_eps) : 0.f;
  }
  g.inv_norm = 1.0f / float(seen + P.V);
  return g;
}

__device__ __forceinline__ void v6_seg(const VocabParams& P, const StreamState& S,
                                       const int32_t* rows, NgPart* parts, int seg, int r,
                                       int nseg, int tid, bool active, NgPart* wl) {
  const int lane = tid & 63, w = tid >> 6;
  const int V = P.V;
  const int s = rows[r];
  float h = 0.f, mx = 0.f;
  if (active) {
    // unigram counts in, dense P_K out, four contiguous entries per load and store (V % 4 == 0)
    typedef int32_t i4v __attribute__((ext_vector_type(4)));
    i4v u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
      u[j] = t0 < uint32_t(V) ? *reinterpret_cast<const i4v*>(S.uni + (size_t)s * V + t0)
                              : i4v{0, 0, 0, 0};
    }
    const NgRow g = ng_row(P, S, s);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t0 = seg_index(seg, j, tid, 0);
      if (t0 >= uint32_t(V)) continue;
      f4v out;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t t = t0 + i;
        float pv = float(u[j][i] + 1) * g.inv_norm;  // unigram base (n_t + 1) / (N + V)
        // orders unrolled to the compile-time bound: with a runtime trip count the row weights
        // were indexed dynamically and kept in LDS, two LDS round trips per entry and order
#pragma unroll
        for (int k = 1; k <= kMaxOrder; ++k) {
          if (k > P.K) break;
          if (g.present[k - 1]) pv = (1.0f - g.lam[k - 1]) * pv;
          if (S.pk) S.pk[((size_t)s * P.K + (k - 1)) * V + t] = pv;
        }
        out[i] = pv;
        h = h - pv * log2f(pv);
        mx = fmaxf(mx, pv);
      }
      *reinterpret_cast<f4v*>(S.png + (size_t)s * V + t0) = out;
    }
  }
  h = wave_sum_f(h);
  mx = wave_max_f(mx);
  if (lane == 0) wl[w] = NgPart{h, mx};
  __syncthreads();
  if (active && tid == 0) {
    NgPart acc = wl[0];
    for (int k = 1; k < kSegWaves; ++k) {
      acc.h += wl[k].h;
      acc.mx = fmaxf(acc.mx, wl[k].mx);
    }
    parts[(size_t)r * nseg + seg] = acc;
  }
  __syncthreads();  // wl is reused by the next call
}

// ---- V7: sparse n-gram entries, entropy, skip decision ---------------------------------------

struct alignas(16) FixLds {
  int lt[kMaxOrder][kSlots], lc[kMaxOrder][kSlots], ln[kMaxOrder];
  float sh[kSegThreads], smx[kSegThreads];
};

// The last of the first ln slots of order row q holding tok, or -1 (a pool holds a token at most
// once, so it is also the first); four slots per LDS read.
__device__ __forceinline__ int slot_last(const FixLds& F, int q, int ln, int tok) {
  static_assert(kSlots % 4 == 0, "slot rows are read four at a time");
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  const i4* row = reinterpret_cast<const i4*>(F.lt[q]);
  int at = -1;
  for (int j0 = 0; j0 < ln; j0 += 4) {
    const i4 v = row[j0 >> 2];
    if (v.x == tok) at = j0;
    if (v.y == tok && j0 + 1 < ln) at = j0 + 1;
    if (v.z == tok && j0 + 2 < ln) at = j0 + 2;
    if (v.w == tok && j0 + 3 < ln) at = j0 + 3;
  }
  return at;
}

// 256 threads (tid) of one row; active == false only passes the barriers
__device__ __forceinline__ void v7_row(const VocabParams& P, const StreamState& S,
                                       const int32_t* rows, const NgPart* parts, int nseg,
                                       StepOut* step_out, const Outcome* out, int r, int tid,
                                       bool active, FixLds& F, int pos_given,
                                       const int* pos_base) {
  const int nt = kSegThreads;
  const int V = P.V;
  const int s = rows[r];
  // inputs of the final reduction and of the packed outcome, fetched now so that their latency
  // overlaps the n-gram chain below
  NgPart pre_part{0.f, 0.f};
  if (active && tid < nseg) pre_part = parts[(size_t)r * nseg + tid];
  int pre_pos = 0, pre_sym = 0;
  uint32_t pre_cl = 0, pre_ch = 0;
  float pre_p = 0.f;
  if (active && tid == 0) {
    pre_pos = pos_given >= 0 ? pos_given + (pos_base ? *pos_base : 0) : S.ncommit[s];
    if (step_out) {
      pre_sym = out[r].sym;
      pre_cl = out[r].cl;
      pre_ch = out[r].ch;
      pre_p = out[r].p;
    }
  }
  NgRow g{};
  if (active) g = ng_row(P, S, s);
  if (active && tid < kMaxOrder) F.ln[tid] = 0;
  __syncthreads();
  // wave w reads the kSlots slots of order w + 1 (one slot per lane), so the order is
  // wave-uniform and the row's per-order values are picked without indexing
  static_assert(kSlots == 64 && kMaxOrder * kSlots <= kSegThreads, "one wave per order");
  const int kw = __builtin_amdgcn_readfirstlane(tid >> 6);  // order - 1 of this wave
  int w_present = 0, w_id = -1;
#pragma unroll
  for (int q = 0; q < kMaxOrder; ++q)
    if (kw == q) {
      w_present = g.present[q];
      w_id = g.id[q];
    }
  if (active && kw < P.K && w_present) {
    const int k = kw + 1, j = tid & 63, id = w_id;
    const size_t t = (size_t)s * P.K + (k - 1);
    // the slot is read whether or not it is in use (readers stop at ln), so the slot and the
    // slot count load together
    const int2 tc = *reinterpret_cast<const int2*>(S.pool + ((t * S.maxctx + id) * kSlots + j) * 2);
    const int n = S.pool_n[t * S.maxctx + id];
    if (j == 0) F.ln[k - 1] = n;
    F.lt[k - 1][j] = tc.x;
    F.lc[k - 1][j] = tc.y;
  }
  __syncthreads();
  float dh = 0.f, dmx = 0.f;
  if (active)
    for (int e = tid; e < P.K * kSlots; e += nt) {
      const int k = e / kSlots + 1, j = e % kSlots;
      if (j >= F.ln[k - 1]) continue;
      const int tok = F.lt[k - 1][j];
      // the entry's unigram count and current p_ng are requested before the slot scans
      const int32_t u_tok = S.uni[(size_t)s * V + tok];
      const float old = S.png[(size_t)s * V + tok];
      bool owner = true;  // first occurrence over (order, slot) in increasing order
      for (int k2 = 1; k2 < k && owner; ++k2) owner = slot_last(F, k2 - 1, F.ln[k2 - 1], tok) < 0;
      if (!owner) continue;
      // P_k(tok) = lambda_k Phat_k(tok) + (1 - lambda_k) P_{k-1}(tok), k = 1..K (section 3.5)
      float pv = float(u_tok + 1) * g.inv_norm;  // unigram base (n_t + 1) / (N + V)
#pragma unroll
      for (int k2 = 1; k2 <= kMaxOrder; ++k2) {
        if (k2 > P.K) break;
        if (g.present[k2 - 1]) {
          const int at = slot_last(F, k2 - 1, F.ln[k2 - 1], tok);
          const int cnt = at >= 0 ? F.lc[k2 - 1][at] : 0;
          const float n = float(g.n[k2 - 1]);
          pv = g.lam[k2 - 1] * (float(cnt) / n) + (1.0f - g.lam[k2 - 1]) * pv;
        }
        if (S.pk) S.pk[((size_t)s * P.K + (k2 - 1)) * V + tok] = pv;
      }
      S.png[(size_t)s * V + tok] = pv;
      dh = dh + (old * log2f(old) - pv * log2f(pv));
      dmx = fmaxf(dmx, pv);
    }
  // sparse corrections: wave sums, then the four waves' in order; the dense segment partials are
  // staged in LDS by as many threads, then added in segment order
  dh = wave_sum_f(dh);
  dmx = wave_max_f(dmx);
  if (active && (tid & 63) == 0) {
    F.sh[tid >> 6] = dh;
    F.smx[tid >> 6] = dmx;
  }
  if (active && tid < nseg) {
    F.sh[kSegWaves + tid] = pre_part.h;
    F.smx[kSegWaves + tid] = pre_part.mx;
  }
  __syncthreads();
  if (active && tid == 0) {
    float H = 0.f, mx = 0.f;
    for (int k = 0; k < nseg; ++k) {
      H += F.sh[kSegWaves + k];
      mx = fmaxf(mx, F.smx[kSegWaves + k]);
    }
    float sh = F.sh[0], smx = F.smx[0];
    for (int k = 1; k < kSegWaves; ++k) {
      sh = sh + F.sh[k];
      smx = fmaxf(smx, F.smx[k]);
    }
    H = H + sh;
    mx = fmaxf(mx, smx);
    S.H[s] = H;
    S.pmax[s] = mx;
    const int pos = pre_pos;
    int mode;
    if (P.ensemble) {
      mode = M_ENS;
    } else {
      const bool warm = pos < P.warmup;
      bool skip = false;
      if (P.use_skip && !warm) {
        if (P.skip_mode == 1) skip = H < P.skip_bits;
        if (P.skip_mode == 2) skip = mx >= P.skip_pmax;
      }
      mode = skip ? M_SKIP : ((warm || !P.use_mixer) ? M_LLM : M_MIX);
    }
    S.mode[s] = mode;
    if (step_out) {
      StepOut so{};
      so.sym = pre_sym;
      so.cl = pre_cl;
      so.ch = pre_ch;
      so.next_mode = mode;
      so.p = pre_p;
      step_out[r] = so;
    }
  }
}

// ---- the segmented kernels: one workgroup per (segment, row) ---------------------------------

__global__ __launch_bounds__(kSegThreads) void vocab_lse_kernel(VocabParams P, StreamState S,
                                                                StepArgs A) {
  __shared__ LsePart wl[kSegWaves];
  v1_seg(P, S, A, blockIdx.x, blockIdx.y, gridDim.x, threadIdx.x, true, wl);
}

__global__ __launch_bounds__(kSegThreads) void vocab_count_kernel(VocabParams P, StreamState S,
                                                                  StepArgs A) {
  __shared__ SegLds L;
  v2_seg(P, S, A, blockIdx.x, blockIdx.y, gridDim.x, threadIdx.x, true, L);
}

__global__ __launch_bounds__(kSegThreads) void vocab_scan_kernel(VocabParams P, StreamState S,
                                                                 StepArgs A) {
  __shared__ SegLds L;
  __shared__ int s_sym;
  v3_seg(P, S, A, blockIdx.x, blockIdx.y, gridDim.x, threadIdx.x, true, L, &s_sym);
}

__global__ __launch_bounds__(kSegThreads) void ensemble_bias_kernel(VocabParams P, StreamState S,
                                                                    StepArgs A) {
  v4_seg(P, S, A, blockIdx.x, blockIdx.y, threadIdx.x);
}

__global__ __launch_bounds__(64) void ngram_update_kernel(VocabParams P, StreamState S,
                                                          StepArgs A) {
  v5_row(P, S, A, blockIdx.x, threadIdx.x);
}

__global__ __launch_bounds__(kSegThreads) void ngram_dense_kernel(VocabParams P, StreamState S,
                                                                  const int32_t* rows,
                                                                  NgPart* parts) {
  __shared__ NgPart wl[kSegWaves];
  v6_seg(P, S, rows, parts, blockIdx.x, blockIdx.y, gridDim.x, threadIdx.x, true, wl);
}

__global__ __launch_bounds__(kSegThreads) void ngram_fix_kernel(VocabParams P, StreamState S,
                                                                const int32_t* rows,
                                                                const NgPart* parts, int nseg,
                                                                StepOut* step_out,
                                                                const Outcome* out, int pos,
                                                                const int* pos_base) {
  __shared__ FixLds F;
  v7_row(P, S, rows, parts, nseg, step_out, out, blockIdx.x, threadIdx.x, true, F, pos,
         pos_base);
}

// ---- reset -----------------------------------------------------------------------------------

__global__ void state_reset_kernel(VocabParams P, StreamState S, int n, float w_llm) {
  const int s = blockIdx.x;
  if (s >= n) return;
  const int V = P.V;
  for (int t = threadIdx.x; t < V; t += blockDim.x) {
    S.b[(size_t)s * V + t] = 0.f;
    S.uni[(size_t)s * V + t] = 0;
  }
  if (threadIdx.x == 0) {
    S.nseen[s] = 0;
    S.ncommit[s] = 0;
    float* lw = S.lw + (size_t)s * kMaxExperts;
    for (int j = 0; j < kMaxExperts; ++j) lw[j] = 0.f;  // ensemble gate: uniform
    if (!P.ensemble) {
      lw[0] = logf(w_llm);
      lw[1] = logf(1.0f - w_llm);
    }
    for (int k = 0; k < kMaxOrder; ++k) S.next_ctx[(size_t)s * kMaxOrder + k] = -1;
    if (S.nctx)  // n-gram tables exist only when the n-gram (or the ensemble) is enabled
      for (int k = 0; k < P.K; ++k) S.nctx[(size_t)s * P.K + k] = 0;
    S.mode[s] = P.ensemble ? M_ENS : M_LLM;
    S.H[s] = 0.f;
    S.pmax[s] = 0.f;
  }
}

// ---- standalone ensemble head (shared b and theta over a batch of rows) --------------------

__device__ __forceinline__ void gate_weights(const float* theta, int n, float* w) {
  float mx = theta[0];
  for (int j = 1; j < n; ++j) mx = fmaxf(mx, theta[j]);
  float s = 0.f;
  for (int j = 0; j < n; ++j) s += expf(theta[j] - mx);
  for (int j = 0; j < n; ++j) w[j] = expf(theta[j] - mx) / s;
}

// logsumexp partials of z_r + b per (segment, row)
__global__ __launch_bounds__(kSegThreads) void ens_lse_kernel(const float* __restrict__ z,
                                                              const float* __restrict__ b, int V,
                                                              LsePart* __restrict__ parts) {
  __shared__ LsePart wl[kSegWaves];
  const int seg = blockIdx.x, r = blockIdx.y, nseg = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float u[4][4];
  float m = -INFINITY;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = seg_index(seg, j, tid, i);
      u[j][i] = t < uint32_t(V) ? z[(size_t)r * V + t] + b[t] : -INFINITY;
      m = fmaxf(m, u[j][i]);
    }
  float sum = 0.f;
  if (m != -INFINITY)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) sum += expf(u[j][i] - m);
  LsePart part{m, sum};
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const LsePart o{__shfl_xor(part.m, d, 64), __shfl_xor(part.s, d, 64)};
    part = (lane & d) ? lse_merge(o, part) : lse_merge(part, o);
  }
  if (lane == 0) wl[w] = part;
  __syncthreads();
  if (tid == 0) {
    LsePart acc = wl[0];
    for (int k = 1; k < kSegWaves; ++k) acc = lse_merge(acc, wl[k]);
    parts[(size_t)r * nseg + seg] = acc;
  }
}

// per row: lse, loss = -log p(t*), responsibilities r_j = w_j q_j(t*) / p(t*)
__global__ void ens_row_kernel(const float* __restrict__ z, const float* __restrict__ b,
                               const float* __restrict__ theta, const float* __restrict__ Pk,
                               const int32_t* __restrict__ target, int rows, int V, int nexp,
                               const LsePart* __restrict__ parts, int nseg,
                               float* __restrict__ lse_out, float* __restrict__ loss,
                               float* __restrict__ resp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float w[kMaxExperts];
  gate_weights(theta, nexp, w);
  const float lse = row_lse(parts + (size_t)r * nseg, nseg);
  lse_out[r] = lse;
  const int t = target[r];
  float q[kMaxExperts];
  q[0] = expf(z[(size_t)r * V + t] + b[t] - lse);
  float p = w[0] * q[0];
  for (int j = 1; j < nexp; ++j) {
    q[j] = Pk[((size_t)r * (nexp - 1) + (j - 1)) * V + t];
    p = p + w[j] * q[j];
  }
  if (loss) loss[r] = -logf(p);
  for (int j = 0; j < nexp; ++j) resp[(size_t)r * nexp + j] = w[j] * q[j] / p;
}

__global__ void ens_lse_to_row_kernel(const LsePart* __restrict__ parts, int rows, int nseg,
                                      float* __restrict__ lse) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows) lse[r] = row_lse(parts + (size_t)r * nseg, nseg);
}

// optional full coding distribution p_r
__global__ void ens_prob_kernel(const float* __restrict__ z, const float* __restrict__ b,
                                const float* __restrict__ theta, const float* __restrict__ Pk,
                                int rows, int V, int nexp, const float* __restrict__ lse,
                                float* __restrict__ p) {
  const int r = blockIdx.y;
  float w[kMaxExperts];
  gate_weights(theta, nexp, w);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < V; t += gridDim.x * blockDim.x) {
    float v = w[0] * expf(z[(size_t)r * V + t] + b[t] - lse[r]);
    for (int j = 1; j < nexp; ++j) v = v + w[j] * Pk[((size_t)r * (nexp - 1) + (j - 1)) * V + t];
    p[(size_t)r * V + t] = v;
  }
}

// grad_b[t] = sum_r g_r r_{r,0} (q0_r(t) - 1[t = t*_r]), rows summed in order; SGD on b.
__global__ void ens_grad_b_kernel(const float* __restrict__ z, float* __restrict__ b,
                                  const float* __restrict__ resp, const int32_t* __restrict__ target,
                                  const float* __restrict__ gl, int rows, int V, int nexp,
                                  const float* __restrict__ lse, float lr,
                                  float* __restrict__ gb) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < V; t += gridDim.x * blockDim.x) {
    const float bt = b[t];
    float g = 0.f;
    for (int r = 0; r < rows; ++r) {
      const float q0 = expf(z[(size_t)r * V + t] + bt - lse[r]);
      const float ind = target[r] == t ? 1.f : 0.f;
      g = g + gl[r] * resp[(size_t)r * nexp] * (q0 - ind);
    }
    if (gb) gb[t] = g;
    if (lr != 0.f) b[t] = bt - lr * g;
  }
}

// grad_theta[j] = sum_r g_r (w_j - r_{r,j}); SGD on theta (after every b thread read theta)
__global__ void ens_grad_theta_kernel(float* __restrict__ theta, const float* __restrict__ resp,
                                      const float* __restrict__ gl, int rows, int nexp, float lr,
                                      float* __restrict__ gth) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float w[kMaxExperts];
  gate_weights(theta, nexp, w);
  float g[kMaxExperts];
  for (int j = 0; j < nexp; ++j) {
    g[j] = 0.f;
    for (int r = 0; r < rows; ++r) g[j] = g[j] + gl[r] * (w[j] - resp[(size_t)r * nexp + j]);
  }
  for (int j = 0; j < nexp; ++j) {
    if (gth) gth[j] = g[j];
    if (lr != 0.f) theta[j] = theta[j] - lr * g[j];
  }
}

size_t ensemble_workspace_bytes(int rows, int V) {
  return size_t(rows) * (ceil_div(V, kSeg) * sizeof(LsePart) + sizeof(float)) + 256;
}

void launch_ensemble_forward(const float* z, const float* b, const float* theta, const float* Pk,
                             const int32_t* target, int rows, int V, int nexp, float* loss,
                             float* p, float* resp, void* ws, hipStream_t s) {
  if (rows <= 0) return;
  const int nseg = int(ceil_div(V, kSeg));
  LsePart* parts = static_cast<LsePart*>(ws);
  float* lse = reinterpret_cast<float*>(parts + (size_t)rows * nseg);
  hipLaunchKernelGGL(ens_lse_kernel, dim3(nseg, rows), dim3(kSegThreads), 0, s, z, b, V, parts);
  hipLaunchKernelGGL(ens_row_kernel, dim3(ceil_div(rows, 64)), dim3(64), 0, s, z, b, theta, Pk,
                     target, rows, V, nexp, parts, nseg, lse, loss, resp);
  if (p)
    hipLaunchKernelGGL(ens_prob_kernel, dim3(ceil_div(V, 256), rows), dim3(256), 0, s, z, b,
                       theta, Pk, rows, V, nexp, lse, p);
  NC_HIP(hipGetLastError());
}

void launch_ensemble_backward(const float* z, float* b, float* theta, const float* resp,
                              const int32_t* target, const float* gl, int rows, int V, int nexp,
                              float lr, float* gb, float* gth, void* ws, hipStream_t s) {
  if (rows <= 0) return;
  const int nseg = int(ceil_div(V, kSeg));
  LsePart* parts = static_cast<LsePart*>(ws);
  float* lse = reinterpret_cast<float*>(parts + (size_t)rows * nseg);
  hipLaunchKernelGGL(ens_lse_kernel, dim3(nseg, rows), dim3(kSegThreads), 0, s, z, b, V, parts);
  // lse of each row (the forward's, recomputed in the same order)
  hipLaunchKernelGGL(ens_lse_to_row_kernel, dim3(ceil_div(rows, 64)), dim3(64), 0, s, parts,
                     rows, nseg, lse);
  hipLaunchKernelGGL(ens_grad_b_kernel, dim3(ceil_div(V, 256)), dim3(256), 0, s, z, b, resp,
                     target, gl, rows, V, nexp, lse, lr, gb);
  hipLaunchKernelGGL(ens_grad_theta_kernel, dim3(1), dim3(64), 0, s, theta, resp, gl, rows, nexp,
                     lr, gth);
  NC_HIP(hipGetLastError());
}

// ---- launchers ------------------------------------------------------------------------------

void launch_vocab_dist(const VocabParams& P, const StreamState& S, const StepArgs& A,
                       hipStream_t s) {
  if (A.B <= 0) return;
  const int nseg = int(ceil_div(P.V, kSeg));
  const dim3 grid(nseg, A.B);
  if (A.lse) hipLaunchKernelGGL(vocab_lse_kernel, grid, dim3(kSegThreads), 0, s, P, S, A);
  hipLaunchKernelGGL(vocab_count_kernel, grid, dim3(kSegThreads), 0, s, P, S, A);
  hipLaunchKernelGGL(vocab_scan_kernel, grid, dim3(kSegThreads), 0, s, P, S, A);
  if (!A.no_update && P.ensemble)
    hipLaunchKernelGGL(ensemble_bias_kernel, grid, dim3(kSegThreads), 0, s, P, S, A);
  NC_HIP(hipGetLastError());
}

void launch_ngram_update(const VocabParams& P, const StreamState& S, const StepArgs& A,
                         hipStream_t s) {
  if (A.B <= 0 || A.no_update || !A.upd) return;
  hipLaunchKernelGGL(ngram_update_kernel, dim3(A.B), dim3(64), 0, s, P, S, A);
  NC_HIP(hipGetLastError());
}

void launch_vocab_step(const VocabParams& P, const StreamState& S, const StepArgs& A,
                       hipStream_t s) {
  launch_vocab_dist(P, S, A, s);
  launch_ngram_update(P, S, A, s);
}

void launch_ngram_predict(const VocabParams& P, const StreamState& S, const int32_t* rows, int B,
                          NgPart* parts, StepOut* step_out, const Outcome* out, hipStream_t s,
                          int pos, const int* pos_base) {
  if (B <= 0) return;
  const int nseg = int(ceil_div(P.V, kSeg));
  hipLaunchKernelGGL(ngram_dense_kernel, dim3(nseg, B), dim3(kSegThreads), 0, s, P, S, rows,
                     parts);
  hipLaunchKernelGGL(ngram_fix_kernel, dim3(B), dim3(256), 0, s, P, S, rows, parts, nseg,
                     step_out, out, pos, pos_base);
  NC_HIP(hipGetLastError());
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

void launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  NC_HIP(hipGetLastError());
}

void launch_state_reset(const VocabParams& P, const StreamState& S, int n_streams, float w_llm,
                        hipStream_t s) {
  if (n_streams <= 0) return;
  hipLaunchKernelGGL(state_reset_kernel, dim3(n_streams), dim3(256), 0, s, P, S, n_streams, w_llm);
  NC_HIP(hipGetLastError());
}

}  // namespace nc
