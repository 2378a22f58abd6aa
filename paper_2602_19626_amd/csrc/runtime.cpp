// Host runtime of the pipeline: context, device memory, transformer passes, and the encode /
// decode / probe loops of paper Algorithm 1 and its mirror.  All numerics run in the kernels of
// k_llm.hip, k_vocab.hip and k_cdf.hip; the arithmetic coder runs here on the host (section 3.9).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <array>
#include <map>
#include <tuple>
#include <vector>

#include "cdf_dev.hpp"
#include "coder.hpp"
#include "common.hpp"
#include "llm_dev.hpp"
#include "vocab_dev.hpp"

using namespace nc;

namespace {

constexpr int kBOS = 0;

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    NC_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
    n = count;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct Layer {
  float *g_attn, *g_mlp;            // RMSNorm gains (float32)
  void *Wqkv, *Wo, *Wgu, *Wd;       // GEMM precision
  float *Wqkv32, *Wo32, *Wgu32, *Wd32;  // float32 copies (FP32 mode, FP8 calibration)
  float sw_qkv = 1, sw_o = 1, sw_gu = 1, sw_d = 1;  // FP8 weight scales
  float sa_qkv = 1, sa_o = 1, sa_gu = 1, sa_d = 1;  // FP8 activation scales
};

size_t prec_bytes(int p) { return p == P_F32 ? 4 : p == P_BF16 ? 2 : 1; }

}  // namespace

// Output-layer rows per encode chunk (logits 4 V bytes each: 400 MB at V = 49,152).
constexpr int kEncodeHeadRows = 2048;

// Row-count buckets of the launch-shape table: bucket i holds row counts in
// (kRowBucketHi[i - 1], kRowBucketHi[i]].
constexpr int kRowBuckets = 21;
constexpr int kRowBucketHi[kRowBuckets] = {1,    2,    4,    8,    16,   32,    48,
                                           64,   96,   128,  192,  256,  384,   512,
                                           1024, 2048, 4096, 8192, 16384, 32768, 1 << 30};
static int row_bucket(int M) {
  int i = 0;
  while (i + 1 < kRowBuckets && M > kRowBucketHi[i]) ++i;
  return i;
}

struct nc_ctx {
  nc_config cfg{};
  int prec = P_F32, att = P_F32;
  int dev = 0;
  hipStream_t st = nullptr;
  // batched encode: the n-gram update and prediction of the next position run on st2 beside the
  // current position's distribution on st (events ev_dist[parity], ev_pred order them)
  hipStream_t st2 = nullptr;
  hipEvent_t ev_dist[2] = {nullptr, nullptr}, ev_pred = nullptr;
  int d = 0, hq = 0, hk = 0, hd = 0, F = 0, V = 0, nl = 0, R = 0;
  // weights
  std::vector<void*> allocs;
  float* E32 = nullptr;
  void* Elm = nullptr;
  float sw_lm = 1, sa_lm = 1;
  float* g_final = nullptr;
  std::vector<Layer> layers;
  bool fp8_ready = false;
  DevBuf<float> amax;  // calibration amax slots
  // rope
  DevBuf<float> rope;
  int rope_pos = 0;
  // per-stream state
  int S_alloc = 0, T_alloc = 0, n_streams = 0, maxT = 0;
  StreamState S{};
  DevBuf<float> b, png, pk, lw, Hd, pmaxd, hlast;
  DevBuf<int32_t> uni, nseen, hist, ncommit, moded, next_ctx, keys, kidx, pool, pool_n, pool_sum,
      nctx;
  DevBuf<uint8_t> kc, vc;
  long long kv_stride = 0;  // elements per stream per layer (one of K or V^T)
  DevBuf<uint32_t> iv;
  DevBuf<float> ptok;
  // pass buffers
  int rows_alloc = 0;
  DevBuf<float> x;
  DevBuf<uint8_t> qb, ob, hb;
  DevBuf<RowMeta> rowsd;
  DevBuf<AttnItem> itemsd;
  DevBuf<int32_t> lastrow;  // per stream: row of its last position in the latest pass
  DevBuf<float> xinv;       // inverse RMS of each pass row's residual
  DevBuf<float> aws;        // attention group states (decode path)
  DevBuf<int32_t> actr;     // attention chunk counters (zero between launches)
  DevBuf<float> xss;        // block sums of squares of each pass row's residual [rows][d/16]
  DevBuf<float> hinv;       // RMSNorm scale of each stream's newest row (its operand in hlast)
  DevBuf<float> yb;         // operand of the next normed GEMM, quantise(x * gain) [rows][d]
  DevBuf<uint8_t> dstage;   // per-step staged inputs
  void* spin = nullptr;     // pinned host side of the stage
  size_t spin_bytes = 0;
  // step buffers
  DevBuf<float> z;
  DevBuf<float> zseg;  // encode: logits of a chunk of positions [pos][stream slot][V]
  DevBuf<int32_t> steprows, arows;
  DevBuf<uint32_t> targets;
  DevBuf<LsePart> lsep;
  DevBuf<SegPartial> segp;
  DevBuf<NgPart> ngp;
  DevBuf<Outcome> outc;
  DevBuf<StepOut> sout;
  // decode: step outputs written by the device straight into mapped pinned host memory
  StepOut* sout_h = nullptr;   // host view
  StepOut* sout_hd = nullptr;  // device view of the same memory
  int sout_h_n = 0;
  DevBuf<float> dbgp, dbgpt;
  DevBuf<uint32_t> dbgcdf;
  // pinned host staging
  void* pin = nullptr;
  size_t pin_bytes = 0;
  // host mirrors
  std::vector<std::vector<int32_t>> hhist;  // committed tokens per stream
  std::vector<int> appended;                // x positions in the KV cache per stream
  nc_stats stats{};
  VocabParams vp{};
  // measurement: events around the launches of the enabled kernel classes
  struct ProfClass {
    bool on = false;
    uint32_t stride = 1;   // time every stride-th launch of the class
    uint64_t seen = 0;     // launches of the class since it was enabled
    bool open = false;     // the current launch is being timed
    hipEvent_t ev_open = nullptr;
    nc_kstat k{};
  };
  ProfClass prof[NC_K_COUNT];
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> ev_busy;  // (events, class)
  // measured GEMM launch shapes per (GEMM, row bucket); kind T_AUTO = the fixed rule
  GemmTile tiles[NC_G_COUNT][kRowBuckets];
  // captured transformer passes of the decode / probe paths, by pass shape; every buffer a pass
  // reads or writes is part of the key, so a reallocation selects (and captures) a new graph
  struct GraphKey {
    int n, n_items, n_last;
    size_t off_rows, off_items, off_last;
    std::array<const void*, 12> bufs;
    bool operator<(const GraphKey& o) const {
      return std::tie(n, n_items, n_last, off_rows, off_items, off_last, bufs) <
             std::tie(o.n, o.n_items, o.n_last, o.off_rows, o.off_items, o.off_last, o.bufs);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  // captured chunks of the batched encode's per-position steps, by (positions, active rows, the
  // state buffers' addresses); a replay reads its first position from posbase
  std::map<std::vector<const void*>, hipGraphExec_t> egraphs;
  DevBuf<int32_t> posbase;

  ~nc_ctx();
};

nc_ctx::~nc_ctx() {
  if (dev >= 0) (void)hipSetDevice(dev);
  if (st) (void)hipStreamSynchronize(st);
  for (void* p : allocs) (void)hipFree(p);
  DevBuf<float>* fb[] = {&yb, &xss, &aws, &xinv, &hinv, &amax, &rope, &b, &png, &pk, &lw, &Hd, &pmaxd, &hlast, &x, &ptok, &z, &zseg,
                         &dbgp, &dbgpt};
  for (auto* q : fb) q->release();
  DevBuf<int32_t>* ib[] = {&uni, &nseen, &hist, &ncommit, &moded, &next_ctx, &keys, &kidx,
                           &pool, &pool_n, &pool_sum, &nctx, &lastrow, &steprows, &arows,
                           &actr};
  for (auto* q : ib) q->release();
  kc.release();
  vc.release();
  qb.release();
  ob.release();
  hb.release();
  iv.release();
  targets.release();
  dbgcdf.release();
  rowsd.release();
  itemsd.release();
  lsep.release();
  segp.release();
  ngp.release();
  outc.release();
  sout.release();
  if (pin) (void)hipHostFree(pin);
  if (spin) (void)hipHostFree(spin);
  if (sout_h) (void)hipHostFree(sout_h);
  dstage.release();
  for (auto e : ev_free) (void)hipEventDestroy(e);
  for (auto& pr : ev_busy) {
    (void)hipEventDestroy(pr.first.first);
    (void)hipEventDestroy(pr.first.second);
  }
  for (hipEvent_t e : {ev_dist[0], ev_dist[1], ev_pred})
    if (e) (void)hipEventDestroy(e);
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  for (auto& g : egraphs) (void)hipGraphExecDestroy(g.second);
  if (st2) (void)hipStreamDestroy(st2);
  if (st) (void)hipStreamDestroy(st);
}

namespace {

void* dmalloc(nc_ctx* c, size_t bytes) {
  void* p = nullptr;
  NC_HIP(hipMalloc(&p, bytes));
  c->allocs.push_back(p);
  return p;
}

void* pinned(nc_ctx* c, size_t bytes) {
  if (bytes > c->pin_bytes) {
    if (c->pin) NC_HIP(hipHostFree(c->pin));
    c->pin = nullptr;
    NC_HIP(hipHostMalloc(&c->pin, bytes, hipHostMallocDefault));
    c->pin_bytes = bytes;
  }
  return c->pin;
}

hipEvent_t take_event(nc_ctx* c) {
  if (c->ev_free.empty()) {
    hipEvent_t e;
    NC_HIP(hipEventCreate(&e));
    return e;
  }
  hipEvent_t e = c->ev_free.back();
  c->ev_free.pop_back();
  return e;
}

// Collect the elapsed time of recorded event pairs (the stream has been synchronised).
void prof_flush(nc_ctx* c) {
  for (auto& pr : c->ev_busy) {
    float ms = 0.f;
    NC_HIP(hipEventElapsedTime(&ms, pr.first.first, pr.first.second));
    c->prof[pr.second].k.ms += ms;
    c->ev_free.push_back(pr.first.first);
    c->ev_free.push_back(pr.first.second);
  }
  c->ev_busy.clear();
}

void sync(nc_ctx* c) {
  const auto t0 = std::chrono::steady_clock::now();
  NC_HIP(hipStreamSynchronize(c->st));
  NC_HIP(hipStreamSynchronize(c->st2));
  c->stats.wait_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  prof_flush(c);
}

// Bracket the launches of one kernel class; bytes / flops are the launch's algorithmic work.
void prof_begin(nc_ctx* c, int cls, hipStream_t s = nullptr) {
  auto& P = c->prof[cls];
  if (!P.on) return;
  P.open = P.seen++ % P.stride == 0;
  if (!P.open) return;
  P.ev_open = take_event(c);
  NC_HIP(hipEventRecord(P.ev_open, s ? s : c->st));
}
void prof_end(nc_ctx* c, int cls, double bytes, double flops, hipStream_t s = nullptr) {
  auto& P = c->prof[cls];
  if (!P.on) return;
  P.k.launches += 1;
  if (!P.open) return;
  P.open = false;
  hipEvent_t e = take_event(c);
  NC_HIP(hipEventRecord(e, s ? s : c->st));
  c->ev_busy.push_back({{P.ev_open, e}, cls});
  P.k.timed += 1;
  P.k.bytes += bytes;
  P.k.flops += flops;
  if (c->ev_busy.size() > 4096) sync(c);
}

// The measured launch shape of a GEMM at M rows (the calibration pass runs in float32, whose
// shapes are not tuned, and keeps the fixed rule).
GemmTile tile_for(const nc_ctx* c, bool calib, int gemm, int M) {
  return calib ? GemmTile{} : c->tiles[gemm][row_bucket(M)];
}

double gemm_bytes(const GemmArgs& a, int amode, int epi, int prec, int att) {
  const double es = double(prec_bytes(prec));
  double b = double(a.N) * a.K * es;                                    // weights
  b += double(a.M) * a.K * es;                                          // activations
  if (epi == E_STORE) b += double(a.M) * a.N * 4.0;                     // logits
  if (epi == E_RESID) b += double(a.M) * a.N * 8.0;                     // residual read + write
  if (epi == E_GLU) b += double(a.M) * (a.N / 2) * es;                  // gated activation
  if (epi == E_QKV) b += double(a.M) * a.N * double(prec_bytes(att));   // q, k, v
  return b;
}

template <class T>
void h2d(nc_ctx* c, T* dst, const T* src, size_t n) {
  if (!n) return;
  void* p = pinned(c, n * sizeof(T));
  std::memcpy(p, src, n * sizeof(T));
  NC_HIP(hipMemcpyAsync(dst, p, n * sizeof(T), hipMemcpyHostToDevice, c->st));
  sync(c);
}

template <class T>
void d2h(nc_ctx* c, T* dst, const T* src, size_t n) {
  if (!n) return;
  void* p = pinned(c, n * sizeof(T));
  NC_HIP(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyDeviceToHost, c->st));
  sync(c);
  std::memcpy(dst, p, n * sizeof(T));
}

float host_amax(const float* w, size_t n) {
  float m = 0.f;
  for (size_t i = 0; i < n; ++i) m = std::max(m, std::fabs(w[i]));
  return m;
}

// Upload a float32 matrix and convert it to the GEMM precision on the device.
void* upload_weight(nc_ctx* c, const float* host, size_t n, float* scale_out, float** f32_out) {
  float* w32 = static_cast<float*>(dmalloc(c, n * 4));
  NC_HIP(hipMemcpy(w32, host, n * 4, hipMemcpyHostToDevice));
  if (f32_out) *f32_out = w32;
  if (c->prec == P_F32) {
    if (scale_out) *scale_out = 1.f;
    return w32;
  }
  float inv = 1.f;
  if (c->prec == P_FP8) {
    const float am = host_amax(host, n);
    const float sc = am > 0 ? am / 448.f : 1.f;
    if (scale_out) *scale_out = sc;
    inv = 1.f / sc;
  } else if (scale_out) {
    *scale_out = 1.f;
  }
  void* wp = dmalloc(c, n * prec_bytes(c->prec));
  launch_convert(w32, wp, (long long)n, c->prec, inv, c->st);
  sync(c);
  return wp;
}

void build_rope(nc_ctx* c, int max_pos) {
  if (max_pos <= c->rope_pos) return;
  const int h2 = c->hd / 2;
  std::vector<float> t((size_t)max_pos * h2 * 2);
  for (int p = 0; p < max_pos; ++p)
    for (int i = 0; i < h2; ++i) {
      // angle p * theta^(-2i/hd) in float64, rounded once to float32
      const double inv = std::pow((double)c->cfg.rope_theta, -2.0 * i / c->hd);
      const double a = (double)p * inv;
      t[((size_t)p * h2 + i) * 2 + 0] = (float)std::cos(a);
      t[((size_t)p * h2 + i) * 2 + 1] = (float)std::sin(a);
    }
  c->rope.alloc(t.size());
  NC_HIP(hipMemcpy(c->rope.p, t.data(), t.size() * 4, hipMemcpyHostToDevice));
  c->rope_pos = max_pos;
}

void ensure_rows(nc_ctx* c, int rows) {
  if (rows <= c->rows_alloc) return;
  const int r = std::max(rows, 64);
  c->x.alloc((size_t)r * c->d);
  c->xinv.alloc(r);
  c->xss.alloc((size_t)r * (c->d / 16));
  c->yb.alloc((size_t)r * c->d);  // sized for float32 (calibration pass)
  // sized for float32 so that the calibration pass (float32 GEMMs) fits in any precision
  c->qb.alloc((size_t)r * c->hq * c->hd * 4);
  c->ob.alloc((size_t)r * c->hq * c->hd * 4);
  c->hb.alloc((size_t)r * c->F * 4);
  c->rowsd.alloc(r);
  c->itemsd.alloc((size_t)r * c->hk + 64);
  c->rows_alloc = r;
}

void ensure_step(nc_ctx* c, int B) {
  const int nseg = int(ceil_div(c->V, kSeg));
  c->z.alloc((size_t)B * c->V);
  c->steprows.alloc(B);
  c->arows.alloc(B);
  c->targets.alloc(B);
  c->lsep.alloc((size_t)B * nseg);
  c->segp.alloc((size_t)B * nseg);
  c->ngp.alloc((size_t)B * nseg);
  c->outc.alloc(B);
  c->sout.alloc(B);
  if (B > c->sout_h_n) {
    if (c->sout_h) NC_HIP(hipHostFree(c->sout_h));
    c->sout_h = nullptr;
    c->sout_h_n = 0;
    NC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->sout_h), size_t(B) * sizeof(StepOut),
                         hipHostMallocMapped | hipHostMallocCoherent));
    NC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->sout_hd), c->sout_h, 0));
    c->sout_h_n = B;
  }
}

// ---- one transformer pass over a batch of rows --------------------------------------------

struct BodyOpts {
  bool calib = false;  // FP32 weights with amax recording (FP8 calibration)
  bool graph = false;  // replay a captured graph of the pass (decode and probe paths)
};

// Attention of a pass with fewer items runs the parallel quad + fold pair (decode), otherwise one
// wave per item (prefill); both give the same bits.
constexpr size_t kAttnParallelItems = 1024;
// Captured pass shapes kept per context (each a HIP graph of ~180 kernel nodes).
constexpr size_t kMaxGraphs = 512;

// Small per-step inputs gathered on the host and uploaded with one copy.
struct Stage {
  std::vector<uint8_t> h;
  size_t put(const void* p, size_t n) {
    const size_t off = (h.size() + 255) & ~size_t(255);
    h.resize(off + std::max<size_t>(n, 1));
    if (n) std::memcpy(h.data() + off, p, n);
    return off;
  }
};

// One transformer pass: rows (stream, position, token), attention items, and which rows are the
// newest of their stream (kept in hlast for the output layer).
struct PassPlan {
  std::vector<RowMeta> rows;
  std::vector<AttnItem> items;
  std::vector<int32_t> last;  // n_last source rows, then n_last destination streams
  double attn_bytes = 0, attn_flops = 0;
  bool shared_kv = false;     // some stream's kv head has several attention items
  size_t off_rows = 0, off_items = 0, off_last = 0;
};

PassPlan plan_pass(nc_ctx* c, std::vector<RowMeta> rows, bool calib = false) {
  PassPlan p;
  p.rows = std::move(rows);
  for (RowMeta& r : p.rows) r.slot = r.pos % c->R;
  const std::vector<RowMeta>& R = p.rows;
  const int n = int(R.size());
  const int g = c->hq / c->hk;
  const int L = c->cfg.ctx_len, C = c->cfg.slide;
  auto wstart = [&](int q) { return q < L ? 0 : C * (1 + (q - L) / C); };
  const double esa = double(prec_bytes(calib ? P_F32 : c->att));
  const double eso = double(prec_bytes(calib ? P_F32 : c->prec));
  std::vector<int32_t> src, dst;
  for (int i = 0; i < n;) {
    int j = i;
    while (j + 1 < n && R[j + 1].stream == R[i].stream && R[j + 1].pos == R[j].pos + 1) ++j;
    const int nq = j - i + 1;
    if (nq * g > 16) p.shared_kv = true;
    for (int kvh = 0; kvh < c->hk; ++kvh)
      for (int c0 = 0; c0 < nq * g; c0 += 16) {
        AttnItem it{};
        it.stream = R[i].stream;
        it.kvh = kvh;
        it.row_base = i;
        it.pos_base = R[i].pos;
        it.c0 = c0;
        it.ncols = std::min(16, nq * g - c0);
        p.items.push_back(it);
        for (int cc = 0; cc < it.ncols; ++cc) {
          const int q = it.pos_base + (it.c0 + cc) / g;
          p.attn_flops += 4.0 * double(q - wstart(q) + 1) * c->hd;
        }
      }
    // algorithmic bytes of the run: the union of its rows' windows, [s(first), last], read once
    // per kv head (K and V), the queries in and the outputs out
    p.attn_bytes += double(c->hk) * double(R[j].pos - wstart(R[i].pos) + 1) * c->hd * 2 * esa +
                    double(nq) * c->hq * c->hd * (esa + eso);
    src.push_back(j);
    dst.push_back(R[j].stream);
    i = j + 1;
  }
  p.last = src;
  p.last.insert(p.last.end(), dst.begin(), dst.end());
  return p;
}

void stage_pass(Stage& s, PassPlan& p) {
  p.off_rows = s.put(p.rows.data(), p.rows.size() * sizeof(RowMeta));
  p.off_items = s.put(p.items.data(), p.items.size() * sizeof(AttnItem));
  p.off_last = s.put(p.last.data(), p.last.size() * sizeof(int32_t));
}

// Upload the stage with one asynchronous copy; the step ends with a stream synchronisation
// before the staging memory is written again.
uint8_t* upload_stage(nc_ctx* c, const Stage& s) {
  sync(c);  // earlier work may still read the device stage or the pinned copy
  const size_t n = s.h.size();
  if (n > c->spin_bytes) {
    if (c->spin) NC_HIP(hipHostFree(c->spin));
    c->spin = nullptr;
    NC_HIP(hipHostMalloc(&c->spin, n * 2, hipHostMallocDefault));
    c->spin_bytes = n * 2;
  }
  c->dstage.alloc(std::max<size_t>(n, 256));
  if (n) {
    std::memcpy(c->spin, s.h.data(), n);
    NC_HIP(hipMemcpyAsync(c->dstage.p, c->spin, n, hipMemcpyHostToDevice, c->st));
  }
  return c->dstage.p;
}

// Newest rows of the streams: their output-layer operand rows (d elements of es bytes) and scales.
__global__ void copy_rows_kernel(const uint32_t* y, const float* yinv, const int32_t* src_rows,
                                 const int32_t* dst_rows, int n, int words, uint32_t* out,
                                 float* oinv) {
  const int r = blockIdx.x;
  if (r >= n) return;
  const long long s = src_rows[r], t = dst_rows[r];
  for (int k = threadIdx.x; k < words; k += blockDim.x) out[t * words + k] = y[s * words + k];
  if (threadIdx.x == 0) oinv[t] = yinv[s];
}

// Arguments of the five GEMMs of a pass over n rows (layer l; calib: the float32 calibration
// pass, which also records activation maxima in am).
static float op_inv_scale(int prec, float sc) { return prec == P_FP8 ? 1.0f / sc : 1.0f; }

static long long layer_kv_bytes(const nc_ctx* c) {
  return (long long)c->S_alloc * c->kv_stride * prec_bytes(c->att);
}

GemmArgs args_qkv(nc_ctx* c, int l, int n, const RowMeta* drows, bool calib) {
  Layer& L = c->layers[l];
  GemmArgs a{};
  a.M = n;
  a.N = (c->hq + 2 * c->hk) * c->hd;
  a.K = c->d;
  a.A = c->yb.p;
  a.eps = c->cfg.norm_eps;
  a.a_scale = L.sa_qkv;
  a.W = calib ? (void*)L.Wqkv32 : L.Wqkv;
  a.w_scale = calib ? 1.f : L.sw_qkv;
  a.rows = drows;
  a.rope = c->rope.p;
  a.q_out = c->qb.p;
  a.k_cache = c->kc.p + l * layer_kv_bytes(c);
  a.vt_cache = c->vc.p + l * layer_kv_bytes(c);
  a.kv_stride = c->kv_stride;
  a.Hq = c->hq;
  a.Hk = c->hk;
  a.hd = c->hd;
  a.ring = c->R;
  a.ssq = c->xss.p;
  return a;
}

GemmArgs args_oproj(nc_ctx* c, int l, int n, bool calib, float* am) {
  Layer& L = c->layers[l];
  const int prec = calib ? P_F32 : c->prec;
  GemmArgs ob{};
  ob.M = n;
  ob.N = c->d;
  ob.K = c->hq * c->hd;
  ob.A = c->ob.p;
  ob.a_scale = L.sa_o;
  ob.W = calib ? (void*)L.Wo32 : L.Wo;
  ob.w_scale = calib ? 1.f : L.sw_o;
  ob.out_f32 = c->x.p;
  ob.ldo = c->d;
  ob.ssq_out = c->xss.p;
  ob.y_out = c->yb.p;
  ob.y_gain = L.g_mlp;
  ob.y_inv_scale = op_inv_scale(prec, L.sa_gu);
  ob.y_amax = am ? am + 2 : nullptr;
  return ob;
}

GemmArgs args_gateup(nc_ctx* c, int l, int n, bool calib, float* am) {
  Layer& L = c->layers[l];
  GemmArgs gu{};
  gu.M = n;
  gu.N = 2 * c->F;
  gu.K = c->d;
  gu.A = c->yb.p;
  gu.eps = c->cfg.norm_eps;
  gu.a_scale = L.sa_gu;
  gu.W = calib ? (void*)L.Wgu32 : L.Wgu;
  gu.w_scale = calib ? 1.f : L.sw_gu;
  gu.out_p = c->hb.p;
  gu.out_scale = L.sa_d;
  gu.out_amax = am ? am + 3 : nullptr;
  gu.ssq = c->xss.p;
  return gu;
}

GemmArgs args_down(nc_ctx* c, int l, int n, bool calib) {
  Layer& L = c->layers[l];
  const int prec = calib ? P_F32 : c->prec;
  GemmArgs dn{};
  dn.M = n;
  dn.N = c->d;
  dn.K = c->F;
  dn.A = c->hb.p;
  dn.a_scale = L.sa_d;
  dn.W = calib ? (void*)L.Wd32 : L.Wd;
  dn.w_scale = calib ? 1.f : L.sw_d;
  dn.out_f32 = c->x.p;
  dn.ldo = c->d;
  dn.ssq_out = c->xss.p;
  // the next normed GEMM: the next layer's QKV, or the output layer
  const bool last = l + 1 == c->nl;
  dn.y_out = c->yb.p;
  dn.y_gain = last ? c->g_final : c->layers[l + 1].g_attn;
  dn.y_inv_scale = op_inv_scale(prec, last ? c->sa_lm : c->layers[l + 1].sa_qkv);
  dn.y_amax = calib ? c->amax.p + 4 * (l + 1) : nullptr;
  return dn;
}

// z[m] = final_norm(x) E^T for m < M, from the operand rows A[a_rows[m]] = quantise(x * g_final)
// and their RMSNorm scales Ainv[a_rows[m]].
GemmArgs args_lm(nc_ctx* c, const void* A, const float* Ainv, const int32_t* a_rows, int M,
                 float* zout, bool calib) {
  GemmArgs a{};
  a.M = M;
  a.N = c->V;
  a.K = c->d;
  a.A = A;
  a.a_rows = a_rows;
  a.eps = c->cfg.norm_eps;
  a.a_scale = c->sa_lm;
  a.W = calib ? (void*)c->E32 : c->Elm;
  a.w_scale = calib ? 1.f : c->sw_lm;
  a.out_f32 = zout;
  a.ldo = c->V;
  a.inv = Ainv;
  return a;
}

// Rows from which a pass's normed GEMMs take their RMSNorm scales from one row_rms launch: with
// many rows the tile kernels would otherwise each re-derive them from the block sums of squares
// of their rows (once per column tile), before their first K part.  The scales are the same bits.
constexpr int kRowScaleRows = 512;

// The RMSNorm scale of each of the pass's n rows into c->xinv (from the block sums in c->xss).
static void pass_row_scales(nc_ctx* c, int n) {
  GemmArgs r{};
  r.M = n;
  r.K = c->d;
  r.ssq = c->xss.p;
  r.eps = c->cfg.norm_eps;
  launch_row_rms(r, c->xinv.p, c->st);
}

// The kernels of one transformer pass (see run_pass).
void pass_launches(nc_ctx* c, const PassPlan& p, const uint8_t* dstage, BodyOpts o) {
  const int n = int(p.rows.size());
  const RowMeta* drows = reinterpret_cast<const RowMeta*>(dstage + p.off_rows);
  const AttnItem* ditems = reinterpret_cast<const AttnItem*>(dstage + p.off_items);
  const int prec = o.calib ? P_F32 : c->prec;
  const int att = o.calib ? P_F32 : c->att;
  launch_embed(c->E32, drows, n, c->d, c->x.p, c->xss.p, c->yb.p, c->layers[0].g_attn, prec,
               op_inv_scale(prec, c->layers[0].sa_qkv), o.calib ? c->amax.p : nullptr, c->st);
  for (int l = 0; l < c->nl; ++l) {
    Layer& L = c->layers[l];
    float* am = o.calib ? c->amax.p + 4 * l : nullptr;
    // QKV with RoPE and the KV-ring write
    GemmArgs a = args_qkv(c, l, n, drows, o.calib);
    prof_begin(c, NC_K_QKV);
    if (n >= kRowScaleRows) {
      pass_row_scales(c, n);
      a.inv = c->xinv.p;
    }
    launch_gemm(prec, A_NORM, E_QKV, a, c->st, tile_for(c, o.calib, NC_G_QKV, n));
    prof_end(c, NC_K_QKV, gemm_bytes(a, A_NORM, E_QKV, prec, att), 2.0 * a.M * a.N * a.K);
    // attention
    AttnArgs t{};
    t.items = ditems;
    t.n_items = int(p.items.size());
    t.q = c->qb.p;
    t.k_cache = a.k_cache;
    t.vt_cache = a.vt_cache;
    t.kv_stride = c->kv_stride;
    t.out = c->ob.p;
    t.out_scale = L.sa_o;
    t.out_amax = am ? am + 1 : nullptr;
    t.Hq = c->hq;
    t.Hk = c->hk;
    t.hd = c->hd;
    t.ring = c->R;
    t.ctx_len = c->cfg.ctx_len;
    t.slide = c->cfg.slide;
    t.scale_log2 = float(1.4426950408889634 / std::sqrt((double)c->hd));
    t.xcd_place = p.shared_kv ? 1 : 0;
    prof_begin(c, NC_K_ATTN);
    const bool par = p.items.size() < kAttnParallelItems;
    if (par) {
      t.ws = c->aws.p;
      t.ws_bytes = c->aws.n * 4;
      t.ctr = c->actr.p;
    }
    launch_attention(att, prec, t, par, c->st);
    prof_end(c, NC_K_ATTN, p.attn_bytes, p.attn_flops);
    // O projection + residual
    const GemmArgs ob = args_oproj(c, l, n, o.calib, am);
    prof_begin(c, NC_K_OPROJ);
    launch_gemm(prec, A_DIRECT, E_RESID, ob, c->st, tile_for(c, o.calib, NC_G_OPROJ, n));
    prof_end(c, NC_K_OPROJ, gemm_bytes(ob, A_DIRECT, E_RESID, prec, att), 2.0 * n * ob.N * ob.K);
    // gate/up with SiLU
    GemmArgs gu = args_gateup(c, l, n, o.calib, am);
    prof_begin(c, NC_K_GATEUP);
    if (n >= kRowScaleRows) {
      pass_row_scales(c, n);
      gu.inv = c->xinv.p;
    }
    launch_gemm(prec, A_NORM, E_GLU, gu, c->st, tile_for(c, o.calib, NC_G_GATEUP, n));
    prof_end(c, NC_K_GATEUP, gemm_bytes(gu, A_NORM, E_GLU, prec, att), 2.0 * n * gu.N * gu.K);
    // down projection + residual
    const GemmArgs dn = args_down(c, l, n, o.calib);
    prof_begin(c, NC_K_DOWN);
    launch_gemm(prec, A_DIRECT, E_RESID, dn, c->st, tile_for(c, o.calib, NC_G_DOWN, n));
    prof_end(c, NC_K_DOWN, gemm_bytes(dn, A_DIRECT, E_RESID, prec, att), 2.0 * n * dn.N * dn.K);
  }
  const int nl = int(p.last.size() / 2);
  const int32_t* dl = reinterpret_cast<const int32_t*>(dstage + p.off_last);
  // RMSNorm scale of every final row, for the output layer (same arithmetic as the GEMMs)
  pass_row_scales(c, n);
  const int words = c->d * prec_bytes(prec) / 4;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(nl), dim3(256), 0, c->st,
                     reinterpret_cast<const uint32_t*>(c->yb.p), c->xinv.p, dl, dl + nl, nl, words,
                     reinterpret_cast<uint32_t*>(c->hlast.p), c->hinv.p);
  NC_HIP(hipGetLastError());
}

bool profiling(const nc_ctx* c) {
  for (const auto& P : c->prof)
    if (P.on) return true;
  return false;
}

void graphs_clear(nc_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
  for (auto& g : c->egraphs) (void)hipGraphExecDestroy(g.second);
  c->egraphs.clear();
}

// Appends a planned pass to the KV caches; leaves each row's final residual in x, its
// output-layer operand in yb, and each stream's newest operand row in hlast.  Rows of one stream
// are consecutive positions spanning fewer than `slide` positions (the ring holds at least
// ctx_len + slide entries, so no needed key is overwritten).  With o.graph the pass's ~6 kernels
// per layer are captured into a HIP graph on the first use of its shape (rows, attention items,
// stage offsets and buffers) and replayed afterwards: one launch instead of ~180.  A replay runs
// the same kernels with the same arguments, so the bits are those of the direct launches.
void run_pass(nc_ctx* c, const PassPlan& p, const uint8_t* dstage, BodyOpts o = {}) {
  const int n = int(p.rows.size());
  if (!n) return;
  ensure_rows(c, n);
  if (p.items.size() < kAttnParallelItems)
    c->aws.alloc(attention_ws_bytes(int(p.items.size())) / 4);
  c->stats.body_rows += n;
  if (!o.graph || o.calib || (c->cfg.features & NC_F_EAGER) ||
      !(c->cfg.features & NC_F_DECODE_GRAPHS) || profiling(c)) {
    pass_launches(c, p, dstage, o);
    return;
  }
  nc_ctx::GraphKey k{n,          int(p.items.size()), int(p.last.size()),
                     p.off_rows, p.off_items,         p.off_last,
                     {dstage, c->x.p, c->xinv.p, c->xss.p, c->yb.p, c->qb.p, c->ob.p, c->hb.p,
                      c->aws.p, c->kc.p, c->hlast.p, c->hinv.p}};
  auto it = c->graphs.find(k);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= kMaxGraphs) graphs_clear(c);
    hipGraph_t g = nullptr;
    NC_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    try {
      pass_launches(c, p, dstage, o);
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(c->st, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      throw;
    }
    NC_HIP(hipStreamEndCapture(c->st, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NC_HIP(e);
    it = c->graphs.emplace(k, ex).first;
    c->stats.graph_captures += 1;
  }
  NC_HIP(hipGraphLaunch(it->second, c->st));
  c->stats.graph_replays += 1;
}

void run_lm_head(nc_ctx* c, const void* A, const float* Ainv, const int32_t* a_rows, int M,
                 float* zout, bool calib = false) {
  const GemmArgs a = args_lm(c, A, Ainv, a_rows, M, zout, calib);
  const int prec = calib ? P_F32 : c->prec;
  prof_begin(c, NC_K_LMHEAD);
  launch_gemm(prec, A_NORM, E_STORE, a, c->st, tile_for(c, calib, NC_G_LMHEAD, M));
  prof_end(c, NC_K_LMHEAD, gemm_bytes(a, A_NORM, E_STORE, prec, c->att), 2.0 * M * a.N * a.K);
}

// Plan the appends of x positions [appended[s], upto] of each listed stream, in passes of at most
// `slide` positions per stream; the last pass holds every stream's newest position.
std::vector<PassPlan> plan_catch_up(nc_ctx* c, const std::vector<int>& streams,
                                    const std::vector<int>& upto) {
  const int C = c->cfg.slide;
  int npass = 0;
  std::vector<int> nch(streams.size());
  for (size_t k = 0; k < streams.size(); ++k) {
    const int pend = upto[k] - c->appended[streams[k]] + 1;
    nch[k] = pend > 0 ? (pend + C - 1) / C : 0;
    npass = std::max(npass, nch[k]);
  }
  std::vector<PassPlan> plans;
  for (int pi = 0; pi < npass; ++pi) {
    std::vector<RowMeta> rows;
    for (size_t k = 0; k < streams.size(); ++k) {
      const int s = streams[k];
      const int ci = pi - (npass - nch[k]);
      if (ci < 0) continue;
      const int a = c->appended[s] + ci * C;
      const int e = std::min(upto[k], a + C - 1);
      for (int j = a; j <= e; ++j)
        rows.push_back(RowMeta{s, j, j == 0 ? kBOS : c->hhist[s][j - 1], 0});
    }
    plans.push_back(plan_pass(c, std::move(rows)));
  }
  for (size_t k = 0; k < streams.size(); ++k)
    c->appended[streams[k]] = std::max(c->appended[streams[k]], upto[k] + 1);
  return plans;
}

// Single-stream catch-up (probe and commit calls): plan, upload, run.
void catch_up_now(nc_ctx* c, int s, int upto) {
  std::vector<PassPlan> plans = plan_catch_up(c, {s}, {upto});
  if (plans.empty()) return;
  Stage st;
  for (auto& p : plans) stage_pass(st, p);
  const uint8_t* d = upload_stage(c, st);
  BodyOpts o;
  o.graph = true;
  for (auto& p : plans) run_pass(c, p, d, o);
  sync(c);
}

StreamState make_state(nc_ctx* c) {
  StreamState S{};
  S.V = c->V;
  S.K = c->cfg.ngram_order;
  S.maxT = c->T_alloc;
  S.cap = c->S.cap;
  S.maxctx = c->S.maxctx;
  S.b = c->b.p;
  S.uni = c->uni.p;
  S.nseen = c->nseen.p;
  S.hist = c->hist.p;
  S.ncommit = c->ncommit.p;
  S.png = c->png.p;
  S.pk = (c->cfg.features & NC_F_ENSEMBLE) ? c->pk.p : nullptr;
  S.lw = c->lw.p;
  S.mode = c->moded.p;
  S.H = c->Hd.p;
  S.pmax = c->pmaxd.p;
  S.next_ctx = c->next_ctx.p;
  S.keys = c->keys.p;
  S.kidx = c->kidx.p;
  S.pool = c->pool.p;
  S.pool_n = c->pool_n.p;
  S.pool_sum = c->pool_sum.p;
  S.nctx = c->nctx.p;
  return S;
}

// The state with the n-gram distribution and mode of parity p (the pipelined encode alternates
// them by position; every other path uses parity 0).
StreamState state_par(nc_ctx* c, int p) {
  StreamState S = c->S;
  S.png = c->png.p + (size_t)p * c->S_alloc * c->V;
  S.mode = c->moded.p + (size_t)p * c->S_alloc;
  return S;
}

bool ngram_on(const nc_ctx* c) {
  return (c->cfg.features & (NC_F_NGRAM | NC_F_ENSEMBLE)) != 0;
}

// The stream of each step row.
void set_steprows(nc_ctx* c, const int32_t* rows, size_t n) { h2d(c, c->steprows.p, rows, n); }

void reset_streams(nc_ctx* c, int n, int maxT) {
  NC_CHECK(n >= 1 && n <= c->cfg.max_streams, NC_E_INVALID, "n_streams must be in [1, %d]",
           c->cfg.max_streams);
  NC_CHECK(maxT >= 1, NC_E_INVALID, "max_tokens must be >= 1");
  const int K = c->cfg.ngram_order;
  const int V = c->V;
  if (n > c->S_alloc || maxT > c->T_alloc) {
    const int Sa = std::max(n, c->S_alloc), Ta = std::max(maxT, c->T_alloc);
    int cap = 1;
    while (cap < 2 * (Ta + 1)) cap <<= 1;
    const int maxctx = std::min(Ta, c->cfg.ngram_max_contexts);
    c->b.alloc((size_t)Sa * V);
    c->png.alloc((size_t)2 * Sa * V);  // two parities (pipelined encode), parity 0 otherwise
    if (c->cfg.features & NC_F_ENSEMBLE) c->pk.alloc((size_t)Sa * K * V);
    c->lw.alloc((size_t)Sa * kMaxExperts);
    c->Hd.alloc(Sa);
    c->pmaxd.alloc(Sa);
    c->hlast.alloc((size_t)Sa * c->d);
    c->hinv.alloc(Sa);
    c->uni.alloc((size_t)Sa * V);
    c->nseen.alloc(Sa);
    c->hist.alloc((size_t)Sa * Ta);
    c->ncommit.alloc(Sa);
    c->moded.alloc((size_t)2 * Sa);
    c->next_ctx.alloc((size_t)Sa * kMaxOrder);
    c->nctx.alloc((size_t)Sa * K);
    if (ngram_on(c)) {
      c->keys.alloc((size_t)Sa * K * cap * 4);
      c->kidx.alloc((size_t)Sa * K * cap);
      c->pool.alloc((size_t)Sa * K * maxctx * kSlots * 2);
      c->pool_n.alloc((size_t)Sa * K * maxctx);
      c->pool_sum.alloc((size_t)Sa * K * maxctx);
    }
    c->kv_stride = (long long)c->hk * c->R * c->hd;
    c->kc.release();
    c->vc.release();
    const size_t kvb = (size_t)c->nl * Sa * c->kv_stride * prec_bytes(c->att);
    c->kc.alloc(kvb);
    c->vc.alloc(kvb);
    c->iv.alloc((size_t)Sa * Ta * 2);
    c->ptok.alloc((size_t)Sa * Ta);
    c->S_alloc = Sa;
    c->T_alloc = Ta;
    c->S.cap = cap;
    c->S.maxctx = std::max(1, maxctx);
    build_rope(c, Ta + 2);
  }
  c->n_streams = n;
  c->maxT = maxT;
  c->S = make_state(c);
  if (ngram_on(c)) NC_HIP(hipMemsetAsync(c->kidx.p, 0xFF, c->kidx.n * 4, c->st));
  NC_HIP(hipMemsetAsync(c->kc.p, 0, c->kc.n, c->st));
  NC_HIP(hipMemsetAsync(c->vc.p, 0, c->vc.n, c->st));
  NC_HIP(hipMemsetAsync(c->hlast.p, 0, c->hlast.n * 4, c->st));
  NC_HIP(hipMemsetAsync(c->hinv.p, 0, c->hinv.n * 4, c->st));
  launch_state_reset(c->vp, c->S, c->S_alloc, c->cfg.mix_w_llm, c->st);
  ensure_step(c, std::max(n, 1));
  if (ngram_on(c)) {
    std::vector<int32_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0);
    set_steprows(c, ids.data(), ids.size());
    launch_ngram_predict(c->vp, c->S, c->steprows.p, n, c->ngp.p, nullptr, nullptr, c->st);
  }
  sync(c);
  c->hhist.assign(n, {});
  c->appended.assign(n, 0);
}

StepArgs step_args(nc_ctx* c, int B, bool decode) {
  StepArgs A{};
  A.B = B;
  A.rows = c->steprows.p;
  A.z = c->z.p;
  A.decode = decode ? 1 : 0;
  A.targets = c->targets.p;
  A.lse_parts = c->lsep.p;
  A.seg_parts = c->segp.p;
  A.ng_parts = c->ngp.p;
  A.out = c->outc.p;
  A.step_out = c->sout.p;
  A.pos = -1;
  A.upd = kUpdCounts | kUpdMixer;
  A.lse = 1;
  return A;
}

// One coding step for rows steprows[0..B): updates and next-position prediction included.
void vocab_commit_step(nc_ctx* c, const StepArgs& A) {
  // per row: z and b read by the logsumexp, count and scan passes, p_ng by two, b written
  const double V = c->V;
  prof_begin(c, NC_K_VOCAB);
  launch_vocab_step(c->vp, c->S, A, c->st);
  prof_end(c, NC_K_VOCAB, A.B * V * 4.0 * (2 + 2 + 2 + 2 + 1), A.B * V * 12.0);
  if (ngram_on(c)) {
    prof_begin(c, NC_K_NGRAM);
    launch_ngram_predict(c->vp, c->S, A.rows, A.B, c->ngp.p, A.decode ? A.step_out : nullptr,
                         A.out, c->st);
    prof_end(c, NC_K_NGRAM, A.B * V * 4.0 * 2, A.B * V * 8.0);
  }
}

// One position of the batched encode, every row at position pos, in two streams:
//   st:  the distribution of pos (n-gram parity pos % 2), its interval and bias step, and the
//        mixer update, which needs the step's outcome;
//   st2: the count updates with the known token t_pos, then the n-gram prediction of pos + 1
//        into the other parity, which the distribution of pos - 1 was the last to read.
// st waits for the prediction of pos (ev_pred); st2 waits for the distribution of pos - 1
// (ev_dist of its parity; at pos 0 for everything st has queued).  Every kernel computes what the
// sequential step computes, so the coded bytes are the same.
// kpos >= 0: the kernels see position kpos + *A.pos_base (a step captured into a graph); the
// first step of a capture forks st2 from st inside the capture, and its predecessors are complete
// before the graph starts.
void encode_step_pipelined(nc_ctx* c, StepArgs A, int pos, int kpos = -1,
                           bool capture_first = false) {
  const double V = c->V;
  const int par = pos & 1;
  const StreamState Sp = state_par(c, par), Sn = state_par(c, par ^ 1);
  A.pos = kpos >= 0 ? kpos : pos;
  if (pos > 0 && !capture_first) NC_HIP(hipStreamWaitEvent(c->st, c->ev_pred, 0));
  prof_begin(c, NC_K_VOCAB);
  launch_vocab_dist(c->vp, Sp, A, c->st);
  A.upd = kUpdMixer;
  launch_ngram_update(c->vp, Sp, A, c->st);
  prof_end(c, NC_K_VOCAB, A.B * V * 4.0 * (2 + 2 + 2 + 2 + 1), A.B * V * 12.0);
  NC_HIP(hipEventRecord(c->ev_dist[par], c->st));
  NC_HIP(hipStreamWaitEvent(c->st2, c->ev_dist[(pos > 0 && !capture_first) ? par ^ 1 : par], 0));
  A.upd = kUpdCounts;
  launch_ngram_update(c->vp, Sn, A, c->st2);
  prof_begin(c, NC_K_NGRAM, c->st2);
  launch_ngram_predict(c->vp, Sn, A.rows, A.B, c->ngp.p, nullptr, nullptr, c->st2, A.pos + 1,
                       A.pos_base);
  prof_end(c, NC_K_NGRAM, A.B * V * 4.0 * 2, A.B * V * 8.0, c->st2);
  NC_HIP(hipEventRecord(c->ev_pred, c->st2));
}

// Positions p0 .. p0 + np - 1 of the pipelined encode (B rows each, logits in zseg rows
// (i - p0) * B), captured on the first use of the shape and replayed afterwards: one launch
// instead of about ten launches and event calls per position.  p0 is even, so the parity
// buffers alternate as in the direct path; the kernels compute exactly what they compute there.
void encode_chunk_graph(nc_ctx* c, int p0, int np, int B) {
  c->posbase.alloc(1);
  const StreamState S = c->S;
  std::vector<const void*> key{reinterpret_cast<const void*>(size_t(np)),
                               reinterpret_cast<const void*>(size_t(B)),
                               reinterpret_cast<const void*>(size_t(c->n_streams)),
                               c->zseg.p, c->iv.p, c->ptok.p, c->steprows.p, c->lsep.p, c->segp.p,
                               c->ngp.p, c->outc.p, c->posbase.p, S.b, S.png, S.uni, S.hist,
                               S.pool, S.keys, S.lw, S.mode,
                               reinterpret_cast<const void*>(size_t(c->S_alloc)),
                               reinterpret_cast<const void*>(size_t(c->T_alloc)),
                               reinterpret_cast<const void*>(size_t(S.cap)),
                               reinterpret_cast<const void*>(size_t(S.maxctx))};
  // everything queued before the chunk, on both streams, precedes the replay
  NC_HIP(hipStreamWaitEvent(c->st, c->ev_pred, 0));
  launch_set_int(c->posbase.p, p0, c->st);
  auto it = c->egraphs.find(key);
  if (it == c->egraphs.end()) {
    if (c->egraphs.size() >= 64) {
      for (auto& g : c->egraphs) (void)hipGraphExecDestroy(g.second);
      c->egraphs.clear();
    }
    hipGraph_t g = nullptr;
    NC_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < np; ++k) {
        StepArgs A = step_args(c, B, false);
        A.z = c->zseg.p + size_t(k) * c->n_streams * size_t(c->V);
        A.step_out = nullptr;
        A.iv = c->iv.p;
        A.ptok = c->ptok.p;
        A.pos_base = c->posbase.p;
        encode_step_pipelined(c, A, p0 + k, k, k == 0);
      }
      NC_HIP(hipStreamWaitEvent(c->st, c->ev_pred, 0));  // st2 joins the capture
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(c->st, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      throw;
    }
    NC_HIP(hipStreamEndCapture(c->st, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NC_HIP(e);
    it = c->egraphs.emplace(key, ex).first;
    c->stats.graph_captures += 1;
  }
  NC_HIP(hipGraphLaunch(it->second, c->st));
  c->stats.graph_replays += 1;
  // Events recorded inside a capture order the graph's own nodes only; a later direct step waits
  // on these (the chunk's last distribution and prediction), so they are recorded again after
  // the whole replay.
  NC_HIP(hipEventRecord(c->ev_pred, c->st));
  NC_HIP(hipEventRecord(c->ev_dist[0], c->st));
  NC_HIP(hipEventRecord(c->ev_dist[1], c->st));
}

void check_config(const nc_config* cfg) {
  NC_CHECK(cfg, NC_E_INVALID, "NULL config");
  NC_CHECK(cfg->n_layers >= 0 && cfg->d_model > 0 && cfg->d_model % 16 == 0, NC_E_INVALID,
           "d_model must be a positive multiple of 16");
  NC_CHECK(cfg->n_heads > 0 && cfg->n_kv_heads > 0 && cfg->n_heads % cfg->n_kv_heads == 0,
           NC_E_INVALID, "n_heads must be a multiple of n_kv_heads");
  NC_CHECK(cfg->head_dim >= 16 && cfg->head_dim <= 64 && 64 % cfg->head_dim == 0, NC_E_INVALID,
           "head_dim must be 16, 32 or 64");
  NC_CHECK(cfg->d_ffn > 0 && cfg->d_ffn % 16 == 0, NC_E_INVALID, "d_ffn must be a multiple of 16");
  NC_CHECK(cfg->vocab >= 4 && cfg->vocab <= 262144 && cfg->vocab % 4 == 0, NC_E_INVALID,
           "vocab must be a multiple of 4 in [4, 262144]");
  NC_CHECK(cfg->cdf_total > (uint32_t)cfg->vocab && cfg->cdf_total <= (1u << 24), NC_E_INVALID,
           "cdf_total must satisfy vocab < total <= 2^24");
  NC_CHECK(cfg->slide > 0 && cfg->ctx_len >= cfg->slide && cfg->ctx_len % cfg->slide == 0 &&
               (cfg->ctx_len + cfg->slide) % 16 == 0 && cfg->ctx_len + cfg->slide <= 2816,
           NC_E_INVALID, "ctx_len must be a multiple of slide with ctx_len + slide <= 2816");
  NC_CHECK(cfg->ngram_order >= 1 && cfg->ngram_order <= kMaxOrder, NC_E_INVALID,
           "ngram_order must be in [1, 4]");
  NC_CHECK(cfg->precision >= NC_FP32 && cfg->precision <= NC_FP8, NC_E_INVALID, "bad precision");
  NC_CHECK(cfg->max_streams >= 1, NC_E_INVALID, "max_streams must be >= 1");
  NC_CHECK(cfg->mix_w_llm > 0.f && cfg->mix_w_llm < 1.f, NC_E_INVALID, "mix_w_llm in (0, 1)");
  NC_CHECK(cfg->ngram_eps > 0.f, NC_E_INVALID, "ngram_eps must be positive");
  NC_CHECK(cfg->ngram_max_contexts >= 1, NC_E_INVALID, "ngram_max_contexts must be >= 1");
}

void validate_tokens(const nc_ctx* c, const int32_t* t, size_t n) {
  for (size_t i = 0; i < n; ++i)
    NC_CHECK(t[i] >= 0 && t[i] < c->V, NC_E_INVALID, "token %zu (%d) outside [0, %d)", i, t[i],
             c->V);
}

}  // namespace

// ---- C ABI ------------------------------------------------------------------------------------

extern "C" {

nc_status nc_create(const nc_config* cfg, const float* w, nc_ctx** out) {
  return guard([&] {
    NC_CHECK(out, NC_E_INVALID, "NULL out");
    *out = nullptr;
    check_config(cfg);
    NC_CHECK(w, NC_E_INVALID, "NULL weights");
    auto c = std::make_unique<nc_ctx>();
    c->cfg = *cfg;
    NC_HIP(hipGetDevice(&c->dev));
    NC_HIP(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
    NC_HIP(hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking));
    for (hipEvent_t* e : {&c->ev_dist[0], &c->ev_dist[1], &c->ev_pred})
      NC_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    // the attention chunk counters start at zero; every launch leaves them at zero
    c->actr.alloc(attention_counters(int(kAttnParallelItems)));
    NC_HIP(hipMemsetAsync(c->actr.p, 0, c->actr.n * sizeof(int32_t), c->st));
    NC_HIP(hipStreamSynchronize(c->st));
    c->prec = cfg->precision == NC_FP32 ? P_F32 : cfg->precision == NC_BF16 ? P_BF16 : P_FP8;
    c->att = c->prec == P_F32 ? P_F32 : P_BF16;
    c->d = cfg->d_model;
    c->hq = cfg->n_heads;
    c->hk = cfg->n_kv_heads;
    c->hd = cfg->head_dim;
    c->F = cfg->d_ffn;
    c->V = cfg->vocab;
    c->nl = cfg->n_layers;
    c->R = cfg->ctx_len + cfg->slide;  // ring: any batch spanning < slide positions is safe
    const size_t d = c->d, nqkv = (size_t)(c->hq + 2 * c->hk) * c->hd, F = c->F;
    // flat layout: E, per layer (attn_norm, Wq, Wk, Wv, Wo, mlp_norm, Wg, Wu, Wd), final_norm
    const float* p = w;
    c->E32 = static_cast<float*>(dmalloc(c.get(), (size_t)c->V * d * 4));
    NC_HIP(hipMemcpy(c->E32, p, (size_t)c->V * d * 4, hipMemcpyHostToDevice));
    if (c->prec == P_F32) {
      c->Elm = c->E32;
    } else {
      float* tmp = nullptr;
      c->Elm = upload_weight(c.get(), p, (size_t)c->V * d, &c->sw_lm, &tmp);
    }
    p += (size_t)c->V * d;
    std::vector<float> gu((size_t)2 * F * d);
    for (int l = 0; l < c->nl; ++l) {
      Layer L;
      L.g_attn = static_cast<float*>(dmalloc(c.get(), d * 4));
      NC_HIP(hipMemcpy(L.g_attn, p, d * 4, hipMemcpyHostToDevice));
      p += d;
      L.Wqkv = upload_weight(c.get(), p, nqkv * d, &L.sw_qkv, &L.Wqkv32);  // Wq, Wk, Wv adjacent
      p += nqkv * d;
      L.Wo = upload_weight(c.get(), p, d * c->hq * c->hd, &L.sw_o, &L.Wo32);
      p += d * c->hq * c->hd;
      L.g_mlp = static_cast<float*>(dmalloc(c.get(), d * 4));
      NC_HIP(hipMemcpy(L.g_mlp, p, d * 4, hipMemcpyHostToDevice));
      p += d;
      // interleave gate and up rows in 16-row groups for the fused SiLU epilogue
      const float* Wg = p;
      const float* Wu = p + F * d;
      for (size_t blk = 0; blk < F / 16; ++blk)
        for (size_t r = 0; r < 16; ++r) {
          std::memcpy(&gu[((2 * blk) * 16 + r) * d], Wg + (blk * 16 + r) * d, d * 4);
          std::memcpy(&gu[((2 * blk + 1) * 16 + r) * d], Wu + (blk * 16 + r) * d, d * 4);
        }
      L.Wgu = upload_weight(c.get(), gu.data(), 2 * F * d, &L.sw_gu, &L.Wgu32);
      p += 2 * F * d;
      L.Wd = upload_weight(c.get(), p, d * F, &L.sw_d, &L.Wd32);
      p += d * F;
      c->layers.push_back(L);
    }
    c->g_final = static_cast<float*>(dmalloc(c.get(), d * 4));
    NC_HIP(hipMemcpy(c->g_final, p, d * 4, hipMemcpyHostToDevice));
    c->amax.alloc(4 * c->nl + 1);

    c->fp8_ready = c->prec != P_FP8;
    VocabParams& P = c->vp;
    P.V = c->V;
    P.total = cfg->cdf_total;
    P.use_head = (cfg->features & NC_F_HEAD) ? 1 : 0;
    P.use_ngram = (cfg->features & NC_F_NGRAM) ? 1 : 0;
    P.use_skip = (cfg->features & NC_F_SKIP) && cfg->skip_mode != NC_SKIP_NONE ? 1 : 0;
    P.use_mixer = (cfg->features & NC_F_MIXER) ? 1 : 0;
    P.ensemble = (cfg->features & NC_F_ENSEMBLE) ? 1 : 0;
    if (P.ensemble) P.use_head = 1;
    P.K = cfg->ngram_order;
    P.head_lr = cfg->head_lr;
    P.mix_eta = cfg->mix_eta;
    P.ngram_eps = cfg->ngram_eps;
    P.ngram_max_contexts = cfg->ngram_max_contexts;
    P.warmup = cfg->warmup;
    P.skip_mode = cfg->skip_mode;
    P.skip_bits = cfg->skip_entropy_bits;
    P.skip_pmax = cfg->skip_pmax;
    sync(c.get());
    *out = c.release();
  });
}

void nc_destroy(nc_ctx* c) { delete c; }

nc_status nc_streams_reset(nc_ctx* c, uint32_t n, uint32_t maxT) {
  return guard([&] {
    NC_CHECK(c, NC_E_INVALID, "NULL context");
    NC_HIP(hipSetDevice(c->dev));
    reset_streams(c, int(n), int(maxT));
  });
}

nc_status nc_calibrate_fp8(nc_ctx* c, const int32_t* tokens, size_t n) {
  return guard([&] {
    NC_CHECK(c && tokens && n > 0, NC_E_INVALID, "bad arguments");
    NC_CHECK(c->prec == P_FP8, NC_E_STATE, "context is not FP8");
    NC_HIP(hipSetDevice(c->dev));
    validate_tokens(c, tokens, n);
    reset_streams(c, 1, int(n) + 1);
    NC_HIP(hipMemsetAsync(c->amax.p, 0, c->amax.n * 4, c->st));
    // FP32 passes over x_0..x_{n-1} (BOS, t_0, ..) recording every GEMM input's |max|
    const auto att_save = c->att;
    c->att = P_F32;
    // the FP32 pass needs float32 KV caches: use a temporary allocation
    DevBuf<uint8_t> k32, v32;
    const size_t kvb = (size_t)c->nl * c->S_alloc * c->kv_stride * 4;
    k32.alloc(kvb);
    v32.alloc(kvb);
    NC_HIP(hipMemsetAsync(k32.p, 0, kvb, c->st));
    NC_HIP(hipMemsetAsync(v32.p, 0, kvb, c->st));
    std::swap(c->kc, k32);
    std::swap(c->vc, v32);
    try {
      const int C = c->cfg.slide;
      for (size_t a = 0; a < n; a += C) {
        std::vector<RowMeta> rows;
        for (size_t j = a; j < std::min(n, a + C); ++j)
          rows.push_back(RowMeta{0, int(j), j == 0 ? kBOS : tokens[j - 1], 0});
        BodyOpts o;
        o.calib = true;
        PassPlan p = plan_pass(c, std::move(rows), true);
        std::vector<int32_t> idx(p.rows.size());
        std::iota(idx.begin(), idx.end(), 0);
        Stage stg;
        stage_pass(stg, p);
        const size_t off_ar = stg.put(idx.data(), idx.size() * 4);
        const uint8_t* d = upload_stage(c, stg);
        run_pass(c, p, d, o);
        DevBuf<float> zt;
        zt.alloc(p.rows.size() * (size_t)c->V);
        run_lm_head(c, c->yb.p, c->xinv.p, reinterpret_cast<const int32_t*>(d + off_ar), int(p.rows.size()),
                    zt.p, true);
        sync(c);
        zt.release();
      }
    } catch (...) {
      std::swap(c->kc, k32);
      std::swap(c->vc, v32);
      k32.release();
      v32.release();
      c->att = att_save;
      throw;
    }
    std::swap(c->kc, k32);
    std::swap(c->vc, v32);
    k32.release();
    v32.release();
    c->att = att_save;
    std::vector<float> am(c->amax.n);
    d2h(c, am.data(), c->amax.p, am.size());
    auto sc = [](float m) { return m > 0 ? m / 448.f : 1.f; };
    for (int l = 0; l < c->nl; ++l) {
      c->layers[l].sa_qkv = sc(am[4 * l + 0]);
      c->layers[l].sa_o = sc(am[4 * l + 1]);
      c->layers[l].sa_gu = sc(am[4 * l + 2]);
      c->layers[l].sa_d = sc(am[4 * l + 3]);
    }
    c->sa_lm = sc(am[4 * c->nl]);
    c->fp8_ready = true;
    graphs_clear(c);  // captured passes carry the activation scales as kernel arguments
    reset_streams(c, 1, int(n) + 1);
  });
}

nc_status nc_probs_for_context(nc_ctx* c, uint32_t s, const int32_t* tokens, size_t n,
                               float* probs, nc_probe* probe) {
  return guard([&] {
    NC_CHECK(c && probs && (n == 0 || tokens), NC_E_INVALID, "bad arguments");
    NC_HIP(hipSetDevice(c->dev));
    NC_CHECK(c->fp8_ready, NC_E_STATE, "FP8 context needs nc_calibrate_fp8 first");
    NC_CHECK(int(s) < c->n_streams, NC_E_STATE, "stream %u not reset (call nc_streams_reset)", s);
    NC_CHECK(int(n) < c->maxT, NC_E_STATE, "history longer than the reset max_tokens");
    validate_tokens(c, tokens, n);
    auto& h = c->hhist[s];
    NC_CHECK(n >= h.size(), NC_E_STATE, "history is shorter than the committed tokens");
    for (size_t i = 0; i < h.size(); ++i)
      NC_CHECK(tokens[i] == h[i], NC_E_STATE, "history differs from the committed tokens at %zu",
               i);
    const int32_t sid = int32_t(s);
    set_steprows(c, &sid, 1);
    // commit the new tokens one by one, exactly as the encoder does
    for (size_t j = h.size(); j < n; ++j) {
      NC_HIP(hipMemcpyAsync(c->hist.p + (size_t)s * c->T_alloc + j, tokens + j, 4,
                            hipMemcpyHostToDevice, c->st));
      catch_up_now(c, int(s), int(j));
      run_lm_head(c, c->hlast.p, c->hinv.p, c->steprows.p, 1, c->z.p);
      StepArgs A = step_args(c, 1, false);
      A.step_out = nullptr;
      vocab_commit_step(c, A);
      h.push_back(tokens[j]);
    }
    // distribution of position n
    catch_up_now(c, int(s), int(n));
    run_lm_head(c, c->hlast.p, c->hinv.p, c->steprows.p, 1, c->z.p);
    c->dbgp.alloc(c->V);
    c->dbgpt.alloc(c->V);
    c->dbgcdf.alloc(c->V + 1);
    StepArgs A = step_args(c, 1, true);
    A.no_update = 1;
    A.step_out = nullptr;
    const uint32_t zero = 0;
    h2d(c, c->targets.p, &zero, 1);
    A.dbg_p = c->dbgp.p;
    A.dbg_pt = c->dbgpt.p;
    A.dbg_cdf = c->dbgcdf.p;
    launch_vocab_step(c->vp, c->S, A, c->st);  // probe: no state update is launched
    sync(c);
    d2h(c, probs, c->dbgp.p, c->V);
    if (probe) {
      int32_t mode = 0;
      d2h(c, &mode, c->moded.p + s, 1);
      probe->mode = mode;
      probe->llm_ran = mode != M_SKIP;
      float hv = 0, pm = 0, lw[2] = {0, 0};
      d2h(c, &hv, c->Hd.p + s, 1);
      d2h(c, &pm, c->pmaxd.p + s, 1);
      d2h(c, lw, c->lw.p + (size_t)s * kMaxExperts, 2);
      probe->entropy_bits = hv;
      probe->pmax = pm;
      probe->mix_w[0] = std::exp(lw[0]);
      probe->mix_w[1] = std::exp(lw[1]);
      if (probe->logits) d2h(c, probe->logits, c->z.p, c->V);
      if (probe->ptilde) d2h(c, probe->ptilde, c->dbgpt.p, c->V);
      if (probe->p_ngram) d2h(c, probe->p_ngram, c->png.p + (size_t)s * c->V, c->V);
      if (probe->cdf) d2h(c, probe->cdf, c->dbgcdf.p, c->V + 1);
    }
  });
}

nc_status nc_mix_update(nc_ctx* c, uint32_t s, int32_t token) {
  return guard([&] {
    NC_CHECK(c, NC_E_INVALID, "NULL context");
    NC_HIP(hipSetDevice(c->dev));
    NC_CHECK(int(s) < c->n_streams, NC_E_STATE, "stream %u not reset", s);
    validate_tokens(c, &token, 1);
    auto& h = c->hhist[s];
    const size_t j = h.size();
    NC_CHECK(int(j) + 1 < c->maxT, NC_E_STATE, "stream is full (max_tokens reached)");
    const int32_t sid = int32_t(s);
    set_steprows(c, &sid, 1);
    NC_HIP(hipMemcpyAsync(c->hist.p + (size_t)s * c->T_alloc + j, &token, 4,
                          hipMemcpyHostToDevice, c->st));
    catch_up_now(c, int(s), int(j));
    run_lm_head(c, c->hlast.p, c->hinv.p, c->steprows.p, 1, c->z.p);
    StepArgs A = step_args(c, 1, false);
    A.step_out = nullptr;
    vocab_commit_step(c, A);
    sync(c);
    h.push_back(token);
  });
}

nc_status nc_encode_stream(nc_ctx* c, uint32_t ns, const int32_t* const* tokens,
                           const size_t* n_tokens, uint8_t* const* out, const size_t* out_cap,
                           size_t* out_bytes, uint64_t* out_bits) {
  return guard([&] {
    NC_CHECK(c && tokens && n_tokens && out && out_cap && out_bytes && out_bits, NC_E_INVALID,
             "NULL argument");
    NC_HIP(hipSetDevice(c->dev));
    NC_CHECK(c->fp8_ready, NC_E_STATE, "FP8 context needs nc_calibrate_fp8 first");
    const int n = int(ns);
    size_t maxn = 0;
    bool cap_ok = true;
    for (int s = 0; s < n; ++s) {
      NC_CHECK(tokens[s] || n_tokens[s] == 0, NC_E_INVALID, "NULL token array");
      validate_tokens(c, tokens[s], n_tokens[s]);
      maxn = std::max(maxn, n_tokens[s]);
      if (out_cap[s] < encode_bound(n_tokens[s])) {
        cap_ok = false;
        out_bytes[s] = encode_bound(n_tokens[s]);
      }
    }
    NC_CHECK(cap_ok, NC_E_CAPACITY, "an output buffer is below nc_encode_bound");
    const auto t0 = std::chrono::steady_clock::now();
    reset_streams(c, n, int(maxn) + 1);
    c->stats = nc_stats{};
    // streams by decreasing length: the active ones at position i are a prefix
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return n_tokens[a] > n_tokens[b]; });
    for (int s = 0; s < n; ++s) {
      if (!n_tokens[s]) continue;
      NC_HIP(hipMemcpyAsync(c->hist.p + (size_t)s * c->T_alloc, tokens[s], n_tokens[s] * 4,
                            hipMemcpyHostToDevice, c->st));
    }
    sync(c);
    set_steprows(c, order.data(), order.size());
    if (ngram_on(c))
      launch_ngram_predict(c->vp, c->S, c->steprows.p, n, c->ngp.p, nullptr, nullptr, c->st);
    const int C = c->cfg.slide;
    // the n-gram chain of position i + 1 can run beside the distribution of position i when no
    // ensemble experts (P_1..P_K, single-buffered) are involved
    const bool pipe = ngram_on(c) && !(c->cfg.features & NC_F_ENSEMBLE);
    for (size_t a = 0; a < maxn; a += C) {
      // prefill: x positions [a, a + C) of every stream still active (teacher forcing)
      std::vector<RowMeta> rows;
      std::vector<int> off(n, -1);
      for (int k = 0; k < n; ++k) {
        const int s = order[k];
        if (n_tokens[s] <= a) break;
        off[k] = int(rows.size());
        for (size_t j = a; j < std::min(n_tokens[s], a + C); ++j)
          rows.push_back(RowMeta{s, int(j), j == 0 ? kBOS : tokens[s][j - 1], 0});
      }
      PassPlan plan = plan_pass(c, std::move(rows));
      const size_t seg_len = std::min((size_t)C, maxn - a);
      std::vector<int32_t> ar(seg_len * n, 0);
      std::vector<int> active(seg_len, 0);
      for (size_t i = 0; i < seg_len; ++i)
        for (int k = 0; k < n; ++k)
          if (n_tokens[order[k]] > a + i) {
            ar[i * n + k] = off[k] + int(i);
            active[i] = k + 1;
          }
      Stage stg;
      stage_pass(stg, plan);
      const size_t off_ar = stg.put(ar.data(), ar.size() * 4);
      const uint8_t* dst = upload_stage(c, stg);
      run_pass(c, plan, dst);
      const int32_t* seg_ar = reinterpret_cast<const int32_t*>(dst + off_ar);
      // The output layer depends only on the teacher-forced pass, not on the online models, so it
      // runs once per chunk of positions (up to kEncodeHeadRows rows, one per (position, stream
      // slot)); every position's vocabulary step then reads its B rows of the chunk.
      const int pc = std::max(1, std::min(int(seg_len), kEncodeHeadRows / n));
      c->zseg.alloc(size_t(pc) * n * c->V);
      for (size_t i0 = 0; i0 < seg_len; i0 += pc) {
        const int np = int(std::min(size_t(pc), seg_len - i0));
        run_lm_head(c, c->yb.p, c->xinv.p, seg_ar + i0 * n, np * n, c->zseg.p);
        bool uniform = true;
        for (size_t i = i0; i < i0 + np; ++i) uniform = uniform && active[i] == active[i0];
        const size_t p0 = a + i0;
        if (pipe && uniform && p0 > 0 && p0 % 2 == 0 && np > 1 &&
            !(c->cfg.features & NC_F_EAGER) && !profiling(c)) {
          encode_chunk_graph(c, int(p0), np, active[i0]);
          continue;
        }
        for (size_t i = i0; i < i0 + np; ++i) {
          StepArgs A = step_args(c, active[i], false);
          A.z = c->zseg.p + (i - i0) * n * size_t(c->V);
          A.step_out = nullptr;
          A.iv = c->iv.p;
          A.ptok = c->ptok.p;
          if (pipe)
            encode_step_pipelined(c, A, int(a + i));
          else
            vocab_commit_step(c, A);
        }
      }
    }
    if (pipe) NC_HIP(hipStreamWaitEvent(c->st, c->ev_pred, 0));
    sync(c);
    // host coder, one thread per stream
    std::vector<std::vector<uint32_t>> ivs(n);
    std::vector<std::vector<float>> pts(n);
    for (int s = 0; s < n; ++s) {
      ivs[s].resize(n_tokens[s] * 2);
      pts[s].resize(n_tokens[s]);
      if (!n_tokens[s]) continue;
      NC_HIP(hipMemcpy(ivs[s].data(), c->iv.p + (size_t)s * c->T_alloc * 2, n_tokens[s] * 8,
                       hipMemcpyDeviceToHost));
      NC_HIP(hipMemcpy(pts[s].data(), c->ptok.p + (size_t)s * c->T_alloc, n_tokens[s] * 4,
                       hipMemcpyDeviceToHost));
    }
    std::vector<std::vector<uint8_t>> bufs(n);
    std::vector<uint64_t> bits(n, 0);
    std::vector<int> bad(n, 0);
    auto work = [&](int s) {
      ArithEncoder enc(&bufs[s], c->cfg.cdf_total);
      for (size_t i = 0; i < n_tokens[s]; ++i) {
        const uint32_t cl = ivs[s][2 * i], ch = ivs[s][2 * i + 1];
        if (!(cl < ch && ch <= c->cfg.cdf_total)) {
          bad[s] = 1;
          return;
        }
        enc.encode(cl, ch);
      }
      enc.finish();
      bits[s] = enc.bits();
    };
    {
      const int nt = std::min<int>(n, std::max(1u, std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (int w = 0; w < nt; ++w)
        th.emplace_back([&, w] {
          for (int s = w; s < n; s += nt) work(s);
        });
      for (auto& t : th) t.join();
    }
    for (int s = 0; s < n; ++s) {
      NC_CHECK(!bad[s], NC_E_STATE, "stream %d produced an invalid interval", s);
      NC_CHECK(bufs[s].size() <= out_cap[s], NC_E_CAPACITY, "stream %d output too large", s);
      std::memcpy(out[s], bufs[s].data(), bufs[s].size());
      out_bytes[s] = bufs[s].size();
      out_bits[s] = bits[s];
      c->stats.tokens += n_tokens[s];
      c->stats.bits += double(bits[s]);
      for (float p : pts[s]) c->stats.ideal_bits += -std::log2((double)p);
    }
    c->stats.seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

nc_status nc_decode_stream(nc_ctx* c, uint32_t ns, const uint8_t* const* in,
                           const size_t* in_bytes, const size_t* n_tokens,
                           int32_t* const* tokens_out) {
  return guard([&] {
    NC_CHECK(c && in && in_bytes && n_tokens && tokens_out, NC_E_INVALID, "NULL argument");
    NC_HIP(hipSetDevice(c->dev));
    NC_CHECK(c->fp8_ready, NC_E_STATE, "FP8 context needs nc_calibrate_fp8 first");
    const int n = int(ns);
    size_t maxn = 0;
    for (int s = 0; s < n; ++s) maxn = std::max(maxn, n_tokens[s]);
    const auto t0 = std::chrono::steady_clock::now();
    reset_streams(c, n, int(maxn) + 1);
    c->stats = nc_stats{};
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return n_tokens[a] > n_tokens[b]; });
    set_steprows(c, order.data(), order.size());
    std::vector<ArithDecoder> dec;
    dec.reserve(n);
    for (int s = 0; s < n; ++s) dec.emplace_back(in[s], in_bytes[s], c->cfg.cdf_total);
    std::vector<int32_t> mode(n);
    d2h(c, mode.data(), c->moded.p, n);
    std::vector<uint32_t> tg(n);
    std::vector<StepOut> so(n);
    for (size_t i = 0; i < maxn; ++i) {
      int B = 0;
      while (B < n && n_tokens[order[B]] > i) ++B;
      std::vector<int> llm, upto;
      for (int k = 0; k < B; ++k)
        if (mode[order[k]] != M_SKIP) {
          llm.push_back(order[k]);
          upto.push_back(int(i));
        }
      std::vector<PassPlan> plans;
      if (!llm.empty()) plans = plan_catch_up(c, llm, upto);
      for (int k = 0; k < B; ++k) tg[k] = dec[order[k]].target();
      StepArgs A = step_args(c, B, true);
      if (plans.empty() && B <= kTargetsInline) {
        // nothing to upload: the targets travel in the kernel arguments
        A.targets = nullptr;
        for (int k = 0; k < B; ++k) A.targets_in[k] = tg[k];
      } else {
        Stage stg;
        for (auto& p : plans) stage_pass(stg, p);
        const size_t off_tg = stg.put(tg.data(), size_t(B) * 4);
        const uint8_t* dst = upload_stage(c, stg);
        BodyOpts o;
        o.graph = true;
        for (auto& p : plans) run_pass(c, p, dst, o);
        A.targets = reinterpret_cast<const uint32_t*>(dst + off_tg);
      }
      if (!llm.empty()) {
        run_lm_head(c, c->hlast.p, c->hinv.p, c->steprows.p, B, c->z.p);
        c->stats.llm_rows += llm.size();
      }
      c->stats.skipped += B - llm.size();
      A.lse = llm.empty() ? 0 : 1;  // every row skips the model: no logsumexp needed
      A.step_out = c->sout_hd;      // the outcome goes straight to host memory
      vocab_commit_step(c, A);
      if (!ngram_on(c)) {
        // no n-gram stage: pack the outcome here (mode stays LLM)
        std::vector<Outcome> oc(B);
        d2h(c, oc.data(), c->outc.p, B);
        for (int k = 0; k < B; ++k) so[k] = StepOut{oc[k].sym, oc[k].cl, oc[k].ch, M_LLM, oc[k].p};
      } else {
        sync(c);
        std::memcpy(so.data(), c->sout_h, size_t(B) * sizeof(StepOut));
      }
      for (int k = 0; k < B; ++k) {
        const int s = order[k];
        NC_CHECK(so[k].sym >= 0, NC_E_STATE, "invalid coding distribution on stream %d", s);
        dec[s].consume(so[k].cl, so[k].ch);
        NC_CHECK(!dec[s].overrun(), NC_E_CORRUPT, "stream %d: decoder ran past its input", s);
        tokens_out[s][i] = so[k].sym;
        c->hhist[s].push_back(so[k].sym);
        mode[s] = so[k].next_mode;
        c->stats.ideal_bits += -std::log2((double)so[k].p);
      }
    }
    for (int s = 0; s < n; ++s) c->stats.tokens += n_tokens[s];
    c->stats.seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

nc_status nc_profile(nc_ctx* c, int32_t cls, uint32_t stride) {
  return guard([&] {
    NC_CHECK(c, NC_E_INVALID, "NULL context");
    NC_CHECK(cls >= -1 && cls <= NC_K_COUNT, NC_E_INVALID, "bad kernel class");
    NC_CHECK(stride >= 1, NC_E_INVALID, "stride must be >= 1");
    NC_HIP(hipSetDevice(c->dev));
    sync(c);
    for (int k = 0; k < NC_K_COUNT; ++k) {
      if (cls != -1 && cls != NC_K_COUNT && cls != k) continue;
      auto& P = c->prof[k];
      P = nc_ctx::ProfClass{};
      P.on = cls != -1;
      P.stride = stride;
    }
  });
}

nc_status nc_autotune(nc_ctx* c, uint32_t max_rows, uint32_t reps, nc_tile* out, uint32_t cap,
                      uint32_t* n_out) {
  return guard([&] {
    NC_CHECK(c, NC_E_INVALID, "NULL context");
    graphs_clear(c);  // captured passes carry the launch shapes
    NC_CHECK(max_rows >= 1 && max_rows <= (1u << 20), NC_E_INVALID,
             "max_rows must be in [1, 2^20]");
    NC_CHECK(reps >= 1 && reps <= 1000, NC_E_INVALID, "reps must be in [1, 1000]");
    NC_CHECK(out || cap == 0, NC_E_INVALID, "NULL output with nonzero capacity");
    NC_HIP(hipSetDevice(c->dev));
    sync(c);
    if (c->S_alloc < 1) reset_streams(c, 1, 1);
    const int Mmax = int(max_rows);
    // output-layer GEMMs see one row per stream (decode) or an encode chunk of positions
    const int Mlm = std::min(Mmax, std::max(c->cfg.max_streams, kEncodeHeadRows));
    ensure_rows(c, Mmax);
    ensure_step(c, std::min(Mmax, c->cfg.max_streams));
    c->zseg.alloc(size_t(Mlm) * c->V);
    // scratch rows: stream 0, consecutive positions inside the RoPE table and the ring
    const int P = std::max(1, std::min(c->R, c->rope_pos));
    std::vector<RowMeta> rows(Mmax);
    for (int m = 0; m < Mmax; ++m) rows[m] = RowMeta{0, m % P, 0, (m % P) % c->R};
    h2d(c, c->rowsd.p, rows.data(), rows.size());
    NC_HIP(hipMemsetAsync(c->x.p, 0, c->x.n * sizeof(float), c->st));
    NC_HIP(hipMemsetAsync(c->xss.p, 0, c->xss.n * sizeof(float), c->st));
    NC_HIP(hipMemsetAsync(c->yb.p, 0, c->yb.n * sizeof(float), c->st));
    NC_HIP(hipMemsetAsync(c->xinv.p, 0, c->xinv.n * sizeof(float), c->st));
    NC_HIP(hipMemsetAsync(c->hb.p, 0, c->hb.n, c->st));
    NC_HIP(hipMemsetAsync(c->ob.p, 0, c->ob.n, c->st));
    struct Events {
      std::vector<hipEvent_t> e;
      hipEvent_t operator[](size_t i) const { return e[i]; }
      ~Events() {
        for (hipEvent_t x : e) (void)hipEventDestroy(x);
      }
    } ev;
    for (uint32_t i = 0; i < 2 * reps; ++i) {
      hipEvent_t x = nullptr;
      NC_HIP(hipEventCreate(&x));
      ev.e.push_back(x);
    }
    struct Scratch {
      DevBuf<uint8_t> b;
      ~Scratch() { b.release(); }
    } fl;  // released when the tuner returns, also on an error
    fl.b.alloc(size_t(512) << 20);
    DevBuf<uint8_t>& flush = fl.b;
    const int prec = c->prec;
    uint32_t n = 0;
    for (int g = 0; g < NC_G_COUNT; ++g) {
      const int top = g == NC_G_LMHEAD ? Mlm : Mmax;
      static const int kEpi[NC_G_COUNT] = {E_QKV, E_RESID, E_GLU, E_RESID, E_STORE};
      static const int kAm[NC_G_COUNT] = {A_NORM, A_DIRECT, A_NORM, A_DIRECT, A_NORM};
      for (int b = 0; b < kRowBuckets; ++b) {
        const int lo = b ? kRowBucketHi[b - 1] + 1 : 1;
        if (lo > top) {
          c->tiles[g][b] = GemmTile{};
          continue;
        }
        const int M = std::min(kRowBucketHi[b], top);
        // the GEMM of every layer in turn, as a pass meets them: weights come from HBM, not
        // from a cache warmed by the previous repetition
        std::vector<GemmArgs> la(g == NC_G_LMHEAD ? 1 : c->nl);
        for (int l = 0; l < int(la.size()); ++l) {
          switch (g) {
            case NC_G_QKV: la[l] = args_qkv(c, l, M, c->rowsd.p, false); break;
            case NC_G_OPROJ: la[l] = args_oproj(c, l, M, false, nullptr); break;
            case NC_G_GATEUP: la[l] = args_gateup(c, l, M, false, nullptr); break;
            case NC_G_DOWN: la[l] = args_down(c, l, M, false); break;
            default: la[l] = args_lm(c, c->yb.p, c->xinv.p, nullptr, M, c->zseg.p, false); break;
          }
        }
        const GemmArgs& a = la[0];
        // each timed launch follows a write over twice the last-level cache, as in a pass, where
        // the KV-cache stream between two uses of a layer's weights evicts them
        auto time_us = [&](const GemmTile& t) {
          launch_gemm(prec, kAm[g], kEpi[g], a, c->st, t);
          for (uint32_t r = 0; r < reps; ++r) {
            NC_HIP(hipMemsetAsync(flush.p, int(r & 0xFF), flush.n, c->st));
            NC_HIP(hipEventRecord(ev[2 * r], c->st));
            launch_gemm(prec, kAm[g], kEpi[g], la[r % la.size()], c->st, t);
            NC_HIP(hipEventRecord(ev[2 * r + 1], c->st));
          }
          NC_HIP(hipEventSynchronize(ev[2 * reps - 1]));
          float tot = 0.f;
          for (uint32_t r = 0; r < reps; ++r) {
            float ms = 0.f;
            NC_HIP(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
            tot += ms;
          }
          return 1000.f * tot / float(reps);
        };
        const float us_default = time_us(GemmTile{});
        GemmTile best{};
        float us_best = us_default;
        for (const GemmTile& t : gemm_candidates(prec, kEpi[g], a)) {
          const float u = time_us(t);
          if (u < us_best) {
            us_best = u;
            best = t;
          }
        }
        c->tiles[g][b] = best;
        if (n < cap)
          out[n] = nc_tile{g, kRowBucketHi[b] < top ? kRowBucketHi[b] : top, best.kind, best.mb,
                           best.waves, us_best, us_default};
        ++n;
      }
    }
    sync(c);
    // the scratch rows overwrote pass buffers and stream 0's cache: every stream needs a reset
    c->n_streams = 0;
    if (n_out) *n_out = n;
  });
}

nc_status nc_tiles_set(nc_ctx* c, const nc_tile* t, uint32_t n) {
  return guard([&] {
    NC_CHECK(c && (t || n == 0), NC_E_INVALID, "NULL argument");
    graphs_clear(c);  // captured passes carry the launch shapes
    static const int kEpi[NC_G_COUNT] = {E_QKV, E_RESID, E_GLU, E_RESID, E_STORE};
    for (uint32_t i = 0; i < n; ++i) {
      const nc_tile& e = t[i];
      NC_CHECK(e.gemm >= 0 && e.gemm < NC_G_COUNT, NC_E_INVALID, "entry %u: bad GEMM id", i);
      NC_CHECK(e.max_rows >= 1, NC_E_INVALID, "entry %u: max_rows must be >= 1", i);
      NC_CHECK(e.kind >= T_AUTO && e.kind <= T_WIDE, NC_E_INVALID, "entry %u: bad kind", i);
      const GemmTile g{e.kind, e.mb, e.waves};
      const int M = e.max_rows;
      GemmArgs a;
      switch (e.gemm) {
        case NC_G_QKV: a = args_qkv(c, 0, M, nullptr, false); break;
        case NC_G_OPROJ: a = args_oproj(c, 0, M, false, nullptr); break;
        case NC_G_GATEUP: a = args_gateup(c, 0, M, false, nullptr); break;
        case NC_G_DOWN: a = args_down(c, 0, M, false); break;
        default: a = args_lm(c, nullptr, nullptr, nullptr, M, nullptr, false); break;
      }
      NC_CHECK(gemm_tile_fits(c->prec, kEpi[e.gemm], a, g), NC_E_INVALID,
               "entry %u: launch shape does not fit this GEMM", i);
      c->tiles[e.gemm][row_bucket(M)] = g;
    }
  });
}

nc_status nc_tiles_reset(nc_ctx* c) {
  return guard([&] {
    NC_CHECK(c, NC_E_INVALID, "NULL context");
    graphs_clear(c);  // captured passes carry the launch shapes
    for (auto& row : c->tiles)
      for (auto& t : row) t = GemmTile{};
  });
}

nc_status nc_profile_read(nc_ctx* c, int32_t cls, nc_kstat* out) {
  return guard([&] {
    NC_CHECK(c && out, NC_E_INVALID, "NULL argument");
    NC_CHECK(cls >= 0 && cls < NC_K_COUNT, NC_E_INVALID, "bad kernel class");
    NC_HIP(hipSetDevice(c->dev));
    sync(c);
    *out = c->prof[cls].k;
  });
}

nc_status nc_get_stats(const nc_ctx* c, nc_stats* out) {
  return guard([&] {
    NC_CHECK(c && out, NC_E_INVALID, "NULL argument");
    *out = c->stats;
  });
}

}  // extern "C"
