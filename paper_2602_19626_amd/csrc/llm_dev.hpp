// Shared declarations of the transformer kernels (k_llm.hip) and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace nc {

enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2 };
// A_NORM: A holds quantise(x * gain) of residual rows x, and each output row is scaled by the
// row's RMSNorm scale 1 / sqrt(mean(x^2) + eps) (RMSNorm(x) * gain * W^T, the scale applied after
// the sum); A_DIRECT: plain A.
enum AMode { A_NORM = 0, A_DIRECT = 1 };
enum Epi { E_STORE = 0, E_RESID = 1, E_GLU = 2, E_QKV = 3 };  // epilogues

// Per-row metadata of a transformer pass: which stream, which position, which token.
struct RowMeta {
  int32_t stream;
  int32_t pos;
  int32_t tok;
  int32_t slot;  // pos mod ring: the KV-ring slot of this position (filled by the host)
};

// Arguments of one GEMM C[M][N] = A[M][K] W[N][K]^T (+ epilogue).
struct GemmArgs {
  int M, N, K;
  const void* A;          // Prec rows [rows][K]
  const int32_t* a_rows;  // optional gather: A row of output row m is a_rows[m]
  // A_NORM row scales: inv[a_rows[m]] if given, else from the block sums of squares ssq[a_rows[m]]
  const float* inv;
  const float* ssq;       // [rows][K/16]
  float eps;
  float a_scale;          // FP8: dequantisation scale of A
  const void* W;          // Prec [N][K]
  float w_scale;          // FP8 weight scale
  // epilogue outputs
  float* out_f32;         // E_STORE: [M][ldo]; E_RESID: residual x [M][ldo] (+=)
  int ldo;
  void* out_p;            // E_GLU: Prec h [M][N/2] (quantised with out_scale for FP8)
  float out_scale;        // FP8 activation scale of the produced tensor (1/scale applied)
  float* out_amax;        // optional: max |output| before quantisation (calibration)
  // E_RESID: the updated rows also give the next normed GEMM its operand and row statistics
  float* ssq_out;         // block sums of squares [M][N/16]
  void* y_out;            // Prec quantise(x * y_gain) [M][N] (FP8: times y_inv_scale), or null
  const float* y_gain;
  float y_inv_scale;
  float* y_amax;          // optional: max |x * y_gain| (calibration)
  // E_QKV
  const RowMeta* rows;
  const float* rope;      // [max_pos][hd/2][2] (cos, sin), built in float64, stored float32
  void* q_out;            // attention precision [M][Hq][hd]
  void* k_cache;          // [stream][kvh][R][hd] for this layer (stream stride kv_stride)
  void* vt_cache;         // [stream][kvh][hd][R]
  long long kv_stride;    // elements per stream in k_cache / vt_cache (one layer)
  int Hq, Hk, hd, ring;
};

// Attention work item: a block of up to 16 (query, head) columns of one stream and kv head.
// Column c maps to global column cc = c0 + c, query row row_base + cc / g and head
// kvh * g + cc % g, with g = Hq / Hkv.
struct AttnItem {
  int32_t stream;
  int32_t kvh;
  int32_t row_base;
  int32_t pos_base;
  int32_t c0;
  int32_t ncols;
  int32_t pad[2];
};

struct AttnArgs {
  const AttnItem* items;
  int n_items;
  const void* q;        // [rows][Hq][hd] attention precision
  const void* k_cache;  // layer base, stream stride kv_stride
  const void* vt_cache;
  long long kv_stride;
  void* out;            // O-projection A operand [rows][Hq*hd] (Prec of the GEMMs)
  float out_scale;      // FP8 quantisation scale of the output
  float* out_amax;      // optional calibration amax
  int Hq, Hk, hd, ring, ctx_len, slide;
  float scale_log2;     // log2(e) / sqrt(hd)
  float* ws;            // group states of the parallel path
  size_t ws_bytes;
  int xcd_place;        // parallel path: items share a stream's K/V; place them XCD-aware
  int* ctr;             // parallel path, optional: attention_counters(n_items) counters, zero
                        // between launches (given: few FP32 items run one workgroup per chunk)
};

// Launch shape of one GEMM.  Every shape evaluates the same per-part MFMA chains and adds them in
// the same order, so the choice changes the speed only, never a bit of the result.
enum GemmKind {
  T_AUTO = 0,    // the fixed size rule
  T_SPLIT = 1,   // a workgroup per (epilogue group, mb row blocks); waves deal the K parts
  T_TILE_S = 2,  // LDS-staged tiles, small (16 x 64, or 16 x 64 gate/up pairs)
  T_TILE_M = 3,  // LDS-staged tiles, 64 x 64
  T_WIDE = 4,    // 128 x 128 tiles with XCD-aware order (BF16 / FP8 only)
};
struct GemmTile {
  int kind = T_AUTO;
  int mb = 0;     // T_SPLIT: 16-row blocks per workgroup (1..4)
  int waves = 0;  // T_SPLIT: waves per workgroup (1..16)
};
void launch_gemm(int prec, int amode, int epi, const GemmArgs& a, hipStream_t s,
                 GemmTile t = GemmTile{});
bool gemm_tile_fits(int prec, int epi, const GemmArgs& a, const GemmTile& t);
// Every launch shape that fits this GEMM (the autotuner's search space).
std::vector<GemmTile> gemm_candidates(int prec, int epi, const GemmArgs& a);
// RMSNorm scale of rows a_rows[m] (from a.ssq) into inv[a_rows[m]]
void launch_row_rms(const GemmArgs& a, float* inv, hipStream_t s);
void launch_attention(int prec_att, int prec_out, const AttnArgs& a, bool parallel,
                      hipStream_t s);
size_t attention_ws_bytes(int n_items);
size_t attention_counters(int n_items);
// x[r] = E[rows[r].tok], its block sums of squares ssq[r][d/16] and the first normed GEMM's
// operand y[r] = quantise(x[r] * gain) in precision prec (FP8: times inv_scale)
void launch_embed(const float* E, const RowMeta* rows, int n, int d, float* x, float* ssq,
                  void* y, const float* gain, int prec, float inv_scale, float* y_amax,
                  hipStream_t s);
void launch_convert(const float* src, void* dst, long long n, int prec, float inv_scale,
                    hipStream_t s);

}  // namespace nc
