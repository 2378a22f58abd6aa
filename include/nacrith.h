/*
 * nacrith.h -- C ABI of the MI355X (gfx950) per-token probability pipeline of the Nacrith
 * neural lossless text compressor (arXiv 2602.19626).
 *
 * The pipeline, per token of each stream (paper Algorithm 1):
 *   135M-shape decoder-only transformer forward over a sliding KV cache (sections 3.2, 3.10)
 *   -> vocabulary softmax (section 3.3) -> adaptive log-space bias head (section 3.7)
 *   -> token n-gram and confidence skip (sections 3.5, 3.8) -> linear mixer (section 3.6)
 *   -> CDF-24 quantisation (section 3.4) -> 32-bit arithmetic coder on the host (section 3.9).
 *
 * Conventions for every call:
 *  - Return value: NC_OK or an nc_status error; nc_last_error() gives a thread-local message.
 *    No C++ exception crosses this interface.
 *  - Buffers: the caller owns every input and output buffer.  Pointers documented as "host" are
 *    ordinary host memory; pointers documented as "device" are HIP device allocations on the
 *    context's device (for example torch tensors on cuda:0); `stream` arguments are hipStream_t
 *    values passed as void* (NULL = the default stream).  The library owns the context and all
 *    device state it allocates.
 *  - A context is used by one host thread at a time.
 *  - Token ids are int32 in [0, vocab).  Probabilities are float32.  CDFs are uint32 with
 *    vocab + 1 entries, cdf[0] = 0 and cdf[vocab] = total.
 */
#ifndef NACRITH_H
#define NACRITH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nc_status {
  NC_OK = 0,
  NC_E_INVALID = 1,   /* bad argument: token out of range, NaN/negative probability, bad shape */
  NC_E_DEVICE = 2,    /* a HIP runtime call failed */
  NC_E_NOMEM = 3,     /* a device or host allocation failed */
  NC_E_CAPACITY = 4,  /* an output buffer is too small; the required size is reported */
  NC_E_CORRUPT = 5,   /* the decoder consumed more than 8 * bytes + 32 bits */
  NC_E_STATE = 6      /* call sequence violates the context state (e.g. history mismatch) */
} nc_status;

enum { NC_FP32 = 0, NC_BF16 = 1, NC_FP8 = 2 };                 /* GEMM operand precision */
enum { NC_SKIP_NONE = 0, NC_SKIP_ENTROPY = 1, NC_SKIP_PMAX = 2 };  /* section 3.8 skip rule */
enum {
  NC_F_HEAD = 1u << 0,      /* adaptive bias head, section 3.7 */
  NC_F_NGRAM = 1u << 1,     /* token n-gram, section 3.5 */
  NC_F_SKIP = 1u << 2,      /* confidence-based LLM skip, section 3.8 */
  NC_F_MIXER = 1u << 3,     /* linear context mixer, section 3.6 */
  NC_F_ENSEMBLE = 1u << 4,  /* softmax-gated {LLM, n-gram orders 1..K} head trained by SGD */
  NC_F_EAGER = 1u << 5,     /* launch every kernel directly: no captured HIP graph is replayed
                               (the batched encode replays captured chunks of its per-position
                               steps otherwise; same bits either way) */
  NC_F_DECODE_GRAPHS = 1u << 6  /* also replay captured HIP graphs of the decode / probe
                                   transformer passes (same bits; measured about 1.5% slower
                                   than direct launches, so off by default) */
};
enum { NC_MODE_LLM = 0, NC_MODE_SKIP = 1, NC_MODE_MIX = 2, NC_MODE_ENSEMBLE = 3 };

/* Model shape, ensemble constants and run options.  All fields are read at nc_create(). */
typedef struct nc_config {
  /* d_model and d_ffn multiples of 16; head_dim 16, 32 or 64; vocab a multiple of 4 */
  int32_t n_layers, d_model, n_heads, n_kv_heads, head_dim, d_ffn, vocab;
  float rope_theta;          /* RoPE base; rotate-half pairs (i, i + head_dim/2) */
  float norm_eps;            /* RMSNorm epsilon */
  int32_t ctx_len;           /* L: KV entries kept (section 3.10); multiple of slide */
  int32_t slide;             /* C: entries dropped when appending to a full cache */
  int32_t ngram_order;       /* K: orders 1..K (section 3.5), 1 <= K <= 4 */
  float ngram_eps;           /* lambda_k = n_k / (n_k + eps), eps = 5 in the paper */
  int32_t ngram_max_contexts;/* per order; no new context is stored once reached (500,000) */
  float head_lr;             /* alpha of the bias head, 1e-3 (section 3.7); also the SGD lr
                                of the ensemble gate */
  float mix_eta;             /* exponential-weights rate of the mixer (section 3.6) */
  float mix_w_llm;           /* initial LLM weight of the two-model mixer (0.85; 0.5 uniform) */
  int32_t warmup;            /* tokens coded by the LLM alone before skip/mix (100) */
  int32_t skip_mode;         /* NC_SKIP_* */
  float skip_entropy_bits;   /* skip when H(p_ngram) < this (1.5 bits) */
  float skip_pmax;           /* skip when max p_ngram >= this (0.99) */
  uint32_t cdf_total;        /* T, 2^24 (section 3.4); vocab < T <= 2^24 */
  int32_t precision;         /* NC_FP32 | NC_BF16 | NC_FP8 */
  uint32_t features;         /* NC_F_* bit set */
  int32_t max_streams;       /* streams that can be coded together by one call */
} nc_config;

/* Optional diagnostics of nc_probs_for_context(); every array pointer may be NULL. */
typedef struct nc_probe {
  float* logits;             /* host, vocab floats: LLM logits z (valid if llm_ran) */
  float* ptilde;             /* host, vocab floats: bias-head output softmax(z + b) */
  float* p_ngram;            /* host, vocab floats: n-gram distribution P_K */
  uint32_t* cdf;             /* host, vocab + 1 uint32: the CDF-24 of the coding distribution */
  int32_t mode;              /* out: NC_MODE_* used at this position */
  int32_t llm_ran;           /* out: 1 if the transformer produced logits for this position */
  float entropy_bits;        /* out: H(p_ngram) in bits */
  float pmax;                /* out: max p_ngram */
  float mix_w[2];            /* out: mixer weights before this position's update */
} nc_probe;

/* Per-call statistics of the last encode/decode on a context. */
typedef struct nc_stats {
  uint64_t tokens;           /* tokens coded */
  uint64_t llm_rows;         /* decode: positions whose logits were used (not skipped) */
  uint64_t skipped;          /* decode: positions coded by the n-gram alone (encode: 0; its
                                modes are decided on the device) */
  uint64_t body_rows;        /* transformer rows evaluated (KV appends) */
  double bits;               /* exact coded bits (sum over streams) */
  double ideal_bits;         /* sum -log2 p_i(t_i) of the float32 coding distributions */
  double seconds;            /* wall time of the call */
  double wait_seconds;       /* part of it the host spent blocked on the device */
  uint64_t graph_replays;    /* transformer passes run by replaying a captured HIP graph */
  uint64_t graph_captures;   /* passes captured (first use of a pass shape) */
} nc_stats;

typedef struct nc_ctx nc_ctx;

/* ---- lifecycle ----------------------------------------------------------------------------- */

/* Create a context on the current HIP device.  weights_f32 (host) is the flat float32 buffer:
 * E[vocab][d], then per layer attn_norm[d], Wq[Hq*hd][d], Wk[Hkv*hd][d], Wv[Hkv*hd][d],
 * Wo[d][Hq*hd], mlp_norm[d], Wg[ffn][d], Wu[ffn][d], Wd[d][ffn], then final_norm[d]
 * (matrices [out][in], y = x W^T; E is tied as the output matrix, section 3.2 Eq. (lm) with no
 * output bias).  It is copied; the caller may free it on return.  The precision copies (BF16,
 * FP8 with per-tensor scales) are made on the device.  Errors: NC_E_INVALID (shape, NULL),
 * NC_E_NOMEM, NC_E_DEVICE. */
nc_status nc_create(const nc_config* cfg, const float* weights_f32, nc_ctx** out);

/* Release a context and all its device memory.  NULL-safe. */
void nc_destroy(nc_ctx* ctx);

/* Reset (and size) the per-stream state for n_streams streams of up to max_tokens tokens each:
 * KV caches, n-gram tables, bias vectors, mixer weights and histories are cleared
 * (Algorithm 1, initialisation).  NC_E_INVALID if n_streams > cfg.max_streams. */
nc_status nc_streams_reset(nc_ctx* ctx, uint32_t n_streams, uint32_t max_tokens);

/* Static FP8 activation scales (per-tensor amax / 448), calibrated by running the FP32 model
 * on tokens[0..n) of a calibration stream.  Required once before FP8 coding. */
nc_status nc_calibrate_fp8(nc_ctx* ctx, const int32_t* tokens, size_t n);

/* ---- the pipeline ------------------------------------------------------------------------ */

/* Coding distribution for position n of `stream` given its history tokens[0..n) (host)
 * (Algorithm 1, the steps before probs_to_cdf).  Tokens beyond those already committed on this
 * stream are committed first, exactly as the encoder would (each one updates the head, mixer and
 * n-gram).  NC_E_STATE if tokens[0..committed) differs from the committed history.
 * probs (host) receives vocab floats; probe may be NULL. */
nc_status nc_probs_for_context(nc_ctx* ctx, uint32_t stream, const int32_t* tokens, size_t n,
                               float* probs, nc_probe* probe);

/* Algorithm 1, the update step after a token is coded: commit `token` as the next token of
 * `stream`.  The n-gram counts always take the token; the bias head and the mixer weights take
 * their SGD and exponential-weights steps when the position's mode ran the LLM (respectively
 * mixed), exactly as in nc_encode_stream.  The position's distribution is recomputed from the
 * committed state, so the result does not depend on whether nc_probs_for_context was called. */
nc_status nc_mix_update(nc_ctx* ctx, uint32_t stream, int32_t token);

/* CDF-24 quantisation, section 3.4 (Algorithm 1 probs_to_cdf(p, 2^24)): for each of `rows`
 * rows, c_i = max(1, floor(p_i (total - vocab))) computed exactly from the float32 value, the
 * residual total - sum(c) added to the lowest-index argmax, cdf = exclusive prefix sum.
 * probs: device, rows x vocab float32 (row-major).  cdf: device, rows x (vocab + 1) uint32.
 * row_status: device, rows int32 (0 ok, 1 = NaN/negative/>1 probability or mass above total,
 * in which case that row's cdf is unspecified); may be NULL.  Pure: no context needed.
 * Errors: NC_E_INVALID for vocab outside [1, 262144], total <= vocab, total > 2^24, NULL
 * pointers.  Uses a library-owned device workspace of rows * ceil(vocab/4096) * 16 bytes, one per
 * (device, stream): calls on one stream share it in stream order, calls on different streams
 * (also from different host threads) never share it.  The first call on a stream, and a call that
 * needs more than that stream's buffer holds, allocates (hipMalloc; a grown buffer is freed after
 * its stream has drained, which blocks the host), so such a call cannot be captured into a
 * HIP graph. */
nc_status nc_quantize_cdf24(const float* probs, uint32_t rows, uint32_t vocab, uint32_t total,
                            uint32_t* cdf, int32_t* row_status, void* stream);

/* nc_quantize_cdf24 for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): same arguments, same integers, but
 * its kernels take their workspace from a fixed device array of 65,536 segment partials
 * (1 MiB per GPU, held until the process ends) instead of a library-allocated buffer; it calls
 * no hipMalloc or hipFree.  The workspace is needed on the segment path (up to 64 rows, rows not
 * 16-byte aligned or with vocab not a multiple of 4, or vocab > 49,152): there rows *
 * ceil(vocab / 4096) must not exceed 65,536, else NC_E_CAPACITY and nothing is launched.  Every
 * call on one GPU shares that GPU's array (nothing in it needs clearing between calls), so two
 * calls whose work overlaps on one GPU -- on different streams, or from different threads --
 * race and give unspecified CDFs; serialise them on one stream.  The first call on a device
 * resolves the array's address there (hipGetSymbolAddress). */
nc_status nc_quantize_cdf24_noalloc(const float* probs, uint32_t rows, uint32_t vocab,
                                    uint32_t total, uint32_t* cdf, int32_t* row_status,
                                    void* stream);

/* Interval lookup on CDF rows (section 3.9): mode 0 (encode) key[r] is a symbol s and the
 * output is (s, cdf[s], cdf[s+1]); mode 1 (decode) key[r] is a target count and the output is
 * the largest s with cdf[s] <= target, with its interval.  cdf: device rows x (vocab+1);
 * key: device rows uint32; out: device rows x 3 uint32. */
nc_status nc_cdf_interval(const uint32_t* cdf, uint32_t rows, uint32_t vocab,
                          const uint32_t* key, int32_t mode, uint32_t* out, void* stream);

/* Worst-case bytes of one encoded stream of n_tokens tokens: ceil((25 n + 64) / 8). */
size_t nc_encode_bound(size_t n_tokens);

/* Compress n_streams independent streams (Algorithm 1 + ArithEncoder.finish), batched on the
 * GPU.  tokens[s] (host) has n_tokens[s] ids; out[s] (host) has out_cap[s] bytes; on return
 * out_bytes[s] and out_bits[s] give the exact code size (bits packed MSB-first, last byte
 * zero-padded).  Resets the stream state first.  NC_E_CAPACITY if out_cap[s] <
 * nc_encode_bound(n_tokens[s]) (out_bytes[s] then holds that bound). */
nc_status nc_encode_stream(nc_ctx* ctx, uint32_t n_streams, const int32_t* const* tokens,
                           const size_t* n_tokens, uint8_t* const* out, const size_t* out_cap,
                           size_t* out_bytes, uint64_t* out_bits);

/* Decompress (the mirror of encode, section 3.1): in[s] (host, in_bytes[s] bytes) holds
 * n_tokens[s] tokens, which are written to tokens_out[s] (host).  NC_E_CORRUPT if a decoder
 * reads past 8 * in_bytes[s] + 32 bits. */
nc_status nc_decode_stream(nc_ctx* ctx, uint32_t n_streams, const uint8_t* const* in,
                           const size_t* in_bytes, const size_t* n_tokens,
                           int32_t* const* tokens_out);

/* Statistics of the last nc_encode_stream / nc_decode_stream call. */
nc_status nc_get_stats(const nc_ctx* ctx, nc_stats* out);

/* ---- measurement ----------------------------------------------------------------------------
 * Kernel classes of the pipeline.  With profiling on for one class, the library records a pair
 * of HIP events on its own stream around every launch of that class and accumulates the elapsed
 * time, the launch count and the algorithmic bytes moved / flops done (from the launch shapes:
 * GEMM weights + activations read + outputs written; attention keys/values of the window + q/o;
 * vocabulary chain z, b, n-gram rows read and b written). */
enum {
  NC_K_QKV = 0,     /* RMSNorm + QKV GEMM + RoPE + KV-ring write */
  NC_K_ATTN = 1,    /* GQA attention over the window */
  NC_K_OPROJ = 2,   /* O projection + residual */
  NC_K_GATEUP = 3,  /* RMSNorm + gate/up GEMM + SiLU gating */
  NC_K_DOWN = 4,    /* down projection + residual */
  NC_K_LMHEAD = 5,  /* final RMSNorm + tied output GEMM */
  NC_K_VOCAB = 6,   /* softmax/head/mix + CDF-24 + interval/search + head/mixer/n-gram update */
  NC_K_NGRAM = 7,   /* n-gram prediction, entropy and skip decision */
  NC_K_COUNT = 8
};
typedef struct nc_kstat {
  double ms;          /* summed event time of the timed launches */
  uint64_t launches;  /* launches of the class */
  uint64_t timed;     /* launches that were timed: the 1st, (stride+1)-th, ... */
  double bytes;       /* algorithmic bytes of the timed launches */
  double flops;       /* algorithmic flops of the timed launches */
} nc_kstat;

/* Enable timing of one kernel class (0 .. NC_K_COUNT-1), or of every class (NC_K_COUNT), and
 * clear its counters; -1 disables and clears every class.  Classes enabled by earlier calls stay
 * enabled.  Every stride-th launch of a class (stride >= 1) is bracketed by events recorded on the
 * stream the class runs on, which bounds the cost of the event records on long runs; ms / timed
 * is the class's average launch duration.  The events add work to the stream, so runs whose wall
 * time is reported should not profile.  NC_E_INVALID for a bad class or stride 0. */
nc_status nc_profile(nc_ctx* ctx, int32_t kernel_class, uint32_t stride);
/* Counters of one kernel class since it was enabled. */
nc_status nc_profile_read(nc_ctx* ctx, int32_t kernel_class, nc_kstat* out);

/* ---- launch-shape autotuner ------------------------------------------------------------------
 * Each transformer GEMM can run in several launch shapes: a split kernel (one workgroup per
 * group of 16-column blocks and 16 mb rows, with `waves` waves dealing the 64-wide K parts), two
 * LDS-staged tile kernels and, in BF16 / FP8, a 128 x 128 tile kernel.  All shapes evaluate the
 * same per-part MFMA chains and add them in the same order, so the choice never changes a bit
 * of any result; it only changes the speed.  Without tuning, a fixed rule on the row count
 * picks the shape.
 *
 * nc_autotune times, with HIP events on the library's stream, the fixed rule and every fitting
 * shape of each GEMM (QKV, O, gate/up, down, output layer) at the top of each row bucket
 * (1, 2, 4, 8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 1024, ... rows) up to max_rows (the
 * output layer up to the larger of max_streams and 2,048, its encode chunk), `reps` launches per
 * shape after one warm-up launch, each
 * timed alone right after a 512 MiB device write that evicts the weights from the caches (as the
 * KV-cache stream of a pass does) and cycling through the layers' weights, and
 * keeps the fastest shape per (GEMM, bucket) for every later call on this context.  It writes
 * scratch rows into the pass buffers and stream 0's KV cache, so afterwards every stream must be
 * reset (nc_streams_reset; the coding calls reset by themselves).  out (host, may be NULL when
 * cap is 0) receives up to cap entries, n_out (may be NULL) the number of (GEMM, bucket) pairs
 * measured.  Errors: NC_E_INVALID for max_rows outside [1, 2^20] or reps outside [1, 1000]. */
enum {
  NC_G_QKV = 0,
  NC_G_OPROJ = 1,
  NC_G_GATEUP = 2,
  NC_G_DOWN = 3,
  NC_G_LMHEAD = 4,
  NC_G_COUNT = 5
};
typedef struct nc_tile {
  int32_t gemm;      /* NC_G_* */
  int32_t max_rows;  /* the bucket's top row count (the rows it was timed at) */
  int32_t kind;      /* 0 fixed rule, 1 split, 2 small tile, 3 64 x 64 tile, 4 128 x 128 tile */
  int32_t mb;        /* split: 16-row blocks per workgroup */
  int32_t waves;     /* split: waves per workgroup */
  float us_best;     /* measured time of the chosen shape per launch, microseconds */
  float us_default;  /* measured time of the fixed rule per launch, microseconds */
} nc_tile;
nc_status nc_autotune(nc_ctx* ctx, uint32_t max_rows, uint32_t reps, nc_tile* out, uint32_t cap,
                      uint32_t* n_out);
/* Install n shapes (host array), e.g. a table saved from nc_autotune: entry i sets the shape of
 * GEMM t[i].gemm for the row bucket that contains t[i].max_rows (kind 0 restores the fixed
 * rule; us_* are ignored).  NC_E_INVALID for a bad id or kind, or a shape that does not fit the
 * GEMM (a split shape outside 1..4 row blocks or 1..16 waves, or over the LDS budget; the
 * 128 x 128 kernel in FP32 or for the QKV GEMM at head_dim 16); entries before it stay set. */
nc_status nc_tiles_set(nc_ctx* ctx, const nc_tile* t, uint32_t n);
/* Forget the measured shapes (back to the fixed rule). */
nc_status nc_tiles_reset(nc_ctx* ctx);

/* ---- host arithmetic coder (section 3.9), exposed for testing and container tools --------- */

/* Encode n intervals (host, n x 2 uint32: cl, ch with 0 <= cl < ch <= total) with the 32-bit
 * coder.  out (host) has cap bytes; NC_E_CAPACITY if too small (out_bytes = needed bound). */
nc_status nc_ac_encode(const uint32_t* intervals, size_t n, uint32_t total, uint8_t* out,
                       size_t cap, size_t* out_bytes, uint64_t* out_bits);

/* Decode n symbols that were all coded against the same CDF (host, vocab + 1 uint32). */
nc_status nc_ac_decode_static(const uint8_t* in, size_t in_bytes, const uint32_t* cdf,
                              uint32_t vocab, size_t n, int32_t* out);

/* ---- softmax-gated ensemble head (differentiation workload) ------------------------------ */

/* Forward of the ensemble head for `rows` rows: q0 = softmax(z + b), w = softmax(theta),
 * p = w_0 q0 + sum_{j>=1} w_j P_j, loss[r] = -log p(t*_r).  All device pointers:
 * z rows x vocab, b vocab, theta n_experts, P rows x (n_experts-1) x vocab, target rows int32;
 * outputs loss rows, p rows x vocab (may be NULL), resp rows x n_experts (responsibilities
 * r_j = w_j q_j(t*) / p(t*), needed by the backward).  n_experts <= 8.  Workspace: as for
 * nc_quantize_cdf24 (one library-owned buffer per device and stream, grown on demand). */
nc_status nc_ensemble_forward(const float* z, const float* b, const float* theta,
                              const float* P, const int32_t* target, uint32_t rows,
                              uint32_t vocab, uint32_t n_experts, float* loss, float* p,
                              float* resp, void* stream);

/* Backward: grad_b[t] = sum_r g_r r_{r,0} (q0_r(t) - 1[t = t*_r]),
 * grad_theta[j] = sum_r g_r (w_j - r_{r,j}), with g = grad_loss (device, rows) -- a fixed-order
 * reduction over rows (no float atomics).  If lr != 0 the SGD step b -= lr grad_b,
 * theta -= lr grad_theta is applied in place as well (b, theta writable device pointers).
 * Workspace: as for nc_ensemble_forward. */
nc_status nc_ensemble_backward(const float* z, float* b, float* theta, const float* resp,
                               const int32_t* target, const float* grad_loss, uint32_t rows,
                               uint32_t vocab, uint32_t n_experts, float lr, float* grad_b,
                               float* grad_theta, void* stream);

/* Thread-local message of the last error on this thread ("" if none). */
const char* nc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NACRITH_H */
