// Device-side state of the per-token vocabulary chain (bias head, mixer, n-gram, CDF-24) and the
// launchers of k_vocab.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nc {

constexpr int kSlots = 64;    // continuation cap per context (paper section 3.5)
constexpr int kMaxOrder = 4;  // n-gram orders 1..4
constexpr int kMaxExperts = 8;

enum { M_LLM = 0, M_SKIP = 1, M_MIX = 2, M_ENS = 3 };

// Per-row outcome of a step: the coded symbol and what the updates need.
struct Outcome {
  int32_t sym;
  uint32_t cl, ch;
  int32_t mode;
  float p;       // coding probability of sym (float32)
  float pt;      // bias-head probability ptilde(sym)
  float png;     // n-gram probability p_ng(sym)
  float lse;     // logsumexp(z + b) of the row
  float pk[kMaxOrder];   // P_1..P_K at sym (ensemble)
  float r[kMaxExperts];  // ensemble responsibilities w_j q_j(sym) / p(sym)
};

// What the host reads back after each decode step.
struct StepOut {
  int32_t sym;
  uint32_t cl, ch;
  int32_t next_mode;
  float p;  // coding probability of sym
  int32_t pad[3];
};

struct LsePart {
  float m, s;
};
struct NgPart {
  float h, mx;
};

// All per-stream device state (arrays indexed by stream).
struct StreamState {
  int V, K, maxT, cap, maxctx;
  float* b;          // [S][V] bias (or ensemble bias)
  int32_t* uni;      // [S][V] unigram counts
  int32_t* nseen;    // [S]
  int32_t* hist;     // [S][maxT] committed tokens
  int32_t* ncommit;  // [S]
  float* png;        // [S][V] p_ng = P_K at the current position
  float* pk;         // [S][K][V] P_1..P_K (ensemble only, else null)
  float* lw;         // [S][kMaxExperts] mixer log-weights / ensemble gate logits
  int32_t* mode;     // [S] mode of the current position
  float* H;          // [S] entropy (bits) of p_ng
  float* pmax;       // [S]
  int32_t* next_ctx; // [S][kMaxOrder] pool index of the order-k context of the current position
  // n-gram tables, one per (stream, order): t = s * K + (k - 1)
  int32_t* keys;     // [t][cap][4]
  int32_t* kidx;     // [t][cap]   -1 = empty
  int32_t* pool;     // [t][maxctx][kSlots][2] (token, count)
  int32_t* pool_n;   // [t][maxctx] slots used
  int32_t* pool_sum; // [t][maxctx] sum of counts = n_k
  int32_t* nctx;     // [t]
};

// Constants of the ensemble chain.
struct VocabParams {
  int V;
  uint32_t total;
  int use_head, use_ngram, use_skip, use_mixer, ensemble;
  int K;
  float head_lr, mix_eta, ngram_eps;
  int ngram_max_contexts;
  int warmup, skip_mode;
  float skip_bits, skip_pmax;
};

// Decode steps of at most kTargetsInline rows pass their targets in the kernel arguments.
constexpr int kTargetsInline = 8;

// Rows of one step: row r is stream rows[r]; z row r of `z` (ld V) holds its logits when its mode
// uses the LLM.  key[r] is the token (encode) or the target count (decode).
struct StepArgs {
  int B;
  const int32_t* rows;
  const float* z;
  int decode;            // 0: key = token from hist at ncommit; 1: key = the row's target
  int no_update;         // 1: probe only (no bias update, no interval output)
  const uint32_t* targets;              // decode: [B] on the device, or null: targets_in
  uint32_t targets_in[kTargetsInline];  // decode with targets == null: the targets of rows 0..B)
  LsePart* lse_parts;    // [B][nseg]
  void* seg_parts;       // SegPartial [B][nseg]
  NgPart* ng_parts;      // [B][nseg]
  Outcome* out;          // [B]
  StepOut* step_out;     // [B] (decode) or null
  uint32_t* iv;          // encode: [S][maxT][2] intervals, or null
  float* ptok;           // encode: [S][maxT] p(t_i), or null
  // optional full-row diagnostics (single-row probes), each [B][V] / [B][V+1] or null
  float* dbg_p;
  float* dbg_pt;
  uint32_t* dbg_cdf;
  // Batched encode: every row is at position pos (>= 0), known to the host, and the update kernel
  // takes the committed token from hist; -1: the position is S.ncommit[stream].  With pos_base
  // (a device int; a step captured into a graph that is replayed for every chunk of positions)
  // the position is pos + *pos_base.
  int pos;
  const int* pos_base;
  // Updates run by the n-gram update kernel: kUpdCounts (token history, unigram and n-gram
  // counts, next contexts, ncommit) and / or kUpdMixer (mixer weights or ensemble gate, which
  // need the step's outcome).
  int upd;
  // 0: no row of the step uses the model's logits (every mode is skip), so the logsumexp pass is
  // not launched
  int lse;
};
constexpr int kUpdCounts = 1, kUpdMixer = 2;

// V1-V3, V4 for the ensemble and the V5 n-gram / mixer update (unless A.no_update)
void launch_vocab_step(const VocabParams& P, const StreamState& S, const StepArgs& A,
                       hipStream_t s);
// n-gram distribution, entropy and mode of the current position of each row's stream; with
// step_out, also packs the step's outcome and the next mode for the host (decode).
// pos: the rows' position (>= 0, batched encode) or -1 (S.ncommit).
void launch_ngram_predict(const VocabParams& P, const StreamState& S, const int32_t* rows, int B,
                          NgPart* parts, StepOut* step_out, const Outcome* out, hipStream_t s,
                          int pos = -1, const int* pos_base = nullptr);
// *p = v (one thread): the position base of a replayed encode graph
void launch_set_int(int* p, int v, hipStream_t s);
// Only the step's distribution, interval and bias step (V1-V3, V4 for the ensemble), and only
// the n-gram update kernel with the updates in A.upd.
void launch_vocab_dist(const VocabParams& P, const StreamState& S, const StepArgs& A,
                       hipStream_t s);
void launch_ngram_update(const VocabParams& P, const StreamState& S, const StepArgs& A,
                         hipStream_t s);
void launch_state_reset(const VocabParams& P, const StreamState& S, int n_streams, float w_llm,
                        hipStream_t s);
// Standalone ensemble head (C ABI): forward and backward over `rows` rows sharing b and theta.
void launch_ensemble_forward(const float* z, const float* b, const float* theta, const float* Pk,
                             const int32_t* target, int rows, int V, int nexp, float* loss,
                             float* p, float* resp, void* ws, hipStream_t s);
void launch_ensemble_backward(const float* z, float* b, float* theta, const float* resp,
                              const int32_t* target, const float* gl, int rows, int V, int nexp,
                              float lr, float* gb, float* gth, void* ws, hipStream_t s);
size_t ensemble_workspace_bytes(int rows, int V);

}  // namespace nc
