// extern "C" entry points of libnacrith: argument checking and error translation only; the work
// happens in the kernels (k_*.hip), the host coder (coder.cpp) and the runtime (runtime.cpp).
#include <cstring>
#include <mutex>
#include <string>
#include <map>
#include <utility>
#include <vector>

#include "coder.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "vocab_dev.hpp"

namespace nc {
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

// Device workspace of the context-free calls: one buffer per (device, stream).  Work queued on one
// stream runs in order, so calls on the same stream can share a buffer; calls on different streams
// never do.  The lock is held until the launch is queued, and a buffer that must grow is freed
// only after its stream has drained, so no queued kernel can lose its workspace.
template <class Launch>
static void with_workspace(hipStream_t stream, size_t bytes, Launch&& launch) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, std::pair<void*, size_t>> bufs;
  int dev = 0;
  NC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto& b = bufs[{dev, stream}];
  if (b.second < bytes) {
    if (b.first) {
      NC_HIP(hipStreamSynchronize(stream));
      NC_HIP(hipFree(b.first));
    }
    b.first = nullptr;
    b.second = 0;
    NC_HIP(hipMalloc(&b.first, bytes));
    b.second = bytes;
  }
  launch(b.first);
}
}  // namespace nc

using namespace nc;

extern "C" {

const char* nc_last_error(void) { return g_last_error.c_str(); }

size_t nc_encode_bound(size_t n_tokens) { return encode_bound(n_tokens); }

nc_status nc_quantize_cdf24(const float* probs, uint32_t rows, uint32_t vocab, uint32_t total,
                            uint32_t* cdf, int32_t* row_status, void* stream) {
  return guard([&] {
    NC_CHECK(probs && cdf, NC_E_INVALID, "NULL pointer");
    NC_CHECK(vocab >= 1 && vocab <= 262144u, NC_E_INVALID, "vocab must be in [1, 262144]");
    NC_CHECK(total > vocab && total <= (1u << 24), NC_E_INVALID,
             "total must satisfy vocab < total <= 2^24");
    if (rows == 0) return;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    with_workspace(st, quantize_workspace_bytes(rows, vocab), [&](void* ws) {
      launch_quantize_cdf(probs, rows, vocab, total, cdf, row_status, ws, st);
    });
  });
}

nc_status nc_quantize_cdf24_noalloc(const float* probs, uint32_t rows, uint32_t vocab,
                                    uint32_t total, uint32_t* cdf, int32_t* row_status,
                                    void* stream) {
  return guard([&] {
    NC_CHECK(probs && cdf, NC_E_INVALID, "NULL pointer");
    NC_CHECK(vocab >= 1 && vocab <= 262144u, NC_E_INVALID, "vocab must be in [1, 262144]");
    NC_CHECK(total > vocab && total <= (1u << 24), NC_E_INVALID,
             "total must satisfy vocab < total <= 2^24");
    if (rows == 0) return;
    const size_t need = quantize_workspace_needed(probs, rows, vocab);
    NC_CHECK(need <= kScratchBytes, NC_E_CAPACITY,
             "rows * ceil(vocab / 4096) = %zu segment partials exceed the %zu of the fixed "
             "scratch array (the segment path runs for up to 64 rows, unaligned rows or "
             "vocab > 49,152)", need / 16, kScratchParts);
    launch_quantize_cdf(probs, rows, vocab, total, cdf, row_status,
                        need ? quantize_scratch_address() : nullptr,
                        static_cast<hipStream_t>(stream));
  });
}

nc_status nc_cdf_interval(const uint32_t* cdf, uint32_t rows, uint32_t vocab, const uint32_t* key,
                          int32_t mode, uint32_t* out, void* stream) {
  return guard([&] {
    NC_CHECK(cdf && key && out, NC_E_INVALID, "NULL pointer");
    NC_CHECK(vocab >= 1, NC_E_INVALID, "vocab must be >= 1");
    NC_CHECK(mode == 0 || mode == 1, NC_E_INVALID, "mode must be 0 (encode) or 1 (decode)");
    launch_cdf_interval(cdf, rows, vocab, key, mode, out, static_cast<hipStream_t>(stream));
  });
}

nc_status nc_ac_encode(const uint32_t* intervals, size_t n, uint32_t total, uint8_t* out,
                       size_t cap, size_t* out_bytes, uint64_t* out_bits) {
  return guard([&] {
    NC_CHECK(out_bytes && out_bits && (n == 0 || intervals), NC_E_INVALID, "NULL pointer");
    NC_CHECK(total >= 2 && total <= (1u << 24), NC_E_INVALID, "total must be in [2, 2^24]");
    for (size_t i = 0; i < n; ++i)
      NC_CHECK(intervals[2 * i] < intervals[2 * i + 1] && intervals[2 * i + 1] <= total,
               NC_E_INVALID, "interval %zu is empty or out of range", i);
    std::vector<uint8_t> buf;
    buf.reserve(encode_bound(n));
    ArithEncoder enc(&buf, total);
    for (size_t i = 0; i < n; ++i) enc.encode(intervals[2 * i], intervals[2 * i + 1]);
    enc.finish();
    *out_bits = enc.bits();
    *out_bytes = buf.size();
    NC_CHECK(out && cap >= buf.size(), NC_E_CAPACITY, "output needs %zu bytes", buf.size());
    std::memcpy(out, buf.data(), buf.size());
  });
}

nc_status nc_ac_decode_static(const uint8_t* in, size_t in_bytes, const uint32_t* cdf,
                              uint32_t vocab, size_t n, int32_t* out) {
  return guard([&] {
    NC_CHECK(cdf && (n == 0 || out) && (in_bytes == 0 || in), NC_E_INVALID, "NULL pointer");
    NC_CHECK(vocab >= 1 && cdf[0] == 0 && cdf[vocab] <= (1u << 24), NC_E_INVALID, "bad cdf");
    for (uint32_t s = 0; s < vocab; ++s)
      NC_CHECK(cdf[s] < cdf[s + 1], NC_E_INVALID, "cdf must be strictly increasing");
    ArithDecoder dec(in, in_bytes, cdf[vocab]);
    for (size_t i = 0; i < n; ++i) {
      const uint32_t t = dec.target();
      uint32_t lo = 0, hi = vocab - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (cdf[mid] <= t)
          lo = mid;
        else
          hi = mid - 1;
      }
      dec.consume(cdf[lo], cdf[lo + 1]);
      NC_CHECK(!dec.overrun(), NC_E_CORRUPT, "decoder ran past the end of the input");
      out[i] = int32_t(lo);
    }
  });
}

nc_status nc_ensemble_forward(const float* z, const float* b, const float* theta,
                              const float* P, const int32_t* target, uint32_t rows,
                              uint32_t vocab, uint32_t n_experts, float* loss, float* p,
                              float* resp, void* stream) {
  return guard([&] {
    NC_CHECK(z && b && theta && target && resp && (n_experts == 1 || P), NC_E_INVALID,
             "NULL pointer");
    NC_CHECK(n_experts >= 1 && n_experts <= kMaxExperts, NC_E_INVALID, "n_experts in [1, 8]");
    NC_CHECK(vocab >= 1 && vocab <= 262144u, NC_E_INVALID, "vocab must be in [1, 262144]");
    if (rows == 0) return;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    with_workspace(st, ensemble_workspace_bytes(int(rows), int(vocab)), [&](void* ws) {
      launch_ensemble_forward(z, b, theta, P, target, int(rows), int(vocab), int(n_experts), loss,
                              p, resp, ws, st);
    });
  });
}

nc_status nc_ensemble_backward(const float* z, float* b, float* theta, const float* resp,
                               const int32_t* target, const float* grad_loss, uint32_t rows,
                               uint32_t vocab, uint32_t n_experts, float lr, float* grad_b,
                               float* grad_theta, void* stream) {
  return guard([&] {
    NC_CHECK(z && b && theta && resp && target && grad_loss, NC_E_INVALID, "NULL pointer");
    NC_CHECK(n_experts >= 1 && n_experts <= kMaxExperts, NC_E_INVALID, "n_experts in [1, 8]");
    NC_CHECK(vocab >= 1 && vocab <= 262144u, NC_E_INVALID, "vocab must be in [1, 262144]");
    if (rows == 0) return;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    with_workspace(st, ensemble_workspace_bytes(int(rows), int(vocab)), [&](void* ws) {
      launch_ensemble_backward(z, b, theta, resp, target, grad_loss, int(rows), int(vocab),
                               int(n_experts), lr, grad_b, grad_theta, ws, st);
    });
  });
}

}  // extern "C"
