// 32-bit Witten-Neal-Cleary arithmetic coder (paper section 3.9), host side.
//
// Interval of a symbol: [cl, ch) out of total T.  Narrowing: R = high - low + 1,
// high = low + floor(R ch / T) - 1, low = low + floor(R cl / T).  Renormalisation: high < 2^31
// emits 0 (then the pending opposite bits), low >= 2^31 emits 1 and subtracts 2^31, a range
// straddling the middle inside [2^30, 3 2^30) increments the pending count and subtracts 2^30;
// each case doubles the range.  Finish: one more pending bit, then 0 if low < 2^30 else 1,
// followed by the pending bits; the last byte is zero-padded; bits are packed MSB first and the
// decoder reads zeros past the end of its input.  R > 2^30 holds after every renormalisation, so
// with T <= 2^24 every one-count symbol keeps a non-empty interval.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace nc {

class BitWriter {
 public:
  explicit BitWriter(std::vector<uint8_t>* out) : out_(out) {}
  void put(unsigned bit) {
    if ((nbits_ & 7) == 0) out_->push_back(0);
    if (bit) out_->back() |= uint8_t(0x80u >> (nbits_ & 7));
    ++nbits_;
  }
  uint64_t bits() const { return nbits_; }

 private:
  std::vector<uint8_t>* out_;
  uint64_t nbits_ = 0;
};

class ArithEncoder {
 public:
  ArithEncoder(std::vector<uint8_t>* out, uint32_t total) : w_(out), total_(total) {}
  void encode(uint32_t cl, uint32_t ch);
  void finish();
  uint64_t bits() const { return w_.bits(); }

 private:
  void emit(unsigned bit);
  BitWriter w_;
  uint64_t total_;
  uint64_t low_ = 0, high_ = 0xFFFFFFFFull, pending_ = 0;
};

class ArithDecoder {
 public:
  ArithDecoder(const uint8_t* data, size_t nbytes, uint32_t total);
  // Count position that the next symbol's interval contains.
  uint32_t target() const {
    if (value_ < low_) return 0;  // only reachable on corrupt input
    uint64_t r = high_ - low_ + 1;
    uint64_t t = ((value_ - low_ + 1) * total_ - 1) / r;
    return t >= total_ ? uint32_t(total_ - 1) : uint32_t(t);
  }
  void consume(uint32_t cl, uint32_t ch);
  bool overrun() const { return pos_ > 8 * uint64_t(nbytes_) + 32; }

 private:
  unsigned next_bit() {
    uint64_t i = pos_++;
    if ((i >> 3) >= nbytes_) return 0;
    return (data_[i >> 3] >> (7 - (i & 7))) & 1u;
  }
  const uint8_t* data_;
  size_t nbytes_;
  uint64_t total_;
  uint64_t pos_ = 0;
  uint64_t low_ = 0, high_ = 0xFFFFFFFFull, value_ = 0;
};

inline size_t encode_bound(size_t n_tokens) { return (25 * n_tokens + 64 + 7) / 8; }

}  // namespace nc
