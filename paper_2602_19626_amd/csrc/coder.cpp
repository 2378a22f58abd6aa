// Host arithmetic coder; see coder.hpp for the exact rules.
#include "coder.hpp"

namespace nc {

static constexpr uint64_t kHalf = 1ull << 31, kQ1 = 1ull << 30, kQ3 = 3ull << 30;

void ArithEncoder::emit(unsigned bit) {
  w_.put(bit);
  for (; pending_ > 0; --pending_) w_.put(bit ^ 1u);
}

void ArithEncoder::encode(uint32_t cl, uint32_t ch) {
  const uint64_t r = high_ - low_ + 1;
  high_ = low_ + (r * ch) / total_ - 1;
  low_ = low_ + (r * cl) / total_;
  for (;;) {
    if (high_ < kHalf) {
      emit(0);
    } else if (low_ >= kHalf) {
      emit(1);
      low_ -= kHalf;
      high_ -= kHalf;
    } else if (low_ >= kQ1 && high_ < kQ3) {
      ++pending_;
      low_ -= kQ1;
      high_ -= kQ1;
    } else {
      break;
    }
    low_ <<= 1;
    high_ = (high_ << 1) | 1u;
  }
}

void ArithEncoder::finish() {
  ++pending_;
  emit(low_ < kQ1 ? 0u : 1u);
}

ArithDecoder::ArithDecoder(const uint8_t* data, size_t nbytes, uint32_t total)
    : data_(data), nbytes_(nbytes), total_(total) {
  for (int i = 0; i < 32; ++i) value_ = (value_ << 1) | next_bit();
}

void ArithDecoder::consume(uint32_t cl, uint32_t ch) {
  const uint64_t r = high_ - low_ + 1;
  high_ = low_ + (r * ch) / total_ - 1;
  low_ = low_ + (r * cl) / total_;
  for (;;) {
    if (high_ < kHalf) {
      // nothing to subtract
    } else if (low_ >= kHalf) {
      low_ -= kHalf;
      high_ -= kHalf;
      value_ -= kHalf;
    } else if (low_ >= kQ1 && high_ < kQ3) {
      low_ -= kQ1;
      high_ -= kQ1;
      value_ -= kQ1;
    } else {
      break;
    }
    low_ <<= 1;
    high_ = (high_ << 1) | 1u;
    value_ = (value_ << 1) | next_bit();
  }
}

}  // namespace nc
