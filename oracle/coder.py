"""32-bit arithmetic coder (paper section 3.9), Witten-Neal-Cleary form, on Python integers.

The paper names the construction (range [low, high] inside [0, 2^32), emit a bit when both ends
sit in the same half, an underflow counter for straddling ranges, a 32-bit value register and a
CDF search in the decoder) but not its termination, bit order or end-of-input rule.  Readings:

- interval of symbol s: [cdf[s], cdf[s+1]) of total T; narrowing uses R = high - low + 1,
  high = low + floor(R*ch/T) - 1, low = low + floor(R*cl/T);
- renormalise: high < 2^31 -> emit 0 (+ pending 1s); low >= 2^31 -> emit 1 (+ pending 0s) and
  subtract 2^31; 2^30 <= low and high < 3*2^30 -> pending += 1 and subtract 2^30; then double
  (low = 2 low, high = 2 high + 1);
- finish: pending += 1, then emit 0 (+ pending 1s) if low < 2^30 else 1 (+ pending 0s), and pad
  the last byte with zeros;
- bits are packed most-significant first; the decoder reads zeros past the end of the input.

After every renormalisation R > 2^30 holds (not 2^31 as printed: the state low = 2^30 - 1,
high = 2^31 stops renormalising with R = 2^30 + 2).  With T = 2^24 a one-count symbol therefore
keeps a width of at least 64.

Pinned by: exhaustive round trips over every sequence of a tiny alphabet, the code-length bound
sum(-log2 c/T) + 2 termination bits + 7 padding bits (+ rounding), and the R > 2^30 invariant
(tests/test_oracle_coder.py).
"""
from __future__ import annotations

HALF = 1 << 31
Q1 = 1 << 30
Q3 = 3 << 30
TOP = (1 << 32) - 1


class Encoder:
    def __init__(self, total: int = 1 << 24):
        self.total = total
        self.low = 0
        self.high = TOP
        self.pending = 0
        self.bits = []
        self.min_range = None   # smallest R seen after a renormalisation (invariant check)

    def _emit(self, bit: int):
        self.bits.append(bit)
        self.bits.extend([1 - bit] * self.pending)
        self.pending = 0

    def encode(self, cl: int, ch: int):
        if not (0 <= cl < ch <= self.total):
            raise ValueError("empty or out-of-range interval")
        r = self.high - self.low + 1
        self.high = self.low + (r * ch) // self.total - 1
        self.low = self.low + (r * cl) // self.total
        while True:
            if self.high < HALF:
                self._emit(0)
            elif self.low >= HALF:
                self._emit(1)
                self.low -= HALF
                self.high -= HALF
            elif self.low >= Q1 and self.high < Q3:
                self.pending += 1
                self.low -= Q1
                self.high -= Q1
            else:
                break
            self.low = 2 * self.low
            self.high = 2 * self.high + 1
        r = self.high - self.low + 1
        self.min_range = r if self.min_range is None else min(self.min_range, r)

    def finish(self) -> bytes:
        self.pending += 1
        self._emit(0 if self.low < Q1 else 1)
        return self.to_bytes()

    @property
    def n_bits(self) -> int:
        return len(self.bits)

    def to_bytes(self) -> bytes:
        out = bytearray((len(self.bits) + 7) // 8)
        for i, b in enumerate(self.bits):
            if b:
                out[i >> 3] |= 0x80 >> (i & 7)
        return bytes(out)


class Decoder:
    def __init__(self, data: bytes, total: int = 1 << 24):
        self.data = data
        self.total = total
        self.pos = 0          # next bit index
        self.low = 0
        self.high = TOP
        self.value = 0
        for _ in range(32):
            self.value = (self.value << 1) | self._bit()

    def _bit(self) -> int:
        i = self.pos
        self.pos += 1
        if (i >> 3) >= len(self.data):
            return 0
        return (self.data[i >> 3] >> (7 - (i & 7))) & 1

    @property
    def overrun(self) -> bool:
        """True once more than 8*len(data) + 32 bits have been consumed (corrupt input)."""
        return self.pos > 8 * len(self.data) + 32

    def target(self) -> int:
        """The count position the next symbol's interval must contain."""
        r = self.high - self.low + 1
        return ((self.value - self.low + 1) * self.total - 1) // r

    def consume(self, cl: int, ch: int):
        r = self.high - self.low + 1
        self.high = self.low + (r * ch) // self.total - 1
        self.low = self.low + (r * cl) // self.total
        while True:
            if self.high < HALF:
                pass
            elif self.low >= HALF:
                self.low -= HALF
                self.high -= HALF
                self.value -= HALF
            elif self.low >= Q1 and self.high < Q3:
                self.low -= Q1
                self.high -= Q1
                self.value -= Q1
            else:
                break
            self.low = 2 * self.low
            self.high = 2 * self.high + 1
            self.value = 2 * self.value + self._bit()

    def decode(self, cdf) -> int:
        """Decode one symbol against an integer CDF (cdf[0] = 0, cdf[-1] = total)."""
        t = self.target()
        # largest s with cdf[s] <= t, by binary search over the CDF
        lo, hi = 0, len(cdf) - 2
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if cdf[mid] <= t:
                lo = mid
            else:
                hi = mid - 1
        self.consume(int(cdf[lo]), int(cdf[lo + 1]))
        return lo


def encode_intervals(intervals, total: int = 1 << 24):
    """Encode a list of (cl, ch) intervals; returns (bytes, exact bit count)."""
    enc = Encoder(total)
    for cl, ch in intervals:
        enc.encode(int(cl), int(ch))
    data = enc.finish()
    return data, enc.n_bits
