"""CDF-24 quantisation (paper section 3.4, "CDF-24 upgrade"), exact integer arithmetic.

Definition followed: every symbol gets c_i = max(1, floor(p_i * (T - V))) counts, where T is the
CDF total (2^24) and V the alphabet size; the residual T - sum(c) (which may be negative when the
float probabilities sum to slightly more than one) is added to the count of the most probable
symbol.  The argmax takes the lowest index among equal maxima.  The CDF is the exclusive prefix sum
of the counts, so cdf[0] = 0 and cdf[V] = T.

T - V is always computed; the paper's printed remainder for V = 49,152 is off by 1,000
(16,728,064 is the true value).

The floor is the exact floor of the real product p_i * (T - V): for float32 inputs the binary64
product is exact (a 24-bit significand times an integer below 2^24 needs at most 48 bits); for
float64 inputs the significand is taken as an exact integer and the product is formed on Python
integers.

Pinned by: the paper's closed forms (floor share V/T, the 2-bit and 0.004233-bit overheads),
hand-derived uniform and one-hot cases, and brute force against ``fractions.Fraction`` on tiny
alphabets (tests/test_oracle_cdf.py).
"""
from __future__ import annotations

import numpy as np


def _floor_scaled(p: np.ndarray, m: int) -> np.ndarray:
    """Exact floor(p * m) for non-negative float32/float64 p and integer 0 < m < 2^24."""
    if p.dtype == np.float32:
        return np.floor(p.astype(np.float64) * float(m)).astype(np.int64)
    if p.dtype != np.float64:
        raise TypeError("probabilities must be float32 or float64")
    # p = mant * 2^(exp - 53) with mant a 53-bit integer; floor(p*m) = (mant*m) >> (53 - exp).
    mant, exp = np.frexp(p)
    mant_i = (mant * float(1 << 53)).astype(np.int64)          # exact: mant in [0.5, 1)
    shift = 53 - exp.astype(np.int64)
    if np.any(shift < 0):
        raise ValueError("probability too large")
    prod = mant_i.astype(object) * int(m)                       # Python integers: no overflow
    return np.right_shift(prod, shift.astype(object)).astype(np.int64)


def quantize_counts(p: np.ndarray, total: int = 1 << 24) -> np.ndarray:
    """Integer counts c[V] (int64) of the CDF-24 quantiser for one distribution p[V]."""
    p = np.asarray(p)
    if p.ndim != 1:
        raise ValueError("p must be one-dimensional")
    v = p.shape[0]
    if v < 1 or v >= total:
        raise ValueError("need 1 <= V < T")
    if not np.all(np.isfinite(p)) or np.any(p < 0):
        raise ValueError("probabilities must be finite and non-negative")
    m = total - v
    c = np.maximum(1, _floor_scaled(p, m))
    a = int(np.argmax(p))                      # numpy returns the first maximal index
    c[a] += total - int(c.sum())
    if c[a] < 1:
        raise ValueError("probability mass exceeds the CDF total")
    return c


def quantize_cdf(p: np.ndarray, total: int = 1 << 24) -> np.ndarray:
    """cdf[V+1] (int64) with cdf[0] = 0, cdf[V] = total, from quantize_counts()."""
    c = quantize_counts(p, total)
    cdf = np.zeros(c.shape[0] + 1, dtype=np.int64)
    np.cumsum(c, out=cdf[1:])
    return cdf


def code_bits(count: int, total: int = 1 << 24) -> float:
    """Ideal cost in bits of coding a symbol that owns `count` of `total` CDF counts."""
    return float(np.log2(total) - np.log2(count))
