"""Pins of the oracle's 32-bit arithmetic coder (paper section 3.9 / 3.4 Safety)."""
import itertools
import math

import numpy as np
import pytest

from oracle.coder import HALF, Q1, Decoder, Encoder, encode_intervals


def _random_cdf(rng, v, total):
    cuts = np.sort(rng.choice(np.arange(1, total), size=v - 1, replace=False))
    return np.concatenate([[0], cuts, [total]]).astype(np.int64)


def _roundtrip(seq, cdf, total):
    data, nbits = encode_intervals([(cdf[s], cdf[s + 1]) for s in seq], total)
    dec = Decoder(data, total)
    return [dec.decode(cdf) for _ in seq], data, nbits


def test_binary_uniform_code_is_the_identity_on_bits():
    # With T = 2 and cdf (0, 1, 2) every symbol halves the range, so the coder emits the symbol
    # bits themselves, then the two termination bits "01".
    bits = [1, 0, 0, 1, 1, 1, 0, 1, 0, 0, 1]
    enc = Encoder(total=2)
    for b in bits:
        enc.encode(b, b + 1)
    enc.finish()
    assert enc.bits == bits + [0, 1]


@pytest.mark.parametrize("n", range(1, 8))
def test_exhaustive_roundtrip_v3(n):
    rng = np.random.default_rng(n)
    for total in (1 << 24, 97):
        cdf = _random_cdf(rng, 3, total)
        for seq in itertools.product(range(3), repeat=n):
            out, _, _ = _roundtrip(list(seq), cdf, total)
            assert out == list(seq)


def test_roundtrip_with_one_count_symbols_and_bound():
    rng = np.random.default_rng(7)
    total = 1 << 24
    v = 300
    counts = np.ones(v, dtype=np.int64)
    counts[0] = total - (v - 1)                     # a one-hot-like CDF with 1-count symbols
    cdf = np.concatenate([[0], np.cumsum(counts)])
    seq = list(rng.integers(0, v, size=400))        # mostly 1-count symbols: ~24 bits each
    out, data, nbits = _roundtrip(seq, cdf, total)
    assert out == seq
    ideal = sum(math.log2(total / counts[s]) for s in seq)
    # each narrowing loses at most log2(1/(1 - T/(c R))) with R > 2^30 (count c >= 1)
    rounding = sum(-math.log2(1 - total / (counts[s] * 2.0 ** 30)) for s in seq)
    assert nbits <= ideal + rounding + 2
    assert len(data) * 8 - nbits < 8


@pytest.mark.parametrize("seed", range(4))
def test_code_length_bound_and_min_range(seed):
    rng = np.random.default_rng(100 + seed)
    total = 1 << 24
    v = 1000
    p = rng.dirichlet(np.full(v, 0.1))
    counts = np.maximum(1, np.floor(p * (total - v))).astype(np.int64)
    counts[np.argmax(counts)] += total - counts.sum()
    cdf = np.concatenate([[0], np.cumsum(counts)])
    seq = rng.choice(v, size=3000, p=counts / total)
    enc = Encoder(total)
    for s in seq:
        enc.encode(int(cdf[s]), int(cdf[s + 1]))
    assert enc.min_range > (1 << 30)                 # the renormalisation invariant
    enc.finish()
    ideal = float(np.sum(np.log2(total / counts[seq])))
    rounding = float(np.sum(-np.log2(1 - total / (counts[seq] * 2.0 ** 30))))
    assert enc.n_bits <= ideal + rounding + 2
    dec = Decoder(enc.to_bytes(), total)
    assert [dec.decode(cdf) for _ in seq] == list(seq)


def test_range_after_renormalisation_can_be_just_above_2_30():
    # low = 2^30 - 1, high = 2^31 is a state at which renormalisation stops (neither end is in a
    # single half and low < Q1), with R = 2^30 + 2: the printed "R >= 2^31" does not hold, so a
    # one-count symbol at T = 2^24 keeps a width of at least 64, not 128.
    low, high = Q1 - 1, HALF
    assert not (high < HALF) and not (low >= HALF) and not (low >= Q1 and high < 3 * Q1)
    r = high - low + 1
    assert r == (1 << 30) + 2
    assert r // (1 << 24) == 64


def test_decoder_reads_zeros_past_end_and_reports_overrun():
    dec = Decoder(b"", 1 << 24)
    assert dec.value == 0
    cdf = [0, 1, 1 << 24]
    for _ in range(40):
        dec.decode(cdf)
    assert dec.overrun
