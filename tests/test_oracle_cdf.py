"""Pins of the oracle's CDF-24 quantiser (paper section 3.4) against printed values, closed forms
and brute force in exact rational arithmetic."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.cdf import code_bits, quantize_cdf, quantize_counts

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
T24 = 1 << 24


def test_printed_floor_shares():
    v = GOLD["vocab"]["value"]
    assert v / 65536 == GOLD["cdf16_floor_share"]["value"]                       # exactly 75%
    assert 65536 - v == GOLD["cdf16_left_for_information"]["value"]
    assert math.log2(65536 / (65536 - v)) == GOLD["cdf16_overhead_bits"]["value"]
    assert round(100 * v / T24, 2) == GOLD["cdf24_floor_share_percent"]["value"]
    assert v / T24 == 0.0029296875
    over = math.log2(T24 / (T24 - v))
    assert abs(over - 0.004233) < 5e-7
    assert round(over, 3) == GOLD["cdf24_overhead_bits_approx"]["value"]


def test_remaining_bins_is_computed_not_printed():
    v = GOLD["vocab"]["value"]
    assert T24 - v == 16_728_064
    assert T24 - v - GOLD["cdf24_remaining_bins_printed"]["value"] == 1000


def test_uniform_512_worked_example():
    p = np.full(512, 2.0 ** -9, dtype=np.float32)
    c = quantize_counts(p)
    assert c[0] == 33279 and np.all(c[1:] == 32767)
    cdf = quantize_cdf(p)
    assert cdf[0] == 0 and cdf[-1] == T24


def test_uniform_full_vocab_worked_example():
    p = np.full(49152, 1.0 / 49152, dtype=np.float32)
    c = quantize_counts(p)
    assert np.all(c[1:] == 340)
    assert int(c[1:].sum()) + 340 == 16_711_680
    assert c[0] == 65_876


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_one_hot_costs_the_floor_overhead(dtype):
    v, k = 49152, 777
    p = np.zeros(v, dtype=dtype)
    p[k] = 1.0
    c = quantize_counts(p)
    assert c[k] == T24 - v + 1 == 16_728_065
    assert np.all(np.delete(c, k) == 1)
    assert abs(code_bits(int(c[k])) - 0.004233) < 5e-6


def test_residual_goes_to_lowest_argmax():
    p = np.array([0.25, 0.375, 0.375, 0.0], dtype=np.float32)
    c = quantize_counts(p, total=1 << 10)
    base = [max(1, math.floor(Fraction(float(x)) * (1020))) for x in p]
    assert list(c) == [base[0], base[1] + (1024 - sum(base)), base[2], base[3]]


def _fraction_reference(p, total):
    v = len(p)
    m = total - v
    c = [max(1, math.floor(Fraction(float(x)) * m)) for x in p]
    a = max(range(v), key=lambda i: (Fraction(float(p[i])), -i))
    c[a] += total - sum(c)
    return c


@pytest.mark.parametrize("v,total", [(2, 16), (3, 64), (4, 256)])
def test_brute_force_grid_vs_fractions(v, total):
    grid = [i / 16 for i in range(17)] + [1 / 3, 0.1, 0.7]
    for tup in itertools.product(grid, repeat=v):
        if sum(tup) > 1.0 + 1e-12 or sum(tup) == 0:
            continue
        for dt in (np.float32, np.float64):
            p = np.array(tup, dtype=dt)
            ref = _fraction_reference(p, total)
            if ref[int(np.argmax(p))] < 1:
                with pytest.raises(ValueError):
                    quantize_counts(p, total)
                continue
            assert list(quantize_counts(p, total)) == ref


def test_float64_floor_is_exact_at_integer_boundaries():
    # p*m lands within one ulp of the integer k: a rounded binary64 product would give k for
    # the value just below, the exact floor gives k - 1.
    m = T24 - 3
    k = 12345
    x = float(Fraction(k, m))
    below = float(np.nextafter(x, -1.0))
    above = float(np.nextafter(x, 2.0))
    assert Fraction(below) * m < k <= Fraction(above) * m
    for val in (x, below, above):
        arr = np.array([val, 0.0, 1.0 - val], dtype=np.float64)
        c = quantize_counts(arr)
        assert c[0] == math.floor(Fraction(val) * m)
    assert quantize_counts(np.array([below, 0.0, 1.0 - below]))[0] == k - 1


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_invariants_random(seed, dt):
    rng = np.random.default_rng(seed)
    v = int(rng.integers(2, 3000))
    p = rng.dirichlet(np.full(v, 0.05)).astype(dt)
    cdf = quantize_cdf(p)
    assert cdf[0] == 0 and cdf[-1] == T24
    assert np.all(np.diff(cdf) >= 1)
    ref = _fraction_reference(p, T24) if v <= 300 else None
    if ref is not None:
        assert list(np.diff(cdf)) == ref


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        quantize_counts(np.array([0.5, np.nan], dtype=np.float32))
    with pytest.raises(ValueError):
        quantize_counts(np.array([0.5, -0.1], dtype=np.float32))
    with pytest.raises(ValueError):
        quantize_counts(np.ones(8, dtype=np.float32), total=16)   # mass far above one
