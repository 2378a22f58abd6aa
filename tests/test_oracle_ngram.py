"""Pins of the oracle's token n-gram (paper section 3.5)."""
from fractions import Fraction

import numpy as np

from oracle.ngram import NGram


def test_empty_model_is_uniform():
    ng = NGram(vocab=37, order=4)
    p = ng.predict([])
    assert np.allclose(p, 1.0 / 37, rtol=0, atol=1e-15)


def test_hand_worked_sequence():
    # history 1,2,1,2,1 over V = 4, orders 1..2, eps = 5 (worked by hand):
    #   c = (0,3,2,0), N = 5          -> P0 = (1/9, 4/9, 3/9, 1/9)
    #   order 1, context (1,): {2: 2} -> lambda = 2/7, P1 = 2/7 e_2 + 5/7 P0
    #   order 2, context (2,1): {2:1} -> lambda = 1/6, P2 = 1/6 e_2 + 5/6 P1
    ng = NGram(vocab=4, order=2)
    hist = []
    for t in [1, 2, 1, 2, 1]:
        ng.update(hist, t)
        hist.append(t)
    p0, p1, p2 = ng.predict_all(hist)
    want0 = [Fraction(1, 9), Fraction(4, 9), Fraction(3, 9), Fraction(1, 9)]
    want1 = [Fraction(5, 63), Fraction(20, 63), Fraction(33, 63), Fraction(5, 63)]
    want2 = [Fraction(25, 378), Fraction(100, 378), Fraction(228, 378), Fraction(25, 378)]
    for got, want in ((p0, want0), (p1, want1), (p2, want2)):
        assert np.allclose(got, [float(w) for w in want], rtol=0, atol=1e-15)
    assert ng.tables[0][(1,)] == [[2, 2]]
    assert ng.tables[0][(2,)] == [[1, 2]]
    assert ng.tables[1][(1, 2)] == [[1, 2]]
    assert ng.tables[1][(2, 1)] == [[2, 1]]


def test_absent_context_leaves_lower_order():
    ng = NGram(vocab=10, order=3)
    hist = []
    for t in [3, 4, 5]:
        ng.update(hist, t)
        hist.append(t)
    p = ng.predict_all([9, 9, 9])              # no stored context of any order
    assert np.array_equal(p[0], p[3])


def test_slot_cap_evicts_lowest_count_lowest_index():
    ng = NGram(vocab=200, order=1, slots=64)
    ctx = [7]
    for t in range(64):                         # 64 distinct continuations of context (7,)
        ng.update(ctx, 100 + t)
    ng.update(ctx, 100 + 5)                      # slot 5 now has count 2
    ng.update(ctx, 42)                           # full: evict the lowest count, lowest index = 0
    slots = ng.tables[0][(7,)]
    assert len(slots) == 64
    assert slots[0] == [42, 1]
    assert slots[5] == [105, 2]
    ng.update(ctx, 43)                           # next eviction: slot 0 again (count 1, index 0)
    assert ng.tables[0][(7,)][0] == [43, 1]


def test_capacity_cap_stops_new_contexts():
    ng = NGram(vocab=50, order=1, max_contexts=3)
    hist = []
    for t in [1, 2, 3, 4, 5]:
        ng.update(hist, t)
        hist.append(t)
    assert len(ng.tables[0]) == 3
    assert (4,) not in ng.tables[0]


def test_distributions_sum_to_one():
    rng = np.random.default_rng(0)
    ng = NGram(vocab=64, order=4)
    hist = []
    for t in rng.integers(0, 8, size=500):
        ng.update(hist, int(t))
        hist.append(int(t))
        if len(hist) % 50 == 0:
            for p in ng.predict_all(hist):
                assert abs(p.sum() - 1.0) < 1e-12 and p.min() > 0
