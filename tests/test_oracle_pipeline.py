"""End-to-end pins of the oracle pipeline (Algorithm 1 and its mirror) on the tiny workload."""
import numpy as np
import pytest

import synth
from oracle import pipeline as op
from oracle.cdf import quantize_counts


@pytest.fixture(scope="module")
def tiny():
    wl = synth.WORKLOADS["tiny"]
    w = synth.make_weights(wl.shape, wl.weight_seed)
    toks = synth.workload_streams(wl)[0]
    return wl, w, toks


def test_roundtrip_exact(tiny):
    wl, w, toks = tiny
    s = op.Settings.from_workload(wl)
    r = op.encode(s, wl.shape, w, toks, block=1)
    out = op.decode(s, wl.shape, w, r.data, len(toks), block=1)
    assert np.array_equal(out, toks)
    # code length: quantised length + termination (2 bits) + rounding, padded to a byte
    assert r.n_bits <= r.quant_bits + 2 + 0.01
    assert len(r.data) == (r.n_bits + 7) // 8
    # the CDF-24 floor costs little: quantised length within 0.01 bits/token of the ideal
    assert (r.quant_bits - r.ideal_bits) / len(toks) < 0.01


def test_modes_follow_warmup_and_flags(tiny):
    wl, w, toks = tiny
    s = op.Settings.from_workload(wl)
    r = op.encode(s, wl.shape, w, toks[:300], quantize=False)
    assert np.all(r.modes[:100] == op.MODE_LLM)
    assert set(np.unique(r.modes[100:])) <= {op.MODE_MIX, op.MODE_SKIP}
    r0 = op.encode(op.Settings.from_workload(wl, use_ngram=False), wl.shape, w, toks[:150],
                   quantize=False)
    assert np.all(r0.modes == op.MODE_LLM)


def test_cdf16_floor_overhead_reaches_two_bits_when_peaked():
    # section 3.4: with T = 2^16 and V = 49,152, a peaked distribution pays log2(4) = 2 bits
    v = 49152
    p = np.zeros(v, dtype=np.float32)
    p[11] = 1.0
    c16 = quantize_counts(p, total=1 << 16)
    assert abs(np.log2((1 << 16) / c16[11]) - 2.0) < 1e-4


def test_generator_statistics():
    s = synth.make_stream(20000, 512, seed=1, span=(4, 32))
    assert s.min() >= 0 and s.max() < 512
    # rank-1 probability of the bounded Zipf(1.1) law: 0.191 (V = 512) and 0.139 (V = 49,152)
    assert abs(synth._zipf_cdf(512, 1.1)[0] - 0.191) < 1e-3
    assert abs(synth._zipf_cdf(49152, 1.1)[0] - 0.139) < 1e-3
    share = np.mean(s == 0)                # copies of earlier text keep a similar mix
    assert 0.05 < share < 0.35
    wl = synth.WORKLOADS["batch64_bf16"]
    assert len(wl.lengths) == 64 and min(wl.lengths) >= 1024 and max(wl.lengths) <= 32768
    assert np.array_equal(synth.make_stream(300, 512, 9)[:100], synth.make_stream(100, 512, 9))
