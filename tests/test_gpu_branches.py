"""GPU parity of the branches the plain workloads never reach, against the FP64 oracle:

* the 64-slot eviction of the n-gram (section 3.5): a stream whose order-1 and order-2 contexts
  see far more than 64 distinct continuations, with count ties, at V = 512 and V = 49,152;
* the p_max >= 0.99 skip rule of the batched workload (section 3.8): modes and coding
  distributions at every position of a tiny stream and along a 135M-shape prefix;
* nc_mix_update through the C-ABI: alternating nc_probs_for_context and nc_mix_update reproduces
  the oracle's distribution at every position, and the intervals of its CDFs code to exactly
  the bytes nc_encode_stream writes (Algorithm 1, the update after each coded token).
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import pipeline as op
from oracle.cdf import quantize_cdf
from oracle.ngram import NGram
from tests.nc_util import gpu_available, kl_bits, make_context

pytestmark = pytest.mark.gpu

TINY = synth.WORKLOADS["tiny"]
FULL = synth.WORKLOADS["full_fp32"]
REL_PNG = 1e-5          # p_ng: integer counts, ~3 float32 operations per order


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def eviction_stream(n_rounds, vocab, seed):
    """(A, B, c) repeated: the contexts (B) and (A, B) collect ~120 distinct continuations c drawn
    from a skewed law (so stored counts differ and tie), far beyond the 64 slots."""
    rng = np.random.default_rng(seed)
    a, b = 3, 5
    pool = np.arange(10, 130) * (vocab // 512)
    w = 1.0 / np.arange(1, len(pool) + 1) ** 0.5
    c = rng.choice(pool, size=n_rounds, p=w / w.sum())
    return np.stack([np.full(n_rounds, a), np.full(n_rounds, b), c], 1).reshape(-1).astype(np.int32)


def _evictions(toks, order):
    """Number of inserts into a full 64-slot context while the oracle n-gram consumes toks."""
    ng = NGram(512 * 96, order)
    n = 0
    for i, t in enumerate(toks):
        for k in range(1, order + 1):
            if i >= k:
                sl = ng.tables[k - 1].get(tuple(int(x) for x in toks[i - k:i]))
                if sl is not None and len(sl) == 64 and all(s[0] != t for s in sl):
                    n += 1
        ng.update(toks[:i], int(t))
    return n


@pytest.mark.parametrize("wl", [TINY, FULL], ids=["V512", "V49152"])
def test_ngram_eviction_matches_oracle(wl):
    toks = eviction_stream(300, wl.shape.vocab, seed=5)
    assert _evictions(toks, wl.ngram_order) > 100
    ctx, _ = make_context(wl, max_streams=1)
    ctx.reset(1, len(toks) + 1)
    ng = NGram(wl.shape.vocab, wl.ngram_order)
    checked = 0
    for i in range(len(toks)):
        if i >= 192 and (i % 3 == 2 or i % 17 == 0):
            _, pr = ctx.probs_for_context(0, toks[:i], probe=True)
            ref = ng.predict(toks[:i])
            rel = np.abs(pr["p_ngram"].astype(np.float64) - ref) / ref
            assert rel.max() <= REL_PNG, (i, rel.max())
            checked += 1
        ng.update(toks[:i], int(toks[i]))
    assert checked >= 200


def test_eviction_stream_roundtrip_and_coded_bits():
    """Encode (the pipelined path) evicts the same way: exact round trip, and the coded bit count
    equals the oracle coder's."""
    wl = TINY
    toks = eviction_stream(300, wl.shape.vocab, seed=6)
    ctx, w = make_context(wl, max_streams=1)
    data, bits = ctx.encode_stream([toks])
    assert np.array_equal(ctx.decode_stream(data, [len(toks)])[0], toks)
    ref = op.encode(op.Settings.from_workload(wl), wl.shape, w, toks, block=1)
    assert bits[0] == ref.n_bits, (bits[0], ref.n_bits)


def _check_pmax(wl, toks, positions, oracle_block):
    ctx, w = make_context(wl, max_streams=1)
    orc = op.encode(op.Settings.from_workload(wl), wl.shape, w, toks, record=positions,
                    quantize=False, block=oracle_block)
    ctx.reset(1, len(toks) + 1)
    seen = {op.MODE_SKIP: 0, op.MODE_MIX: 0, op.MODE_LLM: 0}
    for i in positions:
        p, pr = ctx.probs_for_context(0, toks[:i], probe=True)
        rec = orc.records[i]
        assert abs(pr["pmax"] - rec["pmax"]) <= REL_PNG * rec["pmax"], i
        if pr["mode"] != rec["mode"]:
            assert abs(rec["pmax"] - 0.99) < 1e-6, (i, rec["pmax"])
            continue
        seen[rec["mode"]] += 1
        if rec["mode"] == op.MODE_SKIP:
            assert np.max(np.abs(p - rec["p"]) / rec["p"]) <= REL_PNG, i
        else:
            assert kl_bits(rec["p"], p) < 1e-6, i
        assert np.array_equal(pr["cdf"].astype(np.int64), quantize_cdf(p.astype(np.float32))), i
    return seen, orc


def test_pmax_skip_tiny_every_position():
    wl = dataclasses.replace(TINY, skip="pmax")
    toks = synth.workload_streams(TINY)[0]
    seen, orc = _check_pmax(wl, toks, list(range(len(toks))), oracle_block=1)
    assert seen[op.MODE_SKIP] >= 10 and seen[op.MODE_MIX] >= 100, seen
    ctx, w = make_context(wl, max_streams=1)
    data, bits = ctx.encode_stream([toks])
    assert np.array_equal(ctx.decode_stream(data, [len(toks)])[0], toks)
    assert (bits[0] - orc.ideal_bits) / len(toks) < 0.01


def test_pmax_skip_full_shape_prefix():
    wl = dataclasses.replace(FULL, skip="pmax")
    toks = synth.workload_streams(FULL, max_len=1200)[0]
    pos = list(range(96, 1200, 7))
    seen, _ = _check_pmax(wl, toks, pos, oracle_block=512)
    assert seen[op.MODE_SKIP] >= 10 and seen[op.MODE_MIX] >= 10, seen


def test_mix_update_through_the_abi_reproduces_encode():
    wl = TINY
    n = 400
    toks = synth.workload_streams(wl, max_len=n)[0]
    ctx, w = make_context(wl, max_streams=1)
    orc = op.encode(op.Settings.from_workload(wl), wl.shape, w, toks, record=range(n),
                    quantize=False, block=1)
    ctx.reset(1, n + 1)
    iv = np.zeros((n, 2), np.uint32)
    for i in range(n):
        p, pr = ctx.probs_for_context(0, toks[:i], probe=True)   # nothing new to commit
        rec = orc.records[i]
        assert pr["mode"] == rec["mode"], i
        assert kl_bits(rec["p"], p) < 1e-6, i
        cdf = pr["cdf"].astype(np.int64)
        assert np.array_equal(cdf, quantize_cdf(p.astype(np.float32))), i
        iv[i] = cdf[toks[i]], cdf[toks[i] + 1]
        ctx.mix_update(0, int(toks[i]))
    import paper_2602_19626_amd as nc
    data, bits = nc.ac_encode(iv)
    ref, ref_bits = ctx.encode_stream([toks])
    assert data == ref[0] and bits == ref_bits[0]
    # a committed history cannot be rewritten
    ctx.reset(1, n + 1)
    ctx.mix_update(0, int(toks[0]))
    with pytest.raises(nc.NacrithError) as e:
        ctx.probs_for_context(0, np.array([toks[0] + 1], np.int32))
    assert e.value.status == 6
