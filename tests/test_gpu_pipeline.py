"""GPU parity of the whole per-token pipeline against the FP64 oracle (tiny 2-layer workload):
logits, bias head, n-gram, mixer, modes, CDF-24 on the GPU's own probabilities, exact round trip,
and batch invariance of the coded bytes."""
import numpy as np
import pytest

import synth
from oracle import pipeline as op
from oracle.cdf import quantize_cdf
from tests.nc_util import gpu_available, kl_bits, make_context

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["tiny"]
POS = [0, 1, 5, 99, 100, 101, 127, 128, 129, 160, 300, 777, 1500, 2047]


@pytest.fixture(scope="module")
def setup():
    if not gpu_available():
        pytest.skip("no GPU")
    toks = synth.workload_streams(WL)[0]
    ctx, w = make_context(WL)
    orc = op.encode(op.Settings.from_workload(WL), WL.shape, w, toks, record=POS, block=1,
                    quantize=False)
    return ctx, w, toks, orc


def test_logits_and_distributions_match_oracle(setup):
    ctx, w, toks, orc = setup
    ctx.reset(1, len(toks) + 1)
    worst_z = 0.0
    for i in POS:
        p, pr = ctx.probs_for_context(0, toks[:i], probe=True)
        rec = orc.records[i]
        assert pr["mode"] == rec["mode"], i
        if rec["mode"] != op.MODE_SKIP:
            worst_z = max(worst_z, float(np.max(np.abs(pr["logits"] - rec["z"]))))
            assert np.max(np.abs(pr["ptilde"] - rec["ptilde"])) < 1e-5
        if rec.get("p_ng") is not None:
            assert np.max(np.abs(pr["p_ngram"] - rec["p_ng"])) < 1e-6
            assert abs(pr["entropy_bits"] - rec["entropy"]) < 1e-3
        assert np.max(np.abs(p - rec["p"])) < 1e-5
        assert kl_bits(rec["p"], p) < 1e-6
        # CDF-24 on the GPU's own float32 probabilities is bit-exact with the oracle quantiser
        assert np.array_equal(pr["cdf"].astype(np.int64), quantize_cdf(p.astype(np.float32)))
        assert pr["cdf"][-1] == 1 << 24
    assert worst_z < 1e-3


def test_encode_decode_roundtrip_and_gap(setup):
    ctx, w, toks, orc = setup
    data, bits = ctx.encode_stream([toks])
    st = ctx.stats()
    assert st["tokens"] == len(toks)
    out = ctx.decode_stream(data, [len(toks)])
    assert np.array_equal(out[0], toks)
    gap = (bits[0] - orc.ideal_bits) / len(toks)
    assert gap < 0.01, gap
    # the same bit count as the oracle coder on its own FP64 distributions
    ref = op.encode(op.Settings.from_workload(WL), WL.shape, w, toks, block=1)
    assert bits[0] == ref.n_bits, (bits[0], ref.n_bits)
    # re-encoding gives the same bytes (deterministic)
    data2, bits2 = ctx.encode_stream([toks])
    assert data2 == data and bits2 == bits


def test_batch_invariance_of_coded_bytes(setup):
    ctx, w, toks, orc = setup
    streams = [synth.make_stream(n, WL.shape.vocab, seed=s, span=WL.span)
               for n, s in ((700, 11), (1300, 12), (257, 13))]
    alone = [ctx.encode_stream([s])[0][0] for s in streams]
    import paper_2602_19626_amd as nc
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32", skip=WL.skip,
                         mix_init=WL.mix_init, max_streams=3)
    big = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    together, _ = big.encode_stream(streams)
    assert together == alone
    dec = big.decode_stream(together, [len(s) for s in streams])
    for a, b in zip(dec, streams):
        assert np.array_equal(a, b)


ABLATION_RUNGS = [  # the paper's feature ladder (ablation table), plus two single switches
    dict(cdf_total=1 << 16, use_head=False, use_ngram=False, use_skip=False, use_mixer=False),
    dict(cdf_total=1 << 24, use_head=False, use_ngram=False, use_skip=False, use_mixer=False),
    dict(cdf_total=1 << 24, use_head=True, use_ngram=False, use_skip=False, use_mixer=False),
    dict(cdf_total=1 << 24, use_head=True, use_ngram=True, use_skip=True, use_mixer=False),
    dict(cdf_total=1 << 24, use_head=True, use_ngram=True, use_skip=True, use_mixer=True),
    dict(use_head=False),
    dict(use_skip=False),
]


@pytest.mark.parametrize("over", ABLATION_RUNGS, ids=["A0", "A1", "A2", "A3", "A4", "nohead",
                                                      "noskip"])
def test_ablation_switches_roundtrip(setup, over):
    """Each switch set round-trips exactly and codes within 0.01 bits/token of the oracle coder
    on the oracle's own distributions with the same switches (the 2^16 CDF included).  Exact
    equality is not implied: where an FP32 probability and the FP64 one straddle a quantisation
    step, one count differs by one (the 2^16 rung codes 4,484 bits here against 4,483)."""
    ctx, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    t = toks[:600]
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, skip=WL.skip,
                         mix_init=WL.mix_init, warmup=WL.warmup, head_lr=WL.head_lr, **over)
    c = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    data, bits = c.encode_stream([t])
    assert np.array_equal(c.decode_stream(data, [len(t)])[0], t), over
    ref = op.encode(op.Settings.from_workload(WL, **over), WL.shape, w, t, block=1)
    assert abs(bits[0] - ref.n_bits) <= 0.01 * len(t), (over, bits[0], ref.n_bits)


def test_error_paths(setup):
    ctx, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    with pytest.raises(nc.NacrithError) as e:
        ctx.encode_stream([np.array([1, 2, 512], np.int32)])
    assert e.value.status == 1
    data, _ = ctx.encode_stream([toks[:200]])
    with pytest.raises(nc.NacrithError) as e:
        ctx.decode_stream([data[0][:3]], [200])       # truncated stream: decoder overrun
    assert e.value.status in (5,)


def test_wide_batch_matches_streams_alone(setup):
    """40 streams coded together give each stream the bytes it gets when coded alone."""
    ctx, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    n = 40
    streams = [synth.make_stream(96 + 3 * i, WL.shape.vocab, seed=300 + i, span=WL.span)
               for i in range(n)]
    alone = [ctx.encode_stream([s])[0][0] for s in streams[:6]]
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32", skip=WL.skip,
                         mix_init=WL.mix_init, max_streams=n)
    big = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    together, _ = big.encode_stream(streams)
    assert together[:6] == alone
    dec = big.decode_stream(together, [len(s) for s in streams])
    for a, b in zip(dec, streams):
        assert np.array_equal(a, b)


def test_nc05_container_round_trip(setup):
    _, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    from paper_2602_19626_amd import container as ct
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32", skip=WL.skip,
                         mix_init=WL.mix_init, max_streams=3)
    ctx = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    streams = [toks[:500], toks[500:777], toks[777:780]]
    blob = ct.compress(ctx, streams, ct.config_flags(ctx.cfg))
    flags, tau, chunks = ct.unpack(blob)
    assert flags == ct.config_flags(ctx.cfg) and tau == 1.0
    assert [c.n_tokens for c in chunks] == [len(s) for s in streams]
    out = ct.decompress(ctx, blob)
    for a, b in zip(out, streams):
        assert np.array_equal(a, b)


def test_nc06_hybrid_round_trip(setup):
    """A mixed file (text with embedded control bytes, a large compressible binary block, random
    binary bytes, short binary gaps) through NC06: text pieces coded as parallel GPU streams,
    the binary blob by LZMA; the bytes come back exactly."""
    _, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    from paper_2602_19626_amd import nc06
    rng = np.random.default_rng(3)
    words = [bytes(rng.integers(97, 123, rng.integers(2, 9), dtype=np.uint8)) for _ in range(60)]
    zipf = 1.0 / np.arange(1, 61) ** 1.1

    def text(n):
        out = b""
        while len(out) < n:
            out += words[rng.choice(60, p=zipf / zipf.sum())] + (b"\n" if rng.random() < 0.1
                                                                  else b" ")
        return out[:n]
    data = (text(900) + b"\x00\x01\x02" + text(500) + bytes(range(256)) * 24 + text(1300)
            + bytes(rng.integers(0, 256, 700, dtype=np.uint8)) + text(40) + b"\xff" * 30)
    seg = nc06.segment(data)
    assert [k for k, _, _ in seg].count(nc06.TEXT) >= 2
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32", skip=WL.skip,
                         mix_init=WL.mix_init, max_streams=64)
    ctx = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    blob = nc06.compress(ctx, data, flags=7, max_chunk_tokens=600)
    _, _, ents, codec, _, nraw = nc06.unpack(blob)
    assert codec == nc06.LZMA and nraw >= nc06.LZMA_MIN_BLOB
    texts = [e for e in ents if e.kind == nc06.TEXT]
    assert len(texts) >= 4 and all(e.n_tokens <= 600 for e in texts)
    assert nc06.decompress(ctx, blob) == data
    assert len(blob) < len(data)
    # each text entry's stream is what the pipeline codes for that piece alone
    piece = data[seg[0][1]:seg[0][1] + texts[0].n_bytes]
    assert ctx.encode_stream([nc06.tokens_of(piece)])[0][0] == texts[0].data


def test_graph_replayed_passes_match_direct_launches(setup):
    """Encode chunks and decode passes replayed from captured HIP graphs give the same bytes, the
    same tokens and the same probe distributions as kernels launched one by one; eager work and
    synchronisations run between the replays, and every replay's output feeds the next step."""
    _, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    streams = [toks[:900], synth.make_stream(700, WL.shape.vocab, seed=21, span=WL.span),
               synth.make_stream(333, WL.shape.vocab, seed=22, span=WL.span)]
    ctxs = {}
    for graphs in (True, False):
        cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32",
                             skip=WL.skip, mix_init=WL.mix_init, max_streams=3, graphs=graphs,
                             decode_graphs=graphs)
        ctxs[graphs] = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    data_g, _ = ctxs[True].encode_stream(streams)
    data_e, _ = ctxs[False].encode_stream(streams)
    assert data_g == data_e
    out = ctxs[True].decode_stream(data_g, [len(s) for s in streams])
    st = ctxs[True].stats()
    assert st["graph_captures"] > 0 and st["graph_replays"] > 2 * st["graph_captures"]
    for a, b in zip(out, streams):
        assert np.array_equal(a, b)
    ctxs[False].decode_stream(data_e, [len(s) for s in streams])
    assert ctxs[False].stats()["graph_replays"] == 0
    for c in ctxs.values():
        c.reset(1, 1000)
    for i in (0, 1, 150, 151, 600, 899):
        pg = ctxs[True].probs_for_context(0, toks[:i])
        pe = ctxs[False].probs_for_context(0, toks[:i])
        assert np.array_equal(pg, pe), i


def test_edge_cases_empty_single_and_degenerate_streams(setup):
    """Empty and one-token streams beside ordinary ones, a constant stream (the n-gram becomes
    certain, so most positions skip the model), a stream of the largest token id, and a stream
    whose length puts a slide exactly at its last position: exact round trips, batch-invariant
    bytes, and the coded length of the constant stream within 0.01 bits/token of the oracle."""
    _, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    L = WL.shape.ctx_len
    streams = [np.zeros(0, np.int32), np.array([7], np.int32), np.full(400, 3, np.int32),
               np.full(50, WL.shape.vocab - 1, np.int32), toks[:L + 1], toks[:L + WL.shape.slide]]
    cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32", skip=WL.skip,
                         mix_init=WL.mix_init, max_streams=len(streams))
    ctx = nc.Context(cfg, synth.flat_weights(WL.shape, w))
    data, bits = ctx.encode_stream(streams)
    assert ctx.stats()["tokens"] == sum(len(s) for s in streams)
    assert bits[0] >= 0 and len(data[0]) <= nc.encode_bound(0)
    out = ctx.decode_stream(data, [len(s) for s in streams])
    for a, b in zip(out, streams):
        assert np.array_equal(a, b)
    for k in (1, 2, 5):
        assert ctx.encode_stream([streams[k]])[0][0] == data[k], k
    ref = op.encode(op.Settings.from_workload(WL), WL.shape, w, streams[2], block=1,
                    quantize=False)
    assert abs(bits[2] - ref.ideal_bits) / len(streams[2]) < 0.01 + 9.0 / len(streams[2])
    ctx.decode_stream([data[2]], [len(streams[2])])
    assert ctx.stats()["skipped"] > 250              # the constant stream mostly skips
    with pytest.raises(nc.NacrithError):            # more streams than the context holds
        ctx.encode_stream(streams + [streams[1]])


def test_encode_graph_chunks_then_direct_steps(setup):
    """Uneven stream lengths make the batched encode alternate between replayed chunks (every
    stream active through the chunk) and directly launched positions (a stream ends inside the
    chunk): the bytes equal those of an eager context and of each stream coded alone."""
    _, w, toks, orc = setup
    import paper_2602_19626_amd as nc
    lens = (1000, 1000, 700, 333, 90, 1000)
    streams = [synth.make_stream(n, WL.shape.vocab, seed=40 + i, span=WL.span)
               for i, n in enumerate(lens)]
    out = {}
    for graphs in (True, False):
        cfg = nc.make_config(WL.shape, ngram_order=WL.ngram_order, precision="fp32",
                             skip=WL.skip, mix_init=WL.mix_init, max_streams=len(streams),
                             graphs=graphs)
        ctx = nc.Context(cfg, synth.flat_weights(WL.shape, w))
        out[graphs] = ctx.encode_stream(streams)[0]
        st = ctx.stats()
        assert (st["graph_replays"] > 10) == graphs
        if graphs:
            dec = ctx.decode_stream(out[graphs], list(lens))
            assert all(np.array_equal(a, b) for a, b in zip(dec, streams))
            assert ctx.encode_stream([streams[3]])[0][0] == out[graphs][3]
    assert out[True] == out[False]
