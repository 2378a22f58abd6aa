"""GEMM launch shapes and the autotuner (135M shape).  Every launch shape evaluates the same
per-part MFMA chains and adds them in the same order, so forcing any shape on every GEMM must
leave the logits and the coded bytes bit-identical; a tuned context must still round-trip."""
import numpy as np
import pytest

import synth
from tests.nc_util import gpu_available, make_context

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["full_fp32"]
GEMMS = ("qkv", "oproj", "gateup", "down", "lmhead")
BUCKETS = (1, 2, 4, 8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 1024, 2048)


def _all_buckets(kind, mb=0, waves=0):
    return [{"gemm": g, "max_rows": b, "kind": kind, "mb": mb, "waves": waves}
            for g in GEMMS for b in BUCKETS]


def _streams():
    return [synth.make_stream(n, WL.shape.vocab, seed=s, span=WL.span)
            for n, s in ((600, 91), (300, 92), (40, 93))]


def _logits(ctx, toks):
    """Logits and coding distributions after three prefixes (at least one runs the model)."""
    ctx.reset(1, len(toks) + 1)
    out, ran = [], 0
    for n in (3, 20, len(toks)):
        p, pr = ctx.probs_for_context(0, toks[:n], probe=True)
        out += [pr["logits"].copy(), p.copy()]
        ran += int(pr["llm_ran"])
    assert ran > 0
    return np.concatenate(out)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_every_launch_shape_gives_identical_bits(prec):
    if not gpu_available():
        pytest.skip("no GPU")
    ctx, _ = make_context(WL, precision=prec, max_streams=3)
    streams = _streams()
    ref, ref_bits = ctx.encode_stream(streams)
    ref_z = _logits(ctx, streams[0][:555])
    shapes = [("split", 1, 16), ("split", 2, 5), ("split", 4, 3), ("tile_small", 0, 0),
              ("tile_64", 0, 0)]
    if prec != "fp32":
        shapes.append(("wide_128", 0, 0))
    for kind, mb, waves in shapes:
        ctx.tiles_reset()
        ctx.tiles_set(_all_buckets(kind, mb, waves))
        got, bits = ctx.encode_stream(streams)
        print(f"{prec} {kind} mb={mb} waves={waves}: {sum(bits)} bits", flush=True)
        assert got == ref and bits == ref_bits, (kind, mb, waves)
        assert np.array_equal(_logits(ctx, streams[0][:555]), ref_z), (kind, mb, waves)
    # decode under the last shape reproduces the input
    dec = ctx.decode_stream(ref, [len(s) for s in streams])
    for a, b in zip(dec, streams):
        assert np.array_equal(a, b)


def test_autotune_keeps_bytes_and_round_trips():
    if not gpu_available():
        pytest.skip("no GPU")
    ctx, _ = make_context(WL, precision="bf16", max_streams=3)
    streams = _streams()
    ref, _ = ctx.encode_stream(streams)
    table = ctx.autotune(max_rows=1024, reps=3)
    # 15 row buckets up to 1024 rows for every GEMM (the output layer is tuned up to its encode chunk)
    assert len(table) == 5 * 15
    for e in table:
        assert e["us_best"] <= e["us_default"] and e["us_best"] > 0, e
        if e["kind"] == "split":
            assert 1 <= e["mb"] <= 4 and 1 <= e["waves"] <= 16, e
    print("tuned:", [(e["gemm"], e["max_rows"], e["kind"], e["mb"], e["waves"],
                      round(e["us_default"] / e["us_best"], 2)) for e in table], flush=True)
    # the tuner overwrote stream state: probing needs a reset first
    with pytest.raises(Exception):
        ctx.probs_for_context(0, streams[0][:10])
    got, _ = ctx.encode_stream(streams)
    assert got == ref
    dec = ctx.decode_stream(got, [len(s) for s in streams])
    for a, b in zip(dec, streams):
        assert np.array_equal(a, b)


def test_tile_errors():
    if not gpu_available():
        pytest.skip("no GPU")
    ctx, _ = make_context(WL, precision="fp32", max_streams=1)
    with pytest.raises(Exception):
        ctx.tiles_set([{"gemm": "qkv", "max_rows": 512, "kind": "wide_128"}])  # BF16/FP8 only
    with pytest.raises(Exception):
        ctx.tiles_set([{"gemm": "down", "max_rows": 8, "kind": "split", "mb": 5, "waves": 4}])
    with pytest.raises(Exception):
        ctx.tiles_set([{"gemm": "down", "max_rows": 8, "kind": "split", "mb": 1, "waves": 17}])
    with pytest.raises(Exception):
        ctx.autotune(max_rows=0)
