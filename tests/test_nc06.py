"""NC06 hybrid segmentation and container (paper section 3.11): the four segmentation rules on
hand-made inputs, invariants on random inputs, the binary codec choice, and the container layout.
The GPU round trip is in tests/test_gpu_pipeline.py."""
import numpy as np
import pytest

from paper_2602_19626_amd import nc06

B, T = nc06.BINARY, nc06.TEXT


def _kinds(data):
    return [(k, b - a) for k, a, b in nc06.segment(data)]


def test_rule1_text_like_bytes():
    allb = bytes(range(256))
    got = nc06.text_like(allb)
    want = [(32 <= b <= 126) or b in (9, 10, 13) for b in range(256)]
    assert got.tolist() == want


def test_rule2_short_text_runs_are_demoted():
    z = b"\x00" * 100
    assert _kinds(z + b"a" * 63 + z) == [(B, 263)]
    assert _kinds(z + b"a" * 64 + z) == [(B, 100), (T, 64), (B, 100)]


def test_rule3_and_rule4_gaps():
    t = b"x" * 100
    assert _kinds(t + b"\x01" * 8 + t) == [(T, 208)]          # bridged (rule 3)
    assert _kinds(t + b"\x01" * 63 + t) == [(T, 263)]         # absorbed (rule 4)
    assert _kinds(t + b"\x01" * 64 + t) == [(T, 100), (B, 64), (T, 100)]


def test_rule4_small_binary_next_to_text():
    t = b"y" * 100
    assert _kinds(b"\xff" * 63 + t) == [(T, 163)]
    assert _kinds(t + b"\xff" * 63) == [(T, 163)]
    assert _kinds(b"\xff" * 64 + t) == [(B, 64), (T, 100)]
    assert _kinds(b"\xff" * 10) == [(B, 10)]                   # no text to absorb it


def test_rules_apply_in_the_listed_order():
    """Two 40-byte text runs with a 5-byte gap are demoted by rule 2 before rule 3 could join
    them, so everything is binary."""
    z = b"\x00" * 200
    assert _kinds(z + b"a" * 40 + b"\x02" * 5 + b"b" * 40 + z) == [(B, 485)]


@pytest.mark.parametrize("seed", range(20))
def test_segmentation_invariants_on_random_inputs(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(rng.integers(1, 30)):
        n = int(rng.integers(1, 300))
        if rng.random() < 0.5:
            parts.append(bytes(rng.integers(32, 127, n, dtype=np.uint8)))
        else:
            parts.append(bytes(rng.integers(0, 256, n, dtype=np.uint8)))
    data = b"".join(parts)
    seg = nc06.segment(data)
    assert seg[0][1] == 0 and seg[-1][2] == len(data)
    for (k0, _, b0), (k1, a1, _) in zip(seg, seg[1:]):
        assert b0 == a1 and k0 != k1                          # contiguous, alternating
    for k, a, b in seg:
        if k == T:
            assert b - a >= nc06.MIN_TEXT_RUN
        elif len(seg) > 1:
            assert b - a >= nc06.MIN_BINARY_CHUNK
    for k, a, b in seg:                                       # a binary segment holds no
        if k == B:                                            # text run of 64 or more
            run = 0
            for f in nc06.text_like(data[a:b]):
                run = run + 1 if f else 0
                assert run < nc06.MIN_TEXT_RUN


def test_split_text_at_newlines():
    s = b"abc\n" * 10 + b"z" * 50
    pieces = nc06.split_text(s, 15)
    assert b"".join(pieces) == s
    assert all(len(p) <= 15 for p in pieces)
    assert pieces[0] == b"abc\nabc\nabc\n"
    assert nc06.split_text(b"q" * 40, 16) == [b"q" * 16, b"q" * 16, b"q" * 8]


def test_binary_codec_choice():
    small = b"\x00\x01" * 100
    big = b"\x00\x01\x02" * 3000
    rnd = bytes(np.random.default_rng(0).integers(0, 256, 5000, dtype=np.uint8))
    assert nc06.compress_blob(small)[0] == nc06.GZIP
    assert nc06.compress_blob(big)[0] == nc06.LZMA
    assert nc06.compress_blob(rnd) == (nc06.RAW, rnd)
    for b in (small, big, rnd, b""):
        c, d = nc06.compress_blob(b)
        assert nc06.decompress_blob(c, d, len(b)) == b


def test_container_layout_and_checksum():
    ents = [nc06.Entry(T, 100, 100, 333, b"\x11" * 42), nc06.Entry(B, 70),
            nc06.Entry(T, 80, 80, 90, b"\x22" * 12)]
    blob = nc06.pack(ents, flags=7, tau=1.0, codec=nc06.RAW, blob=b"\x00" * 70, blob_raw=70)
    assert blob[:4] == b"NC06" and blob[4] == 1
    assert len(blob) == nc06.HEADER.size + 3 * nc06.ENTRY.size + 70 + 42 + 12 + 4
    flags, tau, got, codec, binsec, nraw = nc06.unpack(blob)
    assert flags == 7 and tau == 1.0 and codec == nc06.RAW and nraw == 70
    assert [(e.kind, e.n_bytes, e.n_tokens, e.bits, e.data) for e in got] == \
        [(e.kind, e.n_bytes, e.n_tokens, e.bits, e.data) for e in ents]
    bad = bytearray(blob)
    bad[30] ^= 1
    with pytest.raises(ValueError):
        nc06.unpack(bytes(bad))
    with pytest.raises(ValueError):
        nc06.unpack(blob[:10])


def test_byte_tokeniser_round_trip():
    b = bytes(range(256))
    assert nc06.bytes_of(nc06.tokens_of(b)) == b
    with pytest.raises(ValueError):
        nc06.bytes_of([300])
