"""NC05 container (paper section 3.13): header and table layout, round trip, malformed input."""
import struct

import numpy as np
import pytest

from paper_2602_19626_amd import container as ct


def _chunks():
    rng = np.random.default_rng(0)
    return [ct.Chunk(int(n), int(b), bytes(rng.integers(0, 256, size=k, dtype=np.uint8)))
            for n, b, k in ((100, 810, 102), (7, 40, 5), (0, 0, 0), (2048, 16001, 2001))]


def test_layout_matches_the_paper_byte_counts():
    ch = _chunks()
    blob = ct.pack(ch, ct.F_NGRAM | ct.F_HEAD | ct.F_SKIP, tau=1.0, checksum=False)
    # 9-byte header: magic, flags, tau, chunk count; then 12 bytes per chunk; then the payload
    assert blob[:4] == b"NC05"
    assert blob[4] == 7
    assert struct.unpack("<e", blob[5:7])[0] == 1.0
    assert struct.unpack("<H", blob[7:9])[0] == len(ch)
    assert len(blob) == 9 + 12 * len(ch) + sum(len(c.data) for c in ch)
    n, bits, nbytes = struct.unpack("<III", blob[9:21])
    assert (n, bits, nbytes) == (100, 810, 102)
    assert blob[9 + 12 * len(ch):9 + 12 * len(ch) + 102] == ch[0].data


def test_round_trip():
    ch = _chunks()
    flags, tau, back = ct.unpack(ct.pack(ch, ct.F_ENSEMBLE, tau=0.75))
    assert flags == ct.F_ENSEMBLE and tau == 0.75
    assert [(c.n_tokens, c.bits, c.data) for c in back] == [(c.n_tokens, c.bits, c.data) for c in ch]


@pytest.mark.parametrize("cut", [3, 8, 15, 40])
def test_truncated_containers_are_rejected(cut):
    blob = ct.pack(_chunks(), 0, checksum=cut % 2 == 0)
    with pytest.raises(ValueError):
        ct.unpack(blob[:cut])


def test_checksum_trailer_detects_corruption():
    import zlib
    ch = _chunks()
    plain = ct.pack(ch, ct.F_HEAD, checksum=False)
    blob = ct.pack(ch, ct.F_HEAD)
    # the same bytes with flags bit 7 set, plus the CRC-32 of everything before the trailer
    assert len(blob) == len(plain) + 4 and blob[4] == ct.F_HEAD | ct.F_CRC
    assert blob[:4] == plain[:4] and blob[5:-4] == plain[5:]
    assert struct.unpack("<I", blob[-4:])[0] == zlib.crc32(blob[:-4])
    flags, _, back = ct.unpack(blob)
    assert flags == ct.F_HEAD and [c.data for c in back] == [c.data for c in ch]
    for pos in (0, 9, 30, len(blob) - 10, len(blob) - 1):
        bad = bytearray(blob)
        bad[pos] ^= 0x10
        with pytest.raises(ValueError):
            ct.unpack(bytes(bad))
    with pytest.raises(ValueError):
        ct.pack(ch, ct.F_CRC)


def test_bad_magic_trailing_bytes_and_limits():
    blob = ct.pack(_chunks(), 0, checksum=False)
    with pytest.raises(ValueError):
        ct.unpack(b"NC06" + blob[4:])
    with pytest.raises(ValueError):
        ct.unpack(blob + b"\0")
    with pytest.raises(ValueError):
        ct.pack([ct.Chunk(0, 0, b"")] * 65536, 0)
    with pytest.raises(ValueError):
        ct.pack([], 256)
