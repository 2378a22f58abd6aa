"""NC05 container: independently coded token streams in one file (paper section 3.13).

Layout (little-endian), as the paper's format section describes it:
  header, 9 bytes:  magic b"NC05" | flags u8 | tau f16 | chunk count u16
  chunk table:      12 bytes per chunk: token count u32 | bit count u32 | stream bytes u32
  payload:          the chunks' arithmetic-coded streams, concatenated in table order.
  trailer, optional: CRC-32 (zlib polynomial) of every preceding byte, u32, present iff flags
                    bit 7 is set.
The paper names the fields but not their encodings; the integer widths follow from its byte
counts, tau is stored as an IEEE half float, and flags bits are 0 n-gram, 1 adaptive head,
2 confidence skip, 3 mixer, 4 ensemble, 7 checksum trailer (bits 3, 4 and 7 and the trailer are
this implementation's additions; without bit 7 the file is exactly the paper's layout).
Chunks are the unit of parallelism: each is coded with fresh model state, so a decoder needs
only the table to find and decode any of them.
"""
from __future__ import annotations

import struct
import zlib
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

MAGIC = b"NC05"
HEADER = struct.Struct("<4sBeH")
ENTRY = struct.Struct("<III")
F_NGRAM, F_HEAD, F_SKIP, F_MIXER, F_ENSEMBLE = 1, 2, 4, 8, 16
F_CRC = 128
TRAILER = struct.Struct("<I")


@dataclass
class Chunk:
    n_tokens: int
    bits: int
    data: bytes


def pack(chunks: Sequence[Chunk], flags: int, tau: float = 1.0, checksum: bool = True) -> bytes:
    """Header, table and payload; with checksum, flags bit 7 and a CRC-32 trailer."""
    if len(chunks) > 0xFFFF:
        raise ValueError("NC05 holds at most 65,535 chunks")
    if not 0 <= flags <= 0xFF:
        raise ValueError("flags must fit one byte")
    if flags & F_CRC:
        raise ValueError("flags bit 7 is set by pack(checksum=True), not by the caller")
    if checksum:
        flags |= F_CRC
    out = [HEADER.pack(MAGIC, flags, tau, len(chunks))]
    for c in chunks:
        if not (0 <= c.n_tokens < 1 << 32 and 0 <= c.bits < 1 << 32 and len(c.data) < 1 << 32):
            raise ValueError("chunk fields must fit 32 bits")
        out.append(ENTRY.pack(c.n_tokens, c.bits, len(c.data)))
    out.extend(c.data for c in chunks)
    blob = b"".join(out)
    if checksum:
        blob += TRAILER.pack(zlib.crc32(blob))
    return blob


def unpack(blob: bytes):
    """-> (flags, tau, [Chunk]); raises ValueError on a malformed container."""
    if len(blob) < HEADER.size:
        raise ValueError("truncated NC05 header")
    magic, flags, tau, n = HEADER.unpack_from(blob, 0)
    if magic != MAGIC:
        raise ValueError("not an NC05 container")
    if flags & F_CRC:
        if len(blob) < HEADER.size + TRAILER.size:
            raise ValueError("truncated NC05 checksum")
        body, (crc,) = blob[:-TRAILER.size], TRAILER.unpack_from(blob, len(blob) - TRAILER.size)
        if zlib.crc32(body) != crc:
            raise ValueError("NC05 checksum mismatch")
        blob = body
    off = HEADER.size
    if len(blob) < off + n * ENTRY.size:
        raise ValueError("truncated NC05 chunk table")
    entries = [ENTRY.unpack_from(blob, off + i * ENTRY.size) for i in range(n)]
    off += n * ENTRY.size
    chunks = []
    for n_tok, bits, nbytes in entries:
        if off + nbytes > len(blob):
            raise ValueError("truncated NC05 payload")
        chunks.append(Chunk(n_tok, bits, bytes(blob[off:off + nbytes])))
        off += nbytes
    if off != len(blob):
        raise ValueError("trailing bytes after the NC05 payload")
    return flags & ~F_CRC, float(tau), chunks


def config_flags(cfg) -> int:
    """Container flags of an nc_config's feature switches (see make_config)."""
    from ._lib import NC_F_ENSEMBLE, NC_F_HEAD, NC_F_MIXER, NC_F_NGRAM, NC_F_SKIP
    pairs = ((NC_F_NGRAM, F_NGRAM), (NC_F_HEAD, F_HEAD), (NC_F_SKIP, F_SKIP),
             (NC_F_MIXER, F_MIXER), (NC_F_ENSEMBLE, F_ENSEMBLE))
    return sum(f for nc_f, f in pairs if cfg.features & nc_f)


def compress(ctx, streams: Sequence[np.ndarray], flags: int, tau: float = 1.0,
             checksum: bool = True) -> bytes:
    """Code every token stream as one chunk with ctx.encode_stream and wrap them in NC05."""
    data, bits = ctx.encode_stream(list(streams))
    return pack([Chunk(len(s), int(b), d) for s, b, d in zip(streams, bits, data)], flags, tau,
                checksum)


def decompress(ctx, blob: bytes) -> List[np.ndarray]:
    """Decode every chunk of an NC05 container with ctx.decode_stream."""
    _, _, chunks = unpack(blob)
    return ctx.decode_stream([c.data for c in chunks], [c.n_tokens for c in chunks])
