"""NC06 hybrid container: arbitrary bytes split into text-like and binary regions (paper section
3.11, format in section 3.13).

Segmentation, rules applied in the order the paper lists them:
  1. a byte is text-like if it is printable ASCII (32..126) or tab, LF or CR;
  2. text runs shorter than 64 bytes are demoted to binary;
  3. binary gaps of at most 8 bytes between two text runs are bridged (become text);
  4. binary chunks shorter than 64 bytes next to a text chunk are absorbed into the text.
(Under this order every gap that rule 3 bridges is also one rule 4 would absorb; rule 3 is kept
as its own step so the code reads as the paper's list.)

Text chunks are tokenised and coded by the GPU pipeline as independent streams (one NC05-style
table entry each: tokens, bits, stream bytes); a text chunk longer than `max_chunk_tokens` tokens
is cut at its last newline before the limit (else at the limit) so long inputs run as parallel
streams (section 3.12).  All binary chunks are concatenated into one blob compressed with LZMA
(blobs of at least 4 KB) or gzip (smaller), or stored raw when the chosen codec does not shrink
it.

Tokeniser: the paper codes text with the model's BPE tokeniser, which is not available here; a
byte-level stand-in maps byte b to token b (needs vocab >= 256) and back, so any byte string is a
valid text chunk.

Layout (little-endian; field widths are this implementation's, the paper names the fields):
  header, 20 bytes: magic b"NC06" | version u8 (1) | flags u8 | tau f16 | entries u32 |
                    binary codec u8 (0 raw, 1 gzip, 2 lzma) | reserved u8 (0) |
                    binary blob bytes u32 | binary raw bytes u32
  entry table, 17 bytes per entry: kind u8 (0 text, 1 binary) | source bytes u32 |
                    tokens u32 | bits u32 | stream bytes u32   (the last three are 0 for binary)
  binary section:   the compressed blob
  text streams:     the text entries' coded streams, in table order
  trailer:          CRC-32 of every preceding byte, present iff flags bit 7 is set (as in NC05).
"""
from __future__ import annotations

import gzip
import lzma
import struct
import zlib
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

MAGIC = b"NC06"
VERSION = 1
HEADER = struct.Struct("<4sBBeIBBII")
ENTRY = struct.Struct("<BIIII")
TRAILER = struct.Struct("<I")
F_CRC = 128
TEXT, BINARY = 0, 1
RAW, GZIP, LZMA = 0, 1, 2
MIN_TEXT_RUN = 64        # rule 2
MAX_BRIDGE = 8           # rule 3
MIN_BINARY_CHUNK = 64    # rule 4
LZMA_MIN_BLOB = 4096     # LZMA from 4 KB, gzip below


def text_like(data: bytes) -> np.ndarray:
    """Rule 1: printable ASCII 32..126 plus tab, LF and CR."""
    b = np.frombuffer(data, dtype=np.uint8)
    return ((b >= 32) & (b <= 126)) | (b == 9) | (b == 10) | (b == 13)


def _runs(flags) -> List[List[int]]:
    """Maximal runs [kind, start, end) of a per-byte kind array."""
    runs = []
    for i, f in enumerate(flags):
        k = TEXT if f else BINARY
        if runs and runs[-1][0] == k:
            runs[-1][2] = i + 1
        else:
            runs.append([k, i, i + 1])
    return runs


def _merge(runs):
    out = []
    for k, a, b in runs:
        if out and out[-1][0] == k:
            out[-1][2] = b
        else:
            out.append([k, a, b])
    return out


def segment(data: bytes) -> List[Tuple[int, int, int]]:
    """[(kind, start, end)] covering data in order, kinds alternating (rules 1-4)."""
    if not data:
        return []
    runs = _runs(text_like(data))
    # rule 2: short text runs become binary
    runs = _merge([[BINARY if k == TEXT and b - a < MIN_TEXT_RUN else k, a, b]
                   for k, a, b in runs])
    # rule 3: short binary gaps between two text runs become text
    runs = _merge([[TEXT if (k == BINARY and 0 < i < len(runs) - 1 and b - a <= MAX_BRIDGE)
                    else k, a, b] for i, (k, a, b) in enumerate(runs)])
    # rule 4: small binary chunks next to text are absorbed into it
    def next_to_text(i):
        return (i > 0 and runs[i - 1][0] == TEXT) or (i + 1 < len(runs) and runs[i + 1][0] == TEXT)
    runs = _merge([[TEXT if (k == BINARY and b - a < MIN_BINARY_CHUNK and next_to_text(i))
                    else k, a, b] for i, (k, a, b) in enumerate(runs)])
    return [tuple(r) for r in runs]


def split_text(chunk: bytes, max_tokens: int) -> List[bytes]:
    """Cut a text chunk into pieces of at most max_tokens bytes (= byte-level tokens), each cut
    after the last newline before the limit when there is one."""
    out, i = [], 0
    while len(chunk) - i > max_tokens:
        j = chunk.rfind(b"\n", i, i + max_tokens)
        cut = j + 1 if j >= i else i + max_tokens
        out.append(chunk[i:cut])
        i = cut
    out.append(chunk[i:])
    return out


def tokens_of(text: bytes) -> np.ndarray:
    """Byte-level stand-in tokeniser: byte b -> token b."""
    return np.frombuffer(text, dtype=np.uint8).astype(np.int32)


def bytes_of(tokens) -> bytes:
    t = np.asarray(tokens)
    if t.size and (t.min() < 0 or t.max() > 255):
        raise ValueError("decoded token outside the byte range")
    return t.astype(np.uint8).tobytes()


def compress_blob(blob: bytes) -> Tuple[int, bytes]:
    """(codec, bytes): LZMA for blobs of at least 4 KB, gzip below, raw if that does not shrink."""
    if not blob:
        return RAW, b""
    if len(blob) >= LZMA_MIN_BLOB:
        codec, out = LZMA, lzma.compress(blob, preset=9 | lzma.PRESET_EXTREME)
    else:
        codec, out = GZIP, gzip.compress(blob, compresslevel=9, mtime=0)
    return (codec, out) if len(out) < len(blob) else (RAW, blob)


def decompress_blob(codec: int, data: bytes, raw_len: int) -> bytes:
    out = {RAW: lambda d: d, GZIP: gzip.decompress, LZMA: lzma.decompress}[codec](data)
    if len(out) != raw_len:
        raise ValueError("binary section length mismatch")
    return out


@dataclass
class Entry:
    kind: int
    n_bytes: int
    n_tokens: int = 0
    bits: int = 0
    data: bytes = b""


def pack(entries: Sequence[Entry], flags: int, tau: float, codec: int, blob: bytes,
         blob_raw: int, checksum: bool = True) -> bytes:
    if flags & F_CRC:
        raise ValueError("flags bit 7 is set by pack(checksum=True), not by the caller")
    if checksum:
        flags |= F_CRC
    out = [HEADER.pack(MAGIC, VERSION, flags, tau, len(entries), codec, 0, len(blob), blob_raw)]
    for e in entries:
        out.append(ENTRY.pack(e.kind, e.n_bytes, e.n_tokens, e.bits, len(e.data)))
    out.append(blob)
    out.extend(e.data for e in entries if e.kind == TEXT)
    res = b"".join(out)
    if checksum:
        res += TRAILER.pack(zlib.crc32(res))
    return res


def unpack(blob: bytes):
    """-> (flags, tau, entries, codec, binary section, binary raw length)."""
    if len(blob) < HEADER.size:
        raise ValueError("truncated NC06 header")
    magic, ver, flags, tau, n, codec, _, nbin, nraw = HEADER.unpack_from(blob, 0)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("not an NC06 (version 1) container")
    if flags & F_CRC:
        if len(blob) < HEADER.size + TRAILER.size:
            raise ValueError("truncated NC06 checksum")
        body = blob[:-TRAILER.size]
        if zlib.crc32(body) != TRAILER.unpack_from(blob, len(blob) - TRAILER.size)[0]:
            raise ValueError("NC06 checksum mismatch")
        blob = body
    off = HEADER.size
    if len(blob) < off + n * ENTRY.size + nbin:
        raise ValueError("truncated NC06 table or binary section")
    raw = [ENTRY.unpack_from(blob, off + i * ENTRY.size) for i in range(n)]
    off += n * ENTRY.size
    binsec = bytes(blob[off:off + nbin])
    off += nbin
    entries = []
    for kind, nb, nt, bits, ns in raw:
        if kind not in (TEXT, BINARY) or (kind == BINARY and (nt or bits or ns)):
            raise ValueError("bad NC06 entry")
        if off + ns > len(blob):
            raise ValueError("truncated NC06 text stream")
        entries.append(Entry(kind, nb, nt, bits, bytes(blob[off:off + ns])))
        off += ns
    if off != len(blob):
        raise ValueError("trailing bytes after the NC06 text streams")
    if sum(e.n_bytes for e in entries if e.kind == BINARY) != nraw:
        raise ValueError("binary entries do not add up to the binary section")
    return flags & ~F_CRC, float(tau), entries, codec, binsec, nraw


def compress(ctx, data: bytes, flags: int, tau: float = 1.0, max_chunk_tokens: int = 1 << 15,
             checksum: bool = True) -> bytes:
    """Segment data, code every text piece as one stream of ctx (all in one batched
    encode_stream call), compress the binary blob, and pack."""
    if ctx.cfg.vocab < 256:
        raise ValueError("the byte-level tokeniser needs vocab >= 256")
    pieces = []                                    # (kind, bytes)
    for kind, a, b in segment(data):
        if kind == TEXT:
            pieces += [(TEXT, p) for p in split_text(data[a:b], max_chunk_tokens)]
        else:
            pieces.append((BINARY, data[a:b]))
    texts = [tokens_of(p) for k, p in pieces if k == TEXT]
    coded, bits = ctx.encode_stream(texts) if texts else ([], [])
    it = iter(zip(texts, coded, bits))
    entries = []
    for k, p in pieces:
        if k == TEXT:
            t, d, nb = next(it)
            entries.append(Entry(TEXT, len(p), len(t), int(nb), d))
        else:
            entries.append(Entry(BINARY, len(p)))
    raw = b"".join(p for k, p in pieces if k == BINARY)
    codec, blob = compress_blob(raw)
    return pack(entries, flags, tau, codec, blob, len(raw), checksum)


def decompress(ctx, blob: bytes) -> bytes:
    _, _, entries, codec, binsec, nraw = unpack(blob)
    raw = decompress_blob(codec, binsec, nraw)
    texts = [e for e in entries if e.kind == TEXT]
    toks = ctx.decode_stream([e.data for e in texts], [e.n_tokens for e in texts]) if texts else []
    out, ti, bi = [], 0, 0
    for e in entries:
        if e.kind == TEXT:
            piece = bytes_of(toks[ti])
            ti += 1
        else:
            piece = raw[bi:bi + e.n_bytes]
            bi += e.n_bytes
        if len(piece) != e.n_bytes:
            raise ValueError("entry length mismatch")
        out.append(piece)
    return b"".join(out)
