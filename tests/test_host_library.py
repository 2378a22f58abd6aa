"""CPU-side checks of the HIP library: it loads, exports every symbol the header declares, and its
host arithmetic coder is byte-identical to the oracle coder."""
import os
import re

import numpy as np
import pytest

import paper_2602_19626_amd as nc
from oracle.coder import Decoder, encode_intervals

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nacrith.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = nc.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_encode_bound():
    assert nc.encode_bound(0) == 8
    assert nc.encode_bound(100) == (25 * 100 + 64 + 7) // 8


@pytest.mark.parametrize("seed", range(3))
def test_host_coder_bytes_equal_oracle(seed):
    rng = np.random.default_rng(seed)
    total = 1 << 24
    v = 2000
    counts = np.maximum(1, rng.dirichlet(np.full(v, 0.05)) * (total - v)).astype(np.int64)
    counts[0] += total - counts.sum()
    cdf = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    seq = rng.integers(0, v, size=5000)
    iv = np.stack([cdf[seq], cdf[seq + 1]], axis=1)
    data, bits = nc.ac_encode(iv, total)
    ref, ref_bits = encode_intervals(iv.tolist(), total)
    assert data == ref and bits == ref_bits
    out = nc.ac_decode_static(data, cdf, len(seq))
    assert np.array_equal(out, seq)


def test_host_coder_edge_cases():
    # one-count symbols, tiny totals, empty input
    for total in (2, 3, 97, 1 << 24):
        cdf = np.array([0, 1, total], dtype=np.int64)
        seq = np.array([0, 1, 0, 0, 1, 1, 1, 0] * 20)
        iv = np.stack([cdf[seq], cdf[seq + 1]], axis=1)
        data, bits = nc.ac_encode(iv, total)
        ref, ref_bits = encode_intervals(iv.tolist(), total)
        assert (data, bits) == (ref, ref_bits)
        assert np.array_equal(nc.ac_decode_static(data, cdf, len(seq)), seq)
    data, bits = nc.ac_encode(np.zeros((0, 2), np.uint32))
    assert (data, bits) == encode_intervals([], 1 << 24)


def test_error_paths():
    with pytest.raises(nc.NacrithError) as e:
        nc.ac_encode(np.array([[5, 5]], np.uint32))          # empty interval
    assert e.value.status == 1
    cdf = np.array([0, 1 << 23, 1 << 24], np.uint32)          # one bit per symbol
    with pytest.raises(nc.NacrithError) as e:
        nc.ac_decode_static(b"\xff" * 2, cdf, 100)           # 100 bits from 16: corrupt
    assert e.value.status == 5


def test_create_rejects_invalid_configs_before_touching_the_device():
    """nc_create validates the configuration first, so these fail with NC_E_INVALID on any host."""
    import synth
    w = np.zeros(16, np.float32)
    for over in (dict(ngram_max_contexts=0), dict(ngram_order=5), dict(max_streams=0),
                 dict(ngram_eps=0.0), dict(cdf_total=512)):
        cfg = nc.make_config(synth.TINY, **{**dict(ngram_order=3), **over})
        with pytest.raises(nc.NacrithError) as e:
            nc.Context(cfg, w)
        assert e.value.status == 1, over
