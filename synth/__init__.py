"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *produces inputs*: model weights drawn from N(0, 0.02), token streams drawn from
a bounded Zipf law with copied spans, and the table of workload configurations.  It contains none
of the compressor's arithmetic (no transformer, n-gram, mixing, quantisation or coding), so that
both sides of every parity test can consume the same bytes without sharing any method code.

Stand-in inputs: the paper evaluates on natural-language benchmark files with a trained
SmolLM2-135M.  Neither is available here, so every workload is a seeded synthetic token stream
with the statistics given in the workload table (Zipf(1.1) unigram, 30% of free positions start
an LZ77-style copied span) and random-init weights of the 135M shape.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["ModelShape", "Workload", "WORKLOADS", "TINY", "FULL", "make_weights", "flat_weights",
           "weight_layout", "make_stream", "make_streams", "workload_streams"]


@dataclasses.dataclass(frozen=True)
class ModelShape:
    n_layers: int
    d_model: int
    n_heads: int
    n_kv_heads: int
    head_dim: int
    d_ffn: int
    vocab: int
    rope_theta: float
    norm_eps: float = 1e-5
    ctx_len: int = 2048      # L: KV-cache capacity (paper section 3.10)
    slide: int = 512         # C: entries dropped when the cache is full


TINY = ModelShape(n_layers=2, d_model=64, n_heads=4, n_kv_heads=2, head_dim=16, d_ffn=176,
                  vocab=512, rope_theta=1e4, ctx_len=128, slide=32)
FULL = ModelShape(n_layers=30, d_model=576, n_heads=9, n_kv_heads=3, head_dim=64, d_ffn=1536,
                  vocab=49152, rope_theta=1e5, ctx_len=2048, slide=512)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: model shape, ensemble settings and the seeded streams."""
    name: str
    shape: ModelShape
    weight_seed: int
    ngram_order: int
    mix_init: str            # "uniform" or "llm85" (0.85 to the LLM, rest split evenly)
    skip: str                # "entropy" (H < 1.5 bits), "pmax" (p_max >= 0.99) or "none"
    ensemble: bool           # softmax-gated 5-expert head trained by SGD (differentiation form)
    precision: str           # "fp32", "bf16" or "fp8"
    n_streams: int
    lengths: tuple           # per-stream token counts
    stream_seeds: tuple
    span: tuple              # (lo, hi) copied-span length
    head_lr: float = 1e-3
    warmup: int = 100
    cdf_total: int = 1 << 24


def _uniform_lengths(n, lo, hi, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return tuple(int(x) for x in rng.integers(lo, hi + 1, size=n))


WORKLOADS = {
    "tiny": Workload("tiny", TINY, weight_seed=0, ngram_order=3, mix_init="uniform", skip="entropy",
                     ensemble=False, precision="fp32", n_streams=1, lengths=(2048,),
                     stream_seeds=(1,), span=(4, 32)),
    "full_fp32": Workload("full_fp32", FULL, weight_seed=1, ngram_order=4, mix_init="llm85",
                          skip="entropy", ensemble=False, precision="fp32", n_streams=1,
                          lengths=(16384,), stream_seeds=(2,), span=(8, 64)),
    "full_bf16": Workload("full_bf16", FULL, weight_seed=1, ngram_order=4, mix_init="llm85",
                          skip="entropy", ensemble=False, precision="bf16", n_streams=1,
                          lengths=(16384,), stream_seeds=(2,), span=(8, 64)),
    "full_fp8": Workload("full_fp8", FULL, weight_seed=1, ngram_order=4, mix_init="llm85",
                         skip="entropy", ensemble=False, precision="fp8", n_streams=1,
                         lengths=(16384,), stream_seeds=(2,), span=(8, 64)),
    "batch64_bf16": Workload("batch64_bf16", FULL, weight_seed=1, ngram_order=4, mix_init="llm85",
                             skip="pmax", ensemble=False, precision="bf16", n_streams=64,
                             lengths=_uniform_lengths(64, 1024, 32768, 4),
                             stream_seeds=tuple(1000 + s for s in range(64)), span=(8, 64)),
    "ensemble64": Workload("ensemble64", FULL, weight_seed=1, ngram_order=4, mix_init="llm85",
                           skip="none", ensemble=True, precision="fp32", n_streams=64,
                           lengths=(8192,) * 64, stream_seeds=tuple(2000 + s for s in range(64)),
                           span=(8, 64)),
}

# Calibration stream for static FP8 activation scales: a seed no evaluation stream uses.
CALIBRATION_SEED = 3


def weight_layout(shape: ModelShape):
    """Names and shapes of the flat FP32 weight buffer, in storage order.

    Matrices are stored [out_features][in_features] (row-major), so a projection is y = x W^T.
    Storage order: E, then per layer (attn_norm, Wq, Wk, Wv, Wo, mlp_norm, Wg, Wu, Wd), then
    final_norm.  The norm gains are part of the layout so that real checkpoints could be loaded;
    the synthetic generator sets them to one.
    """
    d, hq, hk, hd, f, v = (shape.d_model, shape.n_heads, shape.n_kv_heads, shape.head_dim,
                           shape.d_ffn, shape.vocab)
    out = [("E", (v, d))]
    for l in range(shape.n_layers):
        out += [(f"l{l}.attn_norm", (d,)), (f"l{l}.Wq", (hq * hd, d)), (f"l{l}.Wk", (hk * hd, d)),
                (f"l{l}.Wv", (hk * hd, d)), (f"l{l}.Wo", (d, hq * hd)), (f"l{l}.mlp_norm", (d,)),
                (f"l{l}.Wg", (f, d)), (f"l{l}.Wu", (f, d)), (f"l{l}.Wd", (d, f))]
    out.append(("final_norm", (d,)))
    return out


def make_weights(shape: ModelShape, seed: int, std: float = 0.02):
    """Random-init FP32 weights, N(0, std) for every matrix, gains = 1.

    Draw order is fixed: E, then per layer Wq, Wk, Wv, Wo, Wg, Wu, Wd (numpy PCG64, float32
    standard normals scaled in float32).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.float32(std)
    w = {}
    for name, shp in weight_layout(shape):
        if name.endswith("norm"):
            continue
        w[name] = rng.standard_normal(shp, dtype=np.float32) * s
    for name, shp in weight_layout(shape):
        if name.endswith("norm"):
            w[name] = np.ones(shp, dtype=np.float32)
    return w


def flat_weights(shape: ModelShape, weights: dict) -> np.ndarray:
    """Concatenate a weight dict into the flat FP32 buffer described by weight_layout()."""
    parts = [np.ascontiguousarray(weights[n], dtype=np.float32).reshape(-1)
             for n, _ in weight_layout(shape)]
    return np.concatenate(parts)


def _zipf_cdf(vocab: int, s: float) -> np.ndarray:
    ranks = np.arange(1, vocab + 1, dtype=np.float64)
    w = ranks ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def make_stream(n: int, vocab: int, seed: int, span=(4, 32), p_span=0.3, zipf_s=1.1) -> np.ndarray:
    """One synthetic token stream of n ids in [0, vocab).

    At every position that is not inside a copied span: draw u ~ U[0,1).  If u < p_span and the
    position is not the first, start a span of length U{lo..hi} copying token by token from a
    source start drawn uniformly in [0, i-1] (the source may overlap the span, LZ77 style; spans
    are cut at the stream end).  Otherwise draw a rank r from the bounded Zipf(zipf_s) law over
    1..vocab and emit id r-1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cdf = _zipf_cdf(vocab, zipf_s)
    out = np.empty(n, dtype=np.int32)
    i = 0
    lo, hi = span
    while i < n:
        u = rng.random()
        if i > 0 and u < p_span:
            length = int(rng.integers(lo, hi + 1))
            src = int(rng.integers(0, i))
            for k in range(min(length, n - i)):
                out[i + k] = out[src + k]
            i += min(length, n - i)
        else:
            r = int(np.searchsorted(cdf, rng.random(), side="right"))
            out[i] = min(r, vocab - 1)
            i += 1
    return out


def make_streams(lengths, seeds, vocab, span):
    return [make_stream(int(n), vocab, int(s), span=span) for n, s in zip(lengths, seeds)]


def workload_streams(wl: Workload, max_len: int | None = None, n_streams: int | None = None):
    """The workload's streams, optionally truncated (max_len) or limited to the first n_streams."""
    k = wl.n_streams if n_streams is None else min(n_streams, wl.n_streams)
    lengths = [wl.lengths[i] if max_len is None else min(max_len, wl.lengths[i]) for i in range(k)]
    return make_streams(lengths, wl.stream_seeds[:k], wl.shape.vocab, wl.span)
