"""Algorithm 1 (compression) and its mirror (decompression), per stream, in float64.

Per position i of a stream t_0..t_{n-1} (the LLM sees x = (BOS, t_0, t_1, ...), so the logits
for t_i come from the hidden state of x_i):

1. n-gram distribution p_ng from t_0..t_{i-1}                      (section 3.5)
2. skip test (section 3.8): after the warmup, H(p_ng) < 1.5 bits (or p_max(p_ng) >= 0.99 in the
   batched workload) -> p = p_ng and no LLM;
3. otherwise p_llm = softmax(z), ptilde = softmax(log p_llm + b)   (sections 3.2, 3.3, 3.7);
   during the warmup (i < 100, section 3.6) p = ptilde, after it p = w_llm ptilde + w_ng p_ng;
4. cdf = CDF-24 quantisation of p                                    (section 3.4)
5. code t_i with the 32-bit arithmetic coder                          (section 3.9)
6. update: bias head only when the LLM ran, mixer only when step 3 mixed, n-gram always
   (Algorithm 1's update line, sections 3.5-3.7).

Readings where the paper is silent: the mixer sits between the head and the coder on LLM steps
after the warmup; the warmup suppresses both the skip test and the mixer update; skipped tokens
enter the KV cache when the LLM next runs, which in exact arithmetic equals appending every token
as it arrives, so the oracle appends eagerly.  Ensemble workload: experts (ptilde, P_1..P_K), a
softmax gate trained by SGD jointly with b, no skip and no warmup.

The skip/warmup/mixer placement is a convention shared with the GPU path: parity unpinned against
the paper; the per-step arithmetic is pinned in the component modules.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .cdf import quantize_cdf
from .coder import Decoder, Encoder
from .head import BiasHead, EnsembleGate, Mixer, entropy_bits, softmax
from .ngram import NGram
from .transformer import Transformer

MODE_LLM, MODE_SKIP, MODE_MIX, MODE_ENSEMBLE = 0, 1, 2, 3
BOS = 0


@dataclasses.dataclass
class Settings:
    """Feature switches and constants of one run (defaults: the full method of the paper)."""
    vocab: int
    ngram_order: int = 4
    use_head: bool = True
    use_ngram: bool = True
    use_skip: bool = True
    use_mixer: bool = True
    skip: str = "entropy"          # "entropy" | "pmax" | "none"
    skip_entropy_bits: float = 1.5
    skip_pmax: float = 0.99
    warmup: int = 100
    head_lr: float = 1e-3
    mix_init: str = "llm85"
    mix_eta: float = 1.0
    ngram_eps: float = 5.0
    ngram_slots: int = 64
    ngram_max_contexts: int = 500_000
    ensemble: bool = False
    cdf_total: int = 1 << 24

    @classmethod
    def from_workload(cls, wl, **over):
        kw = dict(vocab=wl.shape.vocab, ngram_order=wl.ngram_order, skip=wl.skip,
                  warmup=wl.warmup, head_lr=wl.head_lr, mix_init=wl.mix_init,
                  ensemble=wl.ensemble, cdf_total=wl.cdf_total, use_skip=wl.skip != "none")
        kw.update(over)
        return cls(**kw)


class LLMFeed:
    """Feeds x = (BOS, t_0, ...) to the transformer and returns the logits of position i."""

    def __init__(self, model: Transformer, block: int):
        self.model = model
        self.block = block
        self.x = [BOS]
        self.appended = 0
        self.buf = {}

    def push(self, token: int):
        self.x.append(int(token))

    def logits(self, i: int) -> np.ndarray:
        while self.appended <= i:
            j = min(len(self.x), self.appended + self.block)
            h = self.model.append(self.x[self.appended:j])
            z = self.model.logits(h)
            for r in range(j - self.appended):
                self.buf[self.appended + r] = z[r]
            self.appended = j
        for k in [k for k in self.buf if k < i]:
            del self.buf[k]
        return self.buf[i]


class StreamState:
    """The ensemble state of one stream (LLM cache, n-gram, bias head, mixer / gate)."""

    def __init__(self, settings: Settings, shape, weights, block: int = 512):
        self.s = settings
        self.feed = LLMFeed(Transformer(shape, weights, max_block=max(block, 1)), block)
        self.ng = NGram(settings.vocab, settings.ngram_order, settings.ngram_eps,
                        settings.ngram_slots, settings.ngram_max_contexts)
        self.head = BiasHead(settings.vocab, settings.head_lr)
        self.mixer = Mixer(2, settings.mix_init, settings.mix_eta)
        self.gate = EnsembleGate(settings.ngram_order + 1, settings.vocab, settings.head_lr)
        self.history = []
        self.i = 0

    def distribution(self):
        """Coding distribution p for position i and the intermediates needed by commit()."""
        s, i = self.s, self.i
        st = {"i": i}
        if s.ensemble:
            ps = self.ng.predict_all(self.history)
            z = self.feed.logits(i)
            q0 = softmax(np.log(softmax(z)) + self.gate.b)
            w, p = EnsembleGate.forward(self.gate.theta, [q0] + ps[1:])
            st.update(mode=MODE_ENSEMBLE, z=z, q0=q0, experts=ps[1:], gate_w=w, skip=False)
            return p, st
        p_ng = self.ng.predict(self.history) if s.use_ngram else None
        warm = i < s.warmup
        skip = False
        if p_ng is not None:
            st["entropy"] = entropy_bits(p_ng)
            st["pmax"] = float(p_ng.max())
            if s.use_skip and not warm:
                if s.skip == "entropy":
                    skip = st["entropy"] < s.skip_entropy_bits
                elif s.skip == "pmax":
                    skip = st["pmax"] >= s.skip_pmax
        st["p_ng"], st["skip"] = p_ng, skip
        if skip:
            st["mode"] = MODE_SKIP
            return p_ng, st
        z = self.feed.logits(i)
        p_llm = softmax(z)
        ptilde = self.head.adjust(p_llm) if s.use_head else p_llm
        st.update(z=z, p_llm=p_llm, ptilde=ptilde)
        if warm or p_ng is None or not s.use_mixer:
            st["mode"] = MODE_LLM
            return ptilde, st
        st["mode"] = MODE_MIX
        st["mix_w"] = self.mixer.weights
        return self.mixer.mix([ptilde, p_ng]), st

    def commit(self, token: int, st, push: bool = True):
        s = self.s
        mode = st["mode"]
        if mode == MODE_ENSEMBLE:
            self.gate.step(st["q0"], st["experts"], token)
        else:
            if mode in (MODE_LLM, MODE_MIX) and s.use_head:
                self.head.update(st["ptilde"], token)
            if mode == MODE_MIX:
                self.mixer.update([st["ptilde"], st["p_ng"]], token)
        if s.use_ngram or s.ensemble:
            self.ng.update(self.history, token)
        self.history.append(int(token))
        if push:
            self.feed.push(token)
        self.i += 1


@dataclasses.dataclass
class StreamResult:
    n: int
    data: bytes
    n_bits: int
    ideal_bits: float            # sum_i -log2 p_i(t_i), float64
    quant_bits: float            # sum_i -log2 (c_i(t_i) / T)
    p_tok: np.ndarray            # p_i(t_i)
    modes: np.ndarray
    intervals: np.ndarray        # [n, 2] (cl, ch) int64
    records: dict                # position -> intermediates


def encode(settings: Settings, shape, weights, tokens, record=(), block: int = 512,
           quantize: bool = True) -> StreamResult:
    """Compress one stream (Algorithm 1).  `record` lists positions whose intermediates are kept.

    With quantize=False only the ideal code length is computed (no CDF, no bitstream).
    """
    st_ = StreamState(settings, shape, weights, block)
    for t in tokens[:-1]:                 # teacher forcing: x_1..x_{n-1} are known up front
        st_.feed.push(t)
    n = len(tokens)
    p_tok = np.zeros(n)
    modes = np.zeros(n, dtype=np.int64)
    iv = np.zeros((n, 2), dtype=np.int64)
    rec = {}
    enc = Encoder(settings.cdf_total)
    record = set(int(r) for r in record)
    for i, t in enumerate(tokens):
        t = int(t)
        p, st = st_.distribution()
        p_tok[i] = p[t]
        modes[i] = st["mode"]
        if quantize:
            cdf = quantize_cdf(p, settings.cdf_total)
            iv[i] = (cdf[t], cdf[t + 1])
            enc.encode(int(cdf[t]), int(cdf[t + 1]))
        if i in record:
            rec[i] = dict(st, p=p, cdf=quantize_cdf(np.asarray(p, dtype=np.float64),
                                                    settings.cdf_total) if quantize else None)
        st_.commit(t, st, push=False)
    data = enc.finish() if quantize else b""
    counts = iv[:, 1] - iv[:, 0]
    qbits = float(np.sum(np.log2(settings.cdf_total) - np.log2(np.maximum(counts, 1)))) \
        if quantize else float("nan")
    return StreamResult(n=n, data=data, n_bits=enc.n_bits if quantize else 0,
                        ideal_bits=float(-np.sum(np.log2(p_tok))), quant_bits=qbits,
                        p_tok=p_tok, modes=modes, intervals=iv, records=rec)


def decode(settings: Settings, shape, weights, data: bytes, n: int, block: int = 512):
    """Decompress n tokens (the mirror of encode); returns int64 tokens."""
    st_ = StreamState(settings, shape, weights, block)
    dec = Decoder(data, settings.cdf_total)
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        p, st = st_.distribution()
        cdf = quantize_cdf(p, settings.cdf_total)
        t = dec.decode(cdf)
        if dec.overrun:
            raise ValueError("corrupt stream: decoder ran past the end of the input")
        out[i] = t
        st_.commit(t, st)
    return out
