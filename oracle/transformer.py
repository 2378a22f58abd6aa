"""FP64 decoder-only transformer with the paper's sliding KV cache.

Passages followed: section 3.2 Eq. (lm) (next-token distribution from the hidden state of the last
position through the output matrix) and section 3.10 (when the cache holds L entries, drop the
oldest C, shift the remaining positions down by C, and evaluate only the new token at its new
position).

Model (the 135M shape: 30 layers, d 576, 9 query / 3 key-value heads of 64, gated-SiLU MLP 1536,
tied 49,152-way output; tiny shape: 2 layers, d 64, 4/2 heads of 16, MLP 176, vocab 512), per
appended token x at cache position pos:

    for each layer:
        y = rmsnorm(x) * g_attn                    rmsnorm(x) = x / sqrt(mean(x^2) + eps)
        q, k, v = y Wq^T, y Wk^T, y Wv^T
        q, k = rope(q, pos), rope(k, pos)          rotate-half pairs (i, i + hd/2),
                                                   angle pos * theta^(-2i/hd)
        append (k, v) to this layer's cache
        head h attends over every cached key of kv-head floor(h / (Hq/Hkv)), scale hd^-1/2
        x += concat_h(attn_h) Wo^T
        y = rmsnorm(x) * g_mlp
        x += (silu(y Wg^T) * (y Wu^T)) Wd^T
    z = (rmsnorm(x) * g_final) E^T                 tied output matrix, no output bias

Readings: the output layer has no bias (the paper's bias symbol in Eq. (lm) is read as the
adaptive bias of section 3.7, which is applied later); the first cache entry is a BOS token
(id 0) at position 0; cached keys are stored already rotated, and a slide re-rotates the kept keys
by -C, which is the paper's position shift; kept keys and values are never recomputed ("stale"
cache: a kept entry keeps the value it got when its token was appended).

Tokens appended together are evaluated with a causal mask, which is the per-token definition
above written for several tokens at once; a block never spans a slide.

Error model of the reduced-precision forms (test infrastructure only; off by default): an optional
``operand_noise(array, kind)`` callable is applied to every matrix-product operand -- kind
"weight" once to each projection matrix and to the output copy of E (the embedding lookup keeps
the exact E), kind "act" to the inputs of the projections and of the output layer, kind "att" to
the attention operands q, k, v and the softmax weights.  The reduced-precision tolerances are
derived from runs with a rounding-sized perturbation there; without the callable the arithmetic
above is unchanged.

Pinned by: torch float64 library attention/norm composition on a tiny model, the relative-shift
invariance of RoPE, single-key attention, GQA with one query head per kv head, the zero-layer
model (tests/test_oracle_transformer.py).
"""
from __future__ import annotations

import numpy as np


def rmsnorm(x: np.ndarray, g: np.ndarray, eps: float) -> np.ndarray:
    return x / np.sqrt(np.mean(x * x, axis=-1, keepdims=True) + eps) * g


def silu(x: np.ndarray) -> np.ndarray:
    return x / (1.0 + np.exp(-x))


class Transformer:
    def __init__(self, shape, weights: dict, max_block: int = 512, operand_noise=None):
        self.shape = shape
        self.w = {k: np.asarray(v, dtype=np.float64) for k, v in weights.items()}
        self.noise = operand_noise
        self.w_out = self.w["E"]
        if operand_noise is not None:
            for k in self.w:
                if k.split(".")[-1] in ("Wq", "Wk", "Wv", "Wo", "Wg", "Wu", "Wd"):
                    self.w[k] = operand_noise(self.w[k], "weight")
            self.w_out = operand_noise(self.w["E"], "weight")
        hd = shape.head_dim
        self.inv_freq = shape.rope_theta ** (-(2.0 * np.arange(hd // 2, dtype=np.float64)) / hd)
        self.max_block = max_block
        self.reset()

    def reset(self):
        s = self.shape
        self.K = [np.zeros((0, s.n_kv_heads, s.head_dim)) for _ in range(s.n_layers)]
        self.V = [np.zeros((0, s.n_kv_heads, s.head_dim)) for _ in range(s.n_layers)]
        self.n_appended = 0
        self.n_slides = 0
        self.cache_len = 0

    def rope(self, x: np.ndarray, pos: np.ndarray) -> np.ndarray:
        """x[n, heads, hd] rotated by angle pos[n] * inv_freq (rotate-half pairing)."""
        h2 = self.shape.head_dim // 2
        ang = np.asarray(pos, dtype=np.float64)[:, None] * self.inv_freq[None, :]
        cos, sin = np.cos(ang)[:, None, :], np.sin(ang)[:, None, :]
        x1, x2 = x[..., :h2], x[..., h2:]
        return np.concatenate([x1 * cos - x2 * sin, x2 * cos + x1 * sin], axis=-1)

    def _slide(self):
        c = self.shape.slide
        for l in range(self.shape.n_layers):
            kept = self.K[l][c:]
            self.K[l] = self.rope(kept, np.full(kept.shape[0], -float(c)))
            self.V[l] = self.V[l][c:]
        self.n_slides += 1
        self.cache_len -= c

    def _op(self, a: np.ndarray, kind: str) -> np.ndarray:
        return a if self.noise is None else self.noise(a, kind)

    def _block(self, tokens: np.ndarray) -> np.ndarray:
        s, w, op = self.shape, self.w, self._op
        n = len(tokens)
        base = self.cache_len
        pos = base + np.arange(n, dtype=np.float64)
        hq, hk, hd = s.n_heads, s.n_kv_heads, s.head_dim
        grp = hq // hk
        x = w["E"][tokens]
        for l in range(s.n_layers):
            p = f"l{l}."
            y = op(rmsnorm(x, w[p + "attn_norm"], s.norm_eps), "act")
            q = (y @ w[p + "Wq"].T).reshape(n, hq, hd)
            k = (y @ w[p + "Wk"].T).reshape(n, hk, hd)
            v = op((y @ w[p + "Wv"].T).reshape(n, hk, hd), "att")
            q, k = op(self.rope(q, pos), "att"), op(self.rope(k, pos), "att")
            self.K[l] = np.concatenate([self.K[l], k], axis=0)
            self.V[l] = np.concatenate([self.V[l], v], axis=0)
            kk, vv = self.K[l], self.V[l]                       # [base + n, hk, hd]
            nk = kk.shape[0]
            mask = np.arange(nk)[None, :] > (base + np.arange(n))[:, None]   # [n, nk]
            o = np.empty((n, hq, hd))
            for h in range(hq):
                g = h // grp
                sc = (q[:, h, :] @ kk[:, g, :].T) / np.sqrt(hd)
                sc[mask] = -np.inf
                sc -= sc.max(axis=1, keepdims=True)
                a = np.exp(sc)
                a /= a.sum(axis=1, keepdims=True)
                o[:, h, :] = op(a, "att") @ vv[:, g, :]
            x = x + op(o.reshape(n, hq * hd), "act") @ w[p + "Wo"].T
            y = op(rmsnorm(x, w[p + "mlp_norm"], s.norm_eps), "act")
            x = x + op(silu(y @ w[p + "Wg"].T) * (y @ w[p + "Wu"].T), "act") @ w[p + "Wd"].T
        self.n_appended += n
        self.cache_len += n
        return rmsnorm(x, w["final_norm"], s.norm_eps)

    def append(self, tokens) -> np.ndarray:
        """Append tokens to the cache; returns the final-normed hidden states [n, d]."""
        tokens = np.asarray(tokens, dtype=np.int64)
        out = []
        i = 0
        while i < len(tokens):
            if self.cache_len == self.shape.ctx_len:
                self._slide()
            m = min(len(tokens) - i, self.shape.ctx_len - self.cache_len, self.max_block)
            out.append(self._block(tokens[i:i + m]))
            i += m
        return np.concatenate(out, axis=0) if out else np.zeros((0, self.shape.d_model))

    def logits(self, hidden: np.ndarray) -> np.ndarray:
        return self._op(hidden, "act") @ self.w_out.T
