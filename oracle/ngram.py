"""Interpolated token n-gram model (paper section 3.5), FP64 probabilities, exact counts.

Definition followed:

- unigram base, Laplace-smoothed: P_0(t) = (c(t) + 1) / (N + V), c(t) the count of t and N the
  number of tokens seen;
- for k = 1..K, with context (t_{i-k}, ..., t_{i-1}) seen n_k times:
  P_k = lambda_k * Phat_k(. | context) + (1 - lambda_k) * P_{k-1}, lambda_k = n_k / (n_k + eps),
  eps = 5; a context that is absent (or a position with fewer than k predecessors) leaves
  P_k = P_{k-1};
- updated online after each token;
- each context keeps at most 64 continuations; inserting into a full context evicts the
  lowest-count continuation.

Readings where the paper is silent: n_k is the sum of the stored continuation counts (so Phat_k
sums to one after evictions); ties for eviction go to the lowest slot index and the newcomer takes
that slot with count 1; contexts are keyed by the exact token tuple (the paper's 64-bit rolling
hash differs only on a hash collision); each order holds at most 500,000 contexts and a new
context is not stored once that cap is reached.

Pinned by: N = 0 gives the uniform 1/V, hand-worked short sequences, sums to one
(tests/test_oracle_ngram.py).  The eviction tie-break and the capacity rule are conventions the
GPU path shares: parity unpinned against the paper.
"""
from __future__ import annotations

import numpy as np


class NGram:
    def __init__(self, vocab: int, order: int, eps: float = 5.0, slots: int = 64,
                 max_contexts: int = 500_000):
        self.vocab = vocab
        self.order = order
        self.eps = float(eps)
        self.slots = slots
        self.max_contexts = max_contexts
        self.uni = np.zeros(vocab, dtype=np.int64)
        self.n = 0
        # tables[k-1]: dict context-tuple -> list of [token, count] in slot order
        self.tables = [dict() for _ in range(order)]

    def unigram(self) -> np.ndarray:
        return (self.uni.astype(np.float64) + 1.0) / float(self.n + self.vocab)

    def context_stats(self, history, k):
        """(tokens, counts, n_k) of the order-k context ending the history, or None if absent."""
        if len(history) < k:
            return None
        ctx = tuple(int(t) for t in history[len(history) - k:])
        slots = self.tables[k - 1].get(ctx)
        if not slots:
            return None
        toks = np.array([s[0] for s in slots], dtype=np.int64)
        cnts = np.array([s[1] for s in slots], dtype=np.float64)
        n_k = float(cnts.sum())
        if n_k <= 0:
            return None
        return toks, cnts, n_k

    def predict_all(self, history):
        """[P_0, P_1, ..., P_K] for the next token after `history` (list of FP64 arrays)."""
        p = self.unigram()
        out = [p]
        for k in range(1, self.order + 1):
            st = self.context_stats(history, k)
            if st is not None:
                toks, cnts, n_k = st
                lam = n_k / (n_k + self.eps)
                phat = np.zeros(self.vocab)
                phat[toks] = cnts / n_k
                p = lam * phat + (1.0 - lam) * p
            out.append(p)
        return out

    def predict(self, history) -> np.ndarray:
        return self.predict_all(history)[-1]

    def update(self, history, token: int):
        token = int(token)
        self.uni[token] += 1
        self.n += 1
        for k in range(1, self.order + 1):
            if len(history) < k:
                continue
            ctx = tuple(int(t) for t in history[len(history) - k:])
            table = self.tables[k - 1]
            slots = table.get(ctx)
            if slots is None:
                if len(table) >= self.max_contexts:
                    continue
                table[ctx] = [[token, 1]]
                continue
            for s in slots:
                if s[0] == token:
                    s[1] += 1
                    break
            else:
                if len(slots) < self.slots:
                    slots.append([token, 1])
                else:
                    j = min(range(len(slots)), key=lambda q: (slots[q][1], q))
                    slots[j] = [token, 1]
