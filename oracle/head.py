"""Vocabulary softmax, adaptive bias head, context mixer, skip statistics and the ensemble gate.

All in float64.  Passages followed:

- section 3.3: p_llm = softmax(z / tau); tau = 1 makes the division a no-op and it is skipped.
- section 3.7: ptilde = softmax(log p_llm + b), b initialised to zero; after the observed token
  t*, b_t -= alpha * (ptilde(t) - 1[t = t*]) with alpha = 1e-3 (one SGD step on -log ptilde(t*)).
- section 3.6: p_mix = sum_j w_j p_j with sum w = 1; after t*, log w_j += eta * log p_j(t*)
  followed by renormalisation.  eta is unspecified; eta = 1 makes the update the Bayes posterior
  the paper says it equals.  Initial weights 0.85 for the LLM and 0.15 split evenly, or uniform.
- section 3.8: Shannon entropy of the n-gram distribution in bits (skip when below 1.5).

Differentiation workload (softmax-gated ensemble): experts q_0 = ptilde and q_j = P_j (n-gram
orders 1..4), gate w = softmax(theta), p = sum_j w_j q_j, loss L = -log p(t*).  With
responsibilities r_j = w_j q_j(t*) / p(t*) the gradients are dL/dtheta_j = w_j - r_j and
dL/db_t = r_0 (q_0(t) - 1[t = t*]); when r_0 = 1 the latter is exactly the bias-head gradient of
section 3.7.

Pinned by: b = 0 gives ptilde = p_llm, the bias gradient against central finite differences,
the mixer's 0.765 lower bound and the Bayes-posterior closed form, and the ensemble gradients
against finite differences (tests/test_oracle_head.py).
"""
from __future__ import annotations

import numpy as np


def logsumexp(x: np.ndarray) -> float:
    m = float(np.max(x))
    return m + float(np.log(np.sum(np.exp(x - m))))


def softmax(z: np.ndarray, tau: float = 1.0) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    if tau != 1.0:
        z = z / tau
    e = np.exp(z - np.max(z))
    return e / e.sum()


def entropy_bits(p: np.ndarray) -> float:
    p = np.asarray(p, dtype=np.float64)
    nz = p[p > 0]
    return float(-(nz * np.log2(nz)).sum())


class BiasHead:
    def __init__(self, vocab: int, lr: float = 1e-3):
        self.b = np.zeros(vocab, dtype=np.float64)
        self.lr = float(lr)

    def adjust(self, p_llm: np.ndarray) -> np.ndarray:
        with np.errstate(divide="ignore"):
            return softmax(np.log(p_llm) + self.b)

    @staticmethod
    def grad(ptilde: np.ndarray, token: int) -> np.ndarray:
        g = ptilde.copy()
        g[token] -= 1.0
        return g

    def update(self, ptilde: np.ndarray, token: int):
        self.b -= self.lr * self.grad(ptilde, token)


def initial_log_weights(n_models: int, mode: str) -> np.ndarray:
    if mode == "uniform":
        w = np.full(n_models, 1.0 / n_models)
    elif mode == "llm85":
        w = np.full(n_models, 0.15 / (n_models - 1))
        w[0] = 0.85
    else:
        raise ValueError(mode)
    return np.log(w)


class Mixer:
    def __init__(self, n_models: int = 2, init: str = "llm85", eta: float = 1.0):
        self.logw = initial_log_weights(n_models, init)
        self.eta = float(eta)

    @property
    def weights(self) -> np.ndarray:
        return np.exp(self.logw)

    def mix(self, preds) -> np.ndarray:
        w = self.weights
        return sum(w[j] * preds[j] for j in range(len(preds)))

    def update(self, preds, token: int):
        for j in range(len(preds)):
            self.logw[j] += self.eta * np.log(preds[j][token])
        self.logw -= logsumexp(self.logw)


class EnsembleGate:
    """Softmax gate over experts trained by SGD on -log p(t*) jointly with the bias vector."""

    def __init__(self, n_experts: int, vocab: int, lr: float = 1e-3):
        self.theta = np.zeros(n_experts, dtype=np.float64)
        self.b = np.zeros(vocab, dtype=np.float64)
        self.lr = float(lr)

    @staticmethod
    def forward(theta, experts):
        w = softmax(theta)
        p = sum(w[j] * experts[j] for j in range(len(experts)))
        return w, p

    @staticmethod
    def loss(theta, b, z, ngram_experts, token):
        """L = -log p(t*) as a function of (theta, b) for fixed logits and n-gram experts."""
        q0 = softmax(np.log(softmax(z)) + b)
        _, p = EnsembleGate.forward(theta, [q0] + list(ngram_experts))
        return -float(np.log(p[token]))

    @staticmethod
    def grads(theta, q0, ngram_experts, token):
        """Closed-form (dL/dtheta, dL/db) for L = -log p(t*)."""
        experts = [q0] + list(ngram_experts)
        w, p = EnsembleGate.forward(theta, experts)
        r = np.array([w[j] * experts[j][token] for j in range(len(experts))]) / p[token]
        g_theta = w - r
        g_b = r[0] * q0
        g_b[token] -= r[0]
        return g_theta, g_b

    def step(self, q0, ngram_experts, token):
        g_theta, g_b = self.grads(self.theta, q0, ngram_experts, token)
        self.theta -= self.lr * g_theta
        self.b -= self.lr * g_b
        return g_theta, g_b
