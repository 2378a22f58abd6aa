"""Pins of the oracle's softmax, bias head (section 3.7), mixer (section 3.6), entropy (section 3.8)
and the ensemble-gate gradients of the differentiation workload."""
import json
import os

import numpy as np
import pytest
from scipy.special import logsumexp as sp_logsumexp
from scipy.special import softmax as sp_softmax

from oracle.head import BiasHead, EnsembleGate, Mixer, entropy_bits, logsumexp, softmax

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_softmax_and_lse_match_library():
    rng = np.random.default_rng(0)
    z = rng.normal(size=1000) * 5
    assert np.allclose(softmax(z), sp_softmax(z), rtol=1e-13, atol=0)
    assert abs(logsumexp(z) - sp_logsumexp(z)) < 1e-12
    assert np.allclose(softmax(z + 123.0), softmax(z), rtol=1e-12, atol=0)


def test_zero_bias_is_identity():
    rng = np.random.default_rng(1)
    p = sp_softmax(rng.normal(size=500))
    assert np.allclose(BiasHead(500).adjust(p), p, rtol=1e-13, atol=0)


def test_bias_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    v, t, h = 40, 17, 1e-4
    p = sp_softmax(rng.normal(size=v))
    b = rng.normal(size=v) * 0.3

    def loss(bb):
        return -np.log(sp_softmax(np.log(p) + bb)[t])

    fd = np.array([(loss(b + h * e) - loss(b - h * e)) / (2 * h) for e in np.eye(v)])
    g = BiasHead.grad(sp_softmax(np.log(p) + b), t)
    assert np.linalg.norm(g - fd) / np.linalg.norm(g) < 1e-7


def test_bias_update_step():
    head = BiasHead(5, lr=GOLD["head_lr"]["value"])
    pt = np.array([0.1, 0.2, 0.3, 0.25, 0.15])
    head.update(pt, 2)
    assert np.allclose(head.b, -1e-3 * (pt - np.eye(5)[2]), rtol=0, atol=1e-18)


def test_mixer_printed_example():
    w_llm = GOLD["mixer_example_w_llm"]["value"]
    p_llm_t = GOLD["mixer_example_p_llm"]["value"]
    m = Mixer(2, "llm85")
    assert abs(m.weights.sum() - 1.0) < 1e-15
    assert abs(m.weights[0] - w_llm) < 1e-15
    a = np.array([p_llm_t, 1 - p_llm_t])
    for q in (0.0, 0.3, 1.0):
        b = np.array([q, 1 - q])
        assert m.mix([a, b])[0] >= GOLD["mixer_example_lower_bound"]["value"] - 1e-15
    assert abs(m.mix([a, np.array([0.0, 1.0])])[0] - 0.765) < 1e-15


def test_mixer_is_bayes_posterior_with_eta_one():
    rng = np.random.default_rng(3)
    v = 6
    m = Mixer(3, "uniform")
    preds_seq = [[sp_softmax(rng.normal(size=v)) for _ in range(3)] for _ in range(30)]
    toks = rng.integers(0, v, size=30)
    prior = np.full(3, 1 / 3)
    log_post = np.log(prior)
    for preds, t in zip(preds_seq, toks):
        m.update(preds, int(t))
        log_post += np.log([pp[t] for pp in preds])
    post = np.exp(log_post - sp_logsumexp(log_post))
    assert np.allclose(m.weights, post, rtol=1e-12, atol=0)
    assert abs(m.weights.sum() - 1) < 1e-14


def test_entropy_bits():
    assert abs(entropy_bits(np.full(512, 1 / 512)) - 9.0) < 1e-12
    e = np.zeros(10)
    e[3] = 1
    assert entropy_bits(e) == 0.0
    assert abs(entropy_bits(np.array([0.5, 0.25, 0.25])) - 1.5) < 1e-15


@pytest.mark.parametrize("seed", range(3))
def test_ensemble_gradients_match_central_differences(seed):
    rng = np.random.default_rng(10 + seed)
    v, t, h = 30, 4, 1e-4
    z = rng.normal(size=v)
    ng = [sp_softmax(rng.normal(size=v) * 2) for _ in range(4)]
    theta = rng.normal(size=5) * 0.5
    b = rng.normal(size=v) * 0.2
    q0 = sp_softmax(np.log(sp_softmax(z)) + b)
    g_th, g_b = EnsembleGate.grads(theta, q0, ng, t)
    fd_th = np.array([(EnsembleGate.loss(theta + h * e, b, z, ng, t)
                       - EnsembleGate.loss(theta - h * e, b, z, ng, t)) / (2 * h)
                      for e in np.eye(5)])
    fd_b = np.array([(EnsembleGate.loss(theta, b + h * e, z, ng, t)
                      - EnsembleGate.loss(theta, b - h * e, z, ng, t)) / (2 * h)
                     for e in np.eye(v)])
    assert np.linalg.norm(g_th - fd_th) / np.linalg.norm(fd_th) < 1e-6
    assert np.linalg.norm(g_b - fd_b) / np.linalg.norm(fd_b) < 1e-6
    assert abs(g_th.sum()) < 1e-14                 # softmax gate: gradient sums to zero


def test_ensemble_reduces_to_head_gradient_for_one_expert():
    rng = np.random.default_rng(5)
    v, t = 20, 3
    q0 = sp_softmax(rng.normal(size=v))
    g_th, g_b = EnsembleGate.grads(np.zeros(1), q0, [], t)
    assert np.allclose(g_b, BiasHead.grad(q0, t), rtol=0, atol=1e-16)
    assert abs(g_th[0]) < 1e-16
