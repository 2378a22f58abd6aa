"""Pins of the oracle's FP64 transformer (paper section 3.2 Eq. (lm), section 3.10 slide)."""
import dataclasses

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth
from oracle.transformer import Transformer, rmsnorm


def _tiny(**over):
    return dataclasses.replace(synth.TINY, **over)


def _torch_reference(shape, w, tokens):
    """Independent float64 composition from torch library routines (no slide: n <= L).

    RoPE is applied as a complex rotation (x1 + i x2) * exp(i pos omega), a different formulation
    from the oracle's rotate-half cosine/sine form.
    """
    t = {k: torch.tensor(v, dtype=torch.float64) for k, v in w.items()}
    n = len(tokens)
    hq, hk, hd, d = shape.n_heads, shape.n_kv_heads, shape.head_dim, shape.d_model
    omega = torch.tensor(shape.rope_theta, dtype=torch.float64) ** (
        -torch.arange(0, hd, 2, dtype=torch.float64) / hd)
    rot = torch.polar(torch.ones(n, hd // 2, dtype=torch.float64),
                      torch.arange(n, dtype=torch.float64)[:, None] * omega[None, :])

    def rope(x):                                   # x [n, heads, hd]
        c = torch.complex(x[..., :hd // 2], x[..., hd // 2:]) * rot[:, None, :]
        return torch.cat([c.real, c.imag], dim=-1)

    x = t["E"][torch.tensor(tokens)]
    for l in range(shape.n_layers):
        p = f"l{l}."
        y = F.rms_norm(x, (d,), t[p + "attn_norm"], eps=shape.norm_eps)
        q = rope(F.linear(y, t[p + "Wq"]).view(n, hq, hd)).transpose(0, 1)
        k = rope(F.linear(y, t[p + "Wk"]).view(n, hk, hd)).transpose(0, 1)
        v = F.linear(y, t[p + "Wv"]).view(n, hk, hd).transpose(0, 1)
        o = F.scaled_dot_product_attention(q[None], k[None], v[None], is_causal=True,
                                           enable_gqa=True)[0]
        x = x + F.linear(o.transpose(0, 1).reshape(n, hq * hd), t[p + "Wo"])
        y = F.rms_norm(x, (d,), t[p + "mlp_norm"], eps=shape.norm_eps)
        x = x + F.linear(F.silu(F.linear(y, t[p + "Wg"])) * F.linear(y, t[p + "Wu"]), t[p + "Wd"])
    h = F.rms_norm(x, (d,), t["final_norm"], eps=shape.norm_eps)
    return F.linear(h, t["E"]).numpy()


@pytest.mark.parametrize("shape", [synth.TINY, _tiny(n_heads=2, n_kv_heads=2),
                                   _tiny(n_heads=4, n_kv_heads=1, n_layers=3)])
def test_matches_torch_library_composition(shape):
    w = synth.make_weights(shape, seed=5)
    for name in w:                                  # non-trivial gains exercise every norm
        if name.endswith("norm"):
            w[name] = (1 + 0.1 * np.random.default_rng(9).normal(size=w[name].shape)).astype(
                np.float32)
    toks = synth.make_stream(100, shape.vocab, seed=3)
    m = Transformer(shape, w, max_block=37)
    z = m.logits(m.append(np.concatenate([[0], toks[:-1]])))
    ref = _torch_reference(shape, w, np.concatenate([[0], toks[:-1]]))
    assert np.max(np.abs(z - ref)) < 1e-12


def test_blocked_equals_token_by_token():
    shape = _tiny(ctx_len=16, slide=4)
    w = synth.make_weights(shape, seed=1)
    toks = synth.make_stream(60, shape.vocab, seed=2)
    a = Transformer(shape, w, max_block=64)
    b = Transformer(shape, w, max_block=1)
    za = a.logits(a.append(toks))
    zb = np.concatenate([b.logits(b.append([t])) for t in toks])
    assert a.n_slides == b.n_slides == (60 - 16 + 3) // 4
    assert np.max(np.abs(za - zb)) < 1e-12


def test_rope_relative_shift_invariance():
    shape = synth.TINY
    w = synth.make_weights(shape, seed=2)
    m = Transformer(shape, w)
    rng = np.random.default_rng(0)
    q = rng.normal(size=(5, 1, shape.head_dim))
    k = rng.normal(size=(5, 1, shape.head_dim))
    pq, pk = np.arange(5) + 7.0, np.arange(5) * 3.0
    s0 = np.einsum("ihd,jhd->ij", m.rope(q, pq), m.rope(k, pk))
    s1 = np.einsum("ihd,jhd->ij", m.rope(q, pq + 512), m.rope(k, pk + 512))
    assert np.max(np.abs(s0 - s1)) < 1e-10
    # rotating by +C then by -C is the identity (the slide's re-rotation)
    assert np.max(np.abs(m.rope(m.rope(k, pk + 32), np.full(5, -32.0)) - m.rope(k, pk))) < 1e-13


def test_slide_keeps_stale_entries_and_matches_absolute_positions():
    shape = _tiny(ctx_len=16, slide=4)
    w = synth.make_weights(shape, seed=4)
    toks = synth.make_stream(16, shape.vocab, seed=5)
    m = Transformer(shape, w)
    m.append(toks)
    before_k = [k.copy() for k in m.K]
    before_v = [v.copy() for v in m.V]
    m.append([toks[0]])                             # triggers a slide, then one append
    assert m.n_slides == 1 and m.cache_len == 13
    for l in range(shape.n_layers):
        assert np.array_equal(m.V[l][:12], before_v[l][4:])           # values never recomputed
        back = m.rope(m.K[l][:12], np.full(12, 4.0))                  # undo the -C re-rotation
        assert np.max(np.abs(back - before_k[l][4:])) < 1e-13


def test_single_key_attention_returns_value():
    shape = _tiny(n_layers=1)
    w = synth.make_weights(shape, seed=6)
    # with one cached key the softmax weight is exactly 1, so x after attention is
    # E[t] + v Wo^T: check it through a model whose MLP is zeroed.
    w["l0.Wd"][:] = 0
    w["final_norm"][:] = 1
    m = Transformer(shape, w)
    h = m.append([7])
    e = w["E"][7].astype(np.float64)
    y = rmsnorm(e, 1.0, shape.norm_eps)
    v = y @ w["l0.Wv"].astype(np.float64).T                 # [hk*hd]
    grp = shape.n_heads // shape.n_kv_heads
    o = np.concatenate([v[(h_ // grp) * shape.head_dim:(h_ // grp + 1) * shape.head_dim]
                        for h_ in range(shape.n_heads)])
    x = e + o @ w["l0.Wo"].astype(np.float64).T
    assert np.max(np.abs(h[0] - rmsnorm(x, 1.0, shape.norm_eps))) < 1e-13


def test_zero_layer_model_is_normed_embedding_product():
    shape = _tiny(n_layers=0)
    w = synth.make_weights(shape, seed=8)
    m = Transformer(shape, w)
    z = m.logits(m.append([3, 9, 400]))
    e = w["E"].astype(np.float64)
    for i, t in enumerate([3, 9, 400]):
        ref = (e[t] / np.sqrt(np.mean(e[t] ** 2) + shape.norm_eps)) @ e.T
        assert np.max(np.abs(z[i] - ref)) < 1e-13


def test_operand_noise_hook_is_off_by_default_and_reaches_every_product():
    """The error-model hook: an identity callable leaves every logit bit-identical; a callable that
    scales one kind of operand by (1 + u) moves the logits, and scaling the output copy of E alone
    scales the logits by exactly (1 + u) (the embedding lookup keeps the exact E)."""
    w = synth.make_weights(synth.TINY, 0)
    toks = [0, 5, 9, 3, 3, 7, 100, 2]
    ref = Transformer(synth.TINY, w)
    z0 = ref.logits(ref.append(toks))
    seen = set()

    def ident(a, kind):
        seen.add(kind)
        return a
    m = Transformer(synth.TINY, w, operand_noise=ident)
    assert np.array_equal(m.logits(m.append(toks)), z0)
    assert seen == {"weight", "act", "att"}
    for kind in ("act", "att"):
        m = Transformer(synth.TINY, w, operand_noise=lambda a, k: a * 1.01 if k == kind else a)
        assert np.max(np.abs(m.logits(m.append(toks)) - z0)) > 1e-6, kind
    e_only = {"n": 0}

    def head_only(a, kind):
        if kind == "weight" and a.shape == w["E"].shape:
            e_only["n"] += 1
            return a * 2.0
        return a
    m = Transformer(synth.TINY, w, operand_noise=head_only)
    assert e_only["n"] == 1
    assert np.array_equal(m.logits(m.append(toks)), 2.0 * z0)


def test_precision_tolerances_file_matches_the_parity_test():
    """The stored error-model tolerances cover the parity test's positions, and each format's
    stored value is the largest over its seeds."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "precision_tolerances.json")
    d = json.load(open(path))
    assert max(d["positions"]) >= 2048
    for f, u in (("bf16", 2.0 ** -8), ("fp8", 2.0 ** -4)):
        assert d[f]["u_weights_activations"] == u and d[f]["u_attention"] == 2.0 ** -8
        assert d[f]["max_abs_logit"] == max(r["max_abs_logit"] for r in d[f]["runs"])
        assert d[f]["mean_kl_bits"] == max(r["mean_kl_bits"] for r in d[f]["runs"])
    assert d["bf16"]["max_abs_logit"] < d["fp8"]["max_abs_logit"]
