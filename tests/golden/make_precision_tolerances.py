"""Writes precision_tolerances.json: the reduced-precision tolerances of the 135M-shape parity test
(tests/test_gpu_full.py), derived from an error model run on the FP64 oracle alone.

Model: every operand of every matrix product is multiplied by (1 + d), d uniform in [-u, u] and
independent per element, where u is the unit roundoff of the format the product runs in:
  BF16: 8 significand bits, u = 2^-8 (weights, activations and the attention operands);
  FP8 e4m3: 4 significand bits, u = 2^-4 (weights and activations); the attention runs in BF16,
    u = 2^-8 there.
Round-to-nearest errs by at most u relative (for normal values) and by u/sqrt(2) RMS over
mantissas, so the uniform +-u model overstates the rounding noise by about sqrt(2) in standard
deviation.  The tolerance of a format is the largest max |logit error| and the largest mean
KL(p_llm exact || p_llm perturbed) over the model's seeds, on the same 2,200-token stream and
positions as the parity test.

Run: python tests/golden/make_precision_tolerances.py   (about two minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.head import softmax  # noqa: E402
from oracle.transformer import Transformer  # noqa: E402

N = 2200
POS = [0, 1, 2, 99, 100, 101, 500, 1000, 1500, 2046, 2047, 2048, 2049, 2100, 2199]
FORMATS = {"bf16": (2.0 ** -8, 2.0 ** -8), "fp8": (2.0 ** -4, 2.0 ** -8)}
SEEDS = (0, 1)


def logits_at(shape, weights, tokens, noise):
    m = Transformer(shape, weights, max_block=512, operand_noise=noise)
    x = np.concatenate([[0], tokens[:-1]])            # BOS, then teacher forcing
    return m.logits(m.append(x)[POS])


def perturbation(u_main, u_att, seed):
    rng = np.random.default_rng(seed)

    def f(a, kind):
        u = u_att if kind == "att" else u_main
        return a * (1.0 + rng.uniform(-u, u, a.shape))
    return f


def kl_bits(p, q):
    return float(np.sum(p * (np.log2(p) - np.log2(q))))


def main():
    wl = synth.WORKLOADS["full_fp32"]
    w = synth.make_weights(wl.shape, wl.weight_seed)
    toks = synth.workload_streams(wl, max_len=N)[0]
    z0 = logits_at(wl.shape, w, toks, None)
    p0 = [softmax(z) for z in z0]
    out = {"_about": __doc__.split("\n\n")[0].replace("\n", " "),
           "workload": "full_fp32 stream (seed 2), first 2,200 tokens; weights seed 1",
           "positions": POS, "seeds": list(SEEDS)}
    for name, (um, ua) in FORMATS.items():
        runs = []
        for seed in SEEDS:
            z = logits_at(wl.shape, w, toks, perturbation(um, ua, seed))
            d = np.abs(z - z0)
            kl = np.mean([kl_bits(p0[i], softmax(z[i])) for i in range(len(POS))])
            runs.append({"seed": seed, "max_abs_logit": float(d.max()),
                         "rms_logit": float(np.sqrt(np.mean(d ** 2))), "mean_kl_bits": float(kl)})
            print(name, runs[-1], flush=True)
        out[name] = {"u_weights_activations": um, "u_attention": ua, "runs": runs,
                     "max_abs_logit": max(r["max_abs_logit"] for r in runs),
                     "mean_kl_bits": max(r["mean_kl_bits"] for r in runs)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_tolerances.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
