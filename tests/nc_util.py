"""Helpers shared by the GPU tests: contexts for a synthetic workload, oracle settings."""
import numpy as np

import synth


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def make_context(wl, precision=None, max_streams=None, **over):
    import paper_2602_19626_amd as nc
    shape = over.pop("shape", wl.shape)
    cfg = nc.make_config(shape, ngram_order=wl.ngram_order,
                         precision=precision or wl.precision, skip=wl.skip,
                         mix_init=wl.mix_init, warmup=wl.warmup, head_lr=wl.head_lr,
                         cdf_total=wl.cdf_total, max_streams=max_streams or wl.n_streams,
                         ensemble=wl.ensemble, **over)
    w = synth.make_weights(shape, wl.weight_seed)
    return nc.Context(cfg, synth.flat_weights(shape, w)), w


def kl_bits(p, q):
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    m = p > 0
    return float(np.sum(p[m] * (np.log2(p[m]) - np.log2(q[m]))))
