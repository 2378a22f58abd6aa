"""MI355X (gfx950) per-token probability pipeline of the Nacrith compressor (arXiv 2602.19626).

Thin Python binding of libnacrith.so (include/nacrith.h): argument marshalling only; every step
of the pipeline runs in the library's HIP kernels and its host coder.  Device buffers are torch
tensors on the current HIP device; torch supplies memory and streams, nothing else.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (NC_BF16, NC_F_DECODE_GRAPHS, NC_F_EAGER, NC_F_ENSEMBLE, NC_F_HEAD,
                   NC_F_MIXER, NC_F_NGRAM, NC_F_SKIP, NC_FP8,
                   NC_FP32, NC_SKIP_ENTROPY, NC_SKIP_NONE, NC_SKIP_PMAX, NacrithError, NcConfig,
                   NcProbe, NcStats, check, lib)

__all__ = ["quantize_cdf24", "quantize_cdf24_noalloc", "cdf_interval", "encode_bound", "ac_encode", "ac_decode_static",
           "make_config", "Context", "NacrithError", "lib"]

PRECISIONS = {"fp32": NC_FP32, "bf16": NC_BF16, "fp8": NC_FP8}
SKIP_MODES = {"none": NC_SKIP_NONE, "entropy": NC_SKIP_ENTROPY, "pmax": NC_SKIP_PMAX}


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on a HIP device")
    return C.c_void_p(t.data_ptr())


def quantize_cdf24(probs, total: int = 1 << 24, stream=None):
    """CDF-24 of each row of probs (float32 [rows, V] on the GPU) -> (cdf uint32-as-int32
    [rows, V+1], status int32 [rows]) on the same device (section 3.4)."""
    import torch
    if probs.dim() == 1:
        probs = probs[None]
    rows, v = probs.shape
    cdf = torch.empty((rows, v + 1), dtype=torch.int32, device=probs.device)
    st = torch.empty(rows, dtype=torch.int32, device=probs.device)
    check(lib().nc_quantize_cdf24(_dev_ptr(probs, torch.float32, "probs"), rows, v, total,
                                  _dev_ptr(cdf, torch.int32, "cdf"),
                                  _dev_ptr(st, torch.int32, "status"), _stream_ptr(stream)))
    return cdf, st


def quantize_cdf24_noalloc(probs, cdf, status, total: int = 1 << 24, stream=None):
    """nc_quantize_cdf24_noalloc into caller-allocated cdf (int32 [rows, V+1]) and status
    (int32 [rows]) tensors: the library allocates nothing (its workspace is a fixed device
    array shared by every call on the GPU)."""
    import torch
    if probs.dim() == 1:
        probs = probs[None]
    rows, v = probs.shape
    if tuple(cdf.shape) != (rows, v + 1) or tuple(status.shape) != (rows,):
        raise ValueError("cdf must be [rows, V+1] and status [rows]")
    check(lib().nc_quantize_cdf24_noalloc(_dev_ptr(probs, torch.float32, "probs"), rows, v, total,
                                          _dev_ptr(cdf, torch.int32, "cdf"),
                                          _dev_ptr(status, torch.int32, "status"),
                                          _stream_ptr(stream)))
    return cdf, status


def cdf_interval(cdf, keys, mode: int, stream=None):
    """(s, cdf[s], cdf[s+1]) per row: mode 0 key = symbol, mode 1 key = target count."""
    import torch
    rows = cdf.shape[0]
    out = torch.empty((rows, 3), dtype=torch.int32, device=cdf.device)
    check(lib().nc_cdf_interval(_dev_ptr(cdf, torch.int32, "cdf"), rows, cdf.shape[1] - 1,
                                _dev_ptr(keys, torch.int32, "keys"), mode,
                                _dev_ptr(out, torch.int32, "out"), _stream_ptr(stream)))
    return out


def encode_bound(n_tokens: int) -> int:
    return int(lib().nc_encode_bound(n_tokens))


def ac_encode(intervals: np.ndarray, total: int = 1 << 24):
    """Host arithmetic coder: (bytes, exact bit count) of a sequence of (cl, ch) intervals."""
    iv = np.ascontiguousarray(intervals, dtype=np.uint32).reshape(-1, 2)
    cap = encode_bound(len(iv))
    buf = (C.c_uint8 * cap)()
    nb, bits = C.c_size_t(), C.c_uint64()
    check(lib().nc_ac_encode(iv.ctypes.data, len(iv), total, buf, cap, C.byref(nb), C.byref(bits)))
    return bytes(buf[:nb.value]), bits.value


def ac_decode_static(data: bytes, cdf: np.ndarray, n: int) -> np.ndarray:
    """Host arithmetic decoder for n symbols all coded against one CDF."""
    c = np.ascontiguousarray(cdf, dtype=np.uint32)
    out = np.zeros(n, dtype=np.int32)
    src = (C.c_uint8 * max(1, len(data))).from_buffer_copy(data if data else b"\0")
    check(lib().nc_ac_decode_static(src, len(data), c.ctypes.data, len(c) - 1, n,
                                    out.ctypes.data))
    return out


def make_config(shape, *, ngram_order=4, precision="fp32", skip="entropy", mix_init="llm85",
                warmup=100, head_lr=1e-3, cdf_total=1 << 24, max_streams=1, use_head=True,
                use_ngram=True, use_skip=True, use_mixer=True, ensemble=False,
                ngram_eps=5.0, ngram_max_contexts=500_000, mix_eta=1.0,
                skip_entropy_bits=1.5, skip_pmax=0.99, graphs=True,
                decode_graphs=False) -> NcConfig:
    """nc_config from a model shape (any object with the ModelShape fields) and options."""
    feats = ((NC_F_HEAD if use_head else 0) | (NC_F_NGRAM if use_ngram else 0)
             | (NC_F_SKIP if (use_skip and skip != "none") else 0)
             | (NC_F_MIXER if use_mixer else 0) | (NC_F_ENSEMBLE if ensemble else 0)
             | (0 if graphs else NC_F_EAGER) | (NC_F_DECODE_GRAPHS if decode_graphs else 0))
    return NcConfig(n_layers=shape.n_layers, d_model=shape.d_model, n_heads=shape.n_heads,
                    n_kv_heads=shape.n_kv_heads, head_dim=shape.head_dim, d_ffn=shape.d_ffn,
                    vocab=shape.vocab, rope_theta=shape.rope_theta, norm_eps=shape.norm_eps,
                    ctx_len=shape.ctx_len, slide=shape.slide, ngram_order=ngram_order,
                    ngram_eps=ngram_eps, ngram_max_contexts=ngram_max_contexts, head_lr=head_lr,
                    mix_eta=mix_eta, mix_w_llm=0.5 if mix_init == "uniform" else 0.85,
                    warmup=warmup, skip_mode=SKIP_MODES[skip],
                    skip_entropy_bits=skip_entropy_bits, skip_pmax=skip_pmax,
                    cdf_total=cdf_total, precision=PRECISIONS[precision], features=feats,
                    max_streams=max_streams)


class Context:
    """Owns an nc_ctx: device weights and per-stream state."""

    def __init__(self, cfg: NcConfig, weights_flat: np.ndarray):
        w = np.ascontiguousarray(weights_flat, dtype=np.float32)
        h = C.c_void_p()
        check(lib().nc_create(C.byref(cfg), w.ctypes.data, C.byref(h)))
        self._h = h
        self.cfg = cfg

    def close(self):
        if getattr(self, "_h", None):
            lib().nc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, n_streams: int, max_tokens: int):
        check(lib().nc_streams_reset(self._h, n_streams, max_tokens))

    def calibrate_fp8(self, tokens):
        t = np.ascontiguousarray(tokens, dtype=np.int32)
        check(lib().nc_calibrate_fp8(self._h, t.ctypes.data, len(t)))

    def probs_for_context(self, stream: int, tokens, probe: bool = False):
        """Coding distribution (float32 [V]) for the position after tokens; with probe=True also
        a dict of diagnostics (logits, ptilde, p_ngram, cdf, mode, ...)."""
        v = self.cfg.vocab
        t = np.ascontiguousarray(tokens, dtype=np.int32)
        p = np.zeros(v, dtype=np.float32)
        pr = None
        if probe:
            arrs = dict(logits=np.zeros(v, np.float32), ptilde=np.zeros(v, np.float32),
                        p_ngram=np.zeros(v, np.float32), cdf=np.zeros(v + 1, np.uint32))
            pr = NcProbe(logits=arrs["logits"].ctypes.data_as(C.POINTER(C.c_float)),
                         ptilde=arrs["ptilde"].ctypes.data_as(C.POINTER(C.c_float)),
                         p_ngram=arrs["p_ngram"].ctypes.data_as(C.POINTER(C.c_float)),
                         cdf=arrs["cdf"].ctypes.data_as(C.POINTER(C.c_uint32)))
        check(lib().nc_probs_for_context(self._h, stream, t.ctypes.data, len(t), p.ctypes.data,
                                         C.byref(pr) if pr is not None else None))
        if not probe:
            return p
        arrs.update(mode=pr.mode, llm_ran=pr.llm_ran, entropy_bits=pr.entropy_bits,
                    pmax=pr.pmax, mix_w=(pr.mix_w[0], pr.mix_w[1]))
        return p, arrs

    def mix_update(self, stream: int, token: int):
        check(lib().nc_mix_update(self._h, stream, int(token)))

    def encode_stream(self, streams):
        """Compress a list of int token arrays; returns (list of bytes, list of bit counts)."""
        n = len(streams)
        arrs = [np.ascontiguousarray(s, dtype=np.int32) for s in streams]
        toks = (C.c_void_p * n)(*[a.ctypes.data for a in arrs])
        lens = (C.c_size_t * n)(*[len(a) for a in arrs])
        caps = [encode_bound(len(a)) for a in arrs]
        bufs = [(C.c_uint8 * c)() for c in caps]
        outs = (C.c_void_p * n)(*[C.addressof(b) for b in bufs])
        capa = (C.c_size_t * n)(*caps)
        nbytes = (C.c_size_t * n)()
        nbits = (C.c_uint64 * n)()
        check(lib().nc_encode_stream(self._h, n, toks, lens, outs, capa, nbytes, nbits))
        return [bytes(bufs[i][:nbytes[i]]) for i in range(n)], [int(nbits[i]) for i in range(n)]

    def decode_stream(self, datas, n_tokens):
        n = len(datas)
        srcs = [(C.c_uint8 * max(1, len(d))).from_buffer_copy(d if d else b"\0") for d in datas]
        ins = (C.c_void_p * n)(*[C.addressof(s) for s in srcs])
        inb = (C.c_size_t * n)(*[len(d) for d in datas])
        lens = (C.c_size_t * n)(*[int(k) for k in n_tokens])
        outs = [np.zeros(int(k), dtype=np.int32) for k in n_tokens]
        outp = (C.c_void_p * n)(*[o.ctypes.data for o in outs])
        check(lib().nc_decode_stream(self._h, n, ins, inb, lens, outp))
        return outs

    def autotune(self, max_rows: int, reps: int = 10) -> list:
        """Time every launch shape of each GEMM per row bucket up to max_rows and keep the
        fastest (results are bit-identical across shapes).  Streams must be reset afterwards."""
        from ._lib import GEMMS, TILE_KINDS, NcTile
        cap = 5 * 32
        arr = (NcTile * cap)()
        n = C.c_uint32()
        check(lib().nc_autotune(self._h, int(max_rows), int(reps), arr, cap, C.byref(n)))
        out = []
        for t in arr[:min(n.value, cap)]:
            out.append({"gemm": GEMMS[t.gemm], "max_rows": t.max_rows, "kind": TILE_KINDS[t.kind],
                        "mb": t.mb, "waves": t.waves, "us_best": t.us_best,
                        "us_default": t.us_default})
        return out

    def tiles_set(self, entries):
        """Install launch shapes: dicts with gemm, max_rows, kind (names as autotune() returns
        them) and, for split shapes, mb and waves."""
        from ._lib import GEMMS, TILE_KINDS, NcTile
        arr = (NcTile * max(1, len(entries)))()
        for i, e in enumerate(entries):
            arr[i] = NcTile(GEMMS.index(e["gemm"]), int(e["max_rows"]),
                            TILE_KINDS.index(e["kind"]), int(e.get("mb", 0)),
                            int(e.get("waves", 0)), 0.0, 0.0)
        check(lib().nc_tiles_set(self._h, arr, len(entries)))

    def tiles_reset(self):
        """Back to the fixed launch-shape rule."""
        check(lib().nc_tiles_reset(self._h))

    def profile(self, kernel_class, stride: int = 1):
        """Time every stride-th launch of a kernel class ("all" = every class; None = off) with
        HIP events on the stream the class runs on."""
        from ._lib import ALL_KERNEL_CLASSES, KERNEL_CLASSES
        cls = -1 if kernel_class is None else (
            ALL_KERNEL_CLASSES if kernel_class == "all" else KERNEL_CLASSES[kernel_class])
        check(lib().nc_profile(self._h, cls, int(stride)))

    def profile_read(self, kernel_class) -> dict:
        from ._lib import KERNEL_CLASSES, NcKstat
        k = NcKstat()
        check(lib().nc_profile_read(self._h, KERNEL_CLASSES[kernel_class], C.byref(k)))
        return {f: getattr(k, f) for f, _ in NcKstat._fields_}

    def stats(self) -> dict:
        s = NcStats()
        check(lib().nc_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in NcStats._fields_}
