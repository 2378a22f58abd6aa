"""ctypes declarations of libnacrith.so (include/nacrith.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnacrith.so")

NC_OK, NC_E_INVALID, NC_E_DEVICE, NC_E_NOMEM, NC_E_CAPACITY, NC_E_CORRUPT, NC_E_STATE = range(7)
STATUS_NAMES = {0: "NC_OK", 1: "NC_E_INVALID", 2: "NC_E_DEVICE", 3: "NC_E_NOMEM",
                4: "NC_E_CAPACITY", 5: "NC_E_CORRUPT", 6: "NC_E_STATE"}
NC_FP32, NC_BF16, NC_FP8 = 0, 1, 2
NC_SKIP_NONE, NC_SKIP_ENTROPY, NC_SKIP_PMAX = 0, 1, 2
NC_F_HEAD, NC_F_NGRAM, NC_F_SKIP, NC_F_MIXER, NC_F_ENSEMBLE, NC_F_EAGER = 1, 2, 4, 8, 16, 32
NC_F_DECODE_GRAPHS = 64
NC_MODE_LLM, NC_MODE_SKIP, NC_MODE_MIX, NC_MODE_ENSEMBLE = 0, 1, 2, 3


class NcConfig(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("d_model", C.c_int32), ("n_heads", C.c_int32),
                ("n_kv_heads", C.c_int32), ("head_dim", C.c_int32), ("d_ffn", C.c_int32),
                ("vocab", C.c_int32), ("rope_theta", C.c_float), ("norm_eps", C.c_float),
                ("ctx_len", C.c_int32), ("slide", C.c_int32), ("ngram_order", C.c_int32),
                ("ngram_eps", C.c_float), ("ngram_max_contexts", C.c_int32),
                ("head_lr", C.c_float), ("mix_eta", C.c_float), ("mix_w_llm", C.c_float),
                ("warmup", C.c_int32), ("skip_mode", C.c_int32),
                ("skip_entropy_bits", C.c_float), ("skip_pmax", C.c_float),
                ("cdf_total", C.c_uint32), ("precision", C.c_int32), ("features", C.c_uint32),
                ("max_streams", C.c_int32)]


class NcProbe(C.Structure):
    _fields_ = [("logits", C.POINTER(C.c_float)), ("ptilde", C.POINTER(C.c_float)),
                ("p_ngram", C.POINTER(C.c_float)), ("cdf", C.POINTER(C.c_uint32)),
                ("mode", C.c_int32), ("llm_ran", C.c_int32), ("entropy_bits", C.c_float),
                ("pmax", C.c_float), ("mix_w", C.c_float * 2)]


class NcStats(C.Structure):
    _fields_ = [("tokens", C.c_uint64), ("llm_rows", C.c_uint64), ("skipped", C.c_uint64),
                ("body_rows", C.c_uint64), ("bits", C.c_double), ("ideal_bits", C.c_double),
                ("seconds", C.c_double), ("wait_seconds", C.c_double),
                ("graph_replays", C.c_uint64), ("graph_captures", C.c_uint64)]


class NcTile(C.Structure):
    _fields_ = [("gemm", C.c_int32), ("max_rows", C.c_int32), ("kind", C.c_int32),
                ("mb", C.c_int32), ("waves", C.c_int32), ("us_best", C.c_float),
                ("us_default", C.c_float)]


GEMMS = ("qkv", "oproj", "gateup", "down", "lmhead")
TILE_KINDS = ("rule", "split", "tile_small", "tile_64", "wide_128")


class NcKstat(C.Structure):
    _fields_ = [("ms", C.c_double), ("launches", C.c_uint64), ("timed", C.c_uint64),
                ("bytes", C.c_double), ("flops", C.c_double)]


KERNEL_CLASSES = {"qkv": 0, "attn": 1, "oproj": 2, "gateup": 3, "down": 4, "lmhead": 5,
                  "vocab": 6, "ngram": 7}
ALL_KERNEL_CLASSES = 8

_P = C.c_void_p
_SIG = {
    "nc_last_error": (C.c_char_p, []),
    "nc_encode_bound": (C.c_size_t, [C.c_size_t]),
    "nc_create": (C.c_int, [C.POINTER(NcConfig), _P, C.POINTER(_P)]),
    "nc_destroy": (None, [_P]),
    "nc_streams_reset": (C.c_int, [_P, C.c_uint32, C.c_uint32]),
    "nc_calibrate_fp8": (C.c_int, [_P, _P, C.c_size_t]),
    "nc_probs_for_context": (C.c_int, [_P, C.c_uint32, _P, C.c_size_t, _P, C.POINTER(NcProbe)]),
    "nc_mix_update": (C.c_int, [_P, C.c_uint32, C.c_int32]),
    "nc_quantize_cdf24": (C.c_int, [_P, C.c_uint32, C.c_uint32, C.c_uint32, _P, _P, _P]),
    "nc_quantize_cdf24_noalloc": (C.c_int, [_P, C.c_uint32, C.c_uint32, C.c_uint32, _P, _P,
                                             _P]),
    "nc_cdf_interval": (C.c_int, [_P, C.c_uint32, C.c_uint32, _P, C.c_int32, _P, _P]),
    "nc_encode_stream": (C.c_int, [_P, C.c_uint32, _P, _P, _P, _P, _P, _P]),
    "nc_decode_stream": (C.c_int, [_P, C.c_uint32, _P, _P, _P, _P]),
    "nc_get_stats": (C.c_int, [_P, C.POINTER(NcStats)]),
    "nc_profile": (C.c_int, [_P, C.c_int32, C.c_uint32]),
    "nc_autotune": (C.c_int, [_P, C.c_uint32, C.c_uint32, C.c_void_p, C.c_uint32,
                              C.POINTER(C.c_uint32)]),
    "nc_tiles_reset": (C.c_int, [_P]),
    "nc_tiles_set": (C.c_int, [_P, C.c_void_p, C.c_uint32]),
    "nc_profile_read": (C.c_int, [_P, C.c_int32, C.POINTER(NcKstat)]),
    "nc_ac_encode": (C.c_int, [_P, C.c_size_t, C.c_uint32, _P, C.c_size_t, _P, _P]),
    "nc_ac_decode_static": (C.c_int, [_P, C.c_size_t, _P, C.c_uint32, C.c_size_t, _P]),
    "nc_ensemble_forward": (C.c_int, [_P, _P, _P, _P, _P, C.c_uint32, C.c_uint32, C.c_uint32,
                                      _P, _P, _P, _P]),
    "nc_ensemble_backward": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_uint32, C.c_uint32,
                                       C.c_uint32, C.c_float, _P, _P, _P]),
}

_lib = None


class NacrithError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _hip_runtimes_mapped():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64.so" in ln})
    except OSError:
        return []


def lib():
    """The loaded library; raises if it has not been built (there is no fallback path).

    torch is imported first so that its HIP runtime is the one libnacrith binds to (both carry
    the soname libamdhip64.so.7; whichever is loaded first serves the process).  Device pointers
    and streams then belong to a single runtime.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2602_19626_amd.build`")
        import torch  # noqa: F401  (loads torch's HIP runtime before ours)
        h = C.CDLL(LIB_PATH)
        rts = _hip_runtimes_mapped()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes are mapped in this process: {rts}")
        for name, (res, args) in _SIG.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int):
    if status != NC_OK:
        raise NacrithError(status, lib().nc_last_error().decode(errors="replace"))
