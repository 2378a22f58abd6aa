"""Throughput of the per-token probability pipeline on one MI355X: tokens/s encode+decode.

One step = encode every stream of the workload and decode it again (the whole hot path:
transformer forward over the sliding KV cache, vocabulary softmax with the bias head, n-gram,
mixer and skip, CDF-24 quantisation, host arithmetic coder).  Inputs are the seeded synthetic
streams and random-init weights of the workload; they are resident on the host before the timed
region and the weights are resident in HBM.

Prints one JSON line with the headline value, the roofline of the profiled kernel class (timed
live with HIP events on the library's stream) and the FP64 oracle timed on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tokens/s encode+decode (135M-shape LM + CDF-24), bpb gap vs FP64 oracle"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}   # dense, published
KERNEL_SOURCES = {"qkv": "k_llm.hip", "attn": "k_llm.hip", "oproj": "k_llm.hip",
                  "gateup": "k_llm.hip", "down": "k_llm.hip", "lmhead": "k_llm.hip",
                  "vocab": "k_vocab.hip", "ngram": "k_vocab.hip"}


# rocprofv3 kernel names of each class (demangled); oproj and down share one kernel and have none
KERNEL_NAME_RE = {"qkv": r"gemm_\w*kernel<\d+, \d+, 3\b", "gateup": r"gemm_\w*kernel<\d+, \d+, 2\b",
                  "lmhead": r"gemm_\w*kernel<\d+, \d+, 0\b", "attn": r"attention_\w*kernel",
                  "vocab": r"(vocab_\w*|ensemble_bias)_kernel", "ngram": r"ngram_\w*_kernel"}
# one dispatch per class launch matches these (a class launch may run several kernels)
KERNEL_PRIMARY_RE = {"attn": r"attention_(quad|seq)_kernel", "vocab": r"vocab_lse_kernel",
                     "ngram": r"ngram_dense_kernel"}
PROBE_RE = r"neg"   # the plain streaming probe kernel (torch.neg: reads N bytes, writes N bytes)


def kernel_source_hash(kernel: str) -> str:
    p = os.path.join(ROOT, "paper_2602_19626_amd", "csrc", KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 counters, if taken on the current source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    t = json.load(open(p))
    if t.get("source_sha") != kernel_source_hash(kernel):
        return None
    return t.get("bytes_per_launch")


def traffic_from(fetch_csv: str, write_csv: str, kernel: str, workload: str, probe_mib: int,
                 command: str) -> dict:
    """HBM bytes per launch of a kernel class from two rocprofv3 --pmc counter files (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch), each scaled by the same counter's reading for the streaming
    probe of known size; written to profiles/traffic_<kernel>_<workload>.json."""
    def per_kernel(path, counter):
        out = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] == counter:
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]) * 1024.0)
        return out
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    probe_bytes = probe_mib * (1 << 20)

    def pick(d, pat):
        return [v for name, vals in d.items() if re.search(pat, name) for v in vals]
    pf, pw = pick(f, PROBE_RE), pick(w, PROBE_RE)
    assert len(pf) == 1 and len(pw) == 1, "expected exactly one probe dispatch per counter run"
    fscale, wscale = probe_bytes / pf[0], probe_bytes / pw[0]
    kf, kw = pick(f, KERNEL_NAME_RE[kernel]), pick(w, KERNEL_NAME_RE[kernel])
    assert kf and kw, f"no {kernel} dispatches in the counter files"
    prim = KERNEL_PRIMARY_RE.get(kernel, KERNEL_NAME_RE[kernel])
    launches = len(pick(f, prim))
    assert launches > 0 and launches == len(pick(w, prim)), "counter runs disagree on launches"
    fb = sum(kf) / launches * fscale
    wb = sum(kw) / launches * wscale
    t = {"kernel": kernel, "workload": workload, "source_sha": kernel_source_hash(kernel),
         "launches": launches, "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
         "bytes_per_launch": round(fb + wb), "probe_bytes": probe_bytes,
         "fetch_scale": round(fscale, 5), "write_scale": round(wscale, 5), "command": command}
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    json.dump(t, open(path, "w"), indent=1)
    return t


def cdf24_standalone(nc, torch, vocab: int, rows_list=(64, 1024), reps: int = 20):
    """nc_quantize_cdf24 alone on float32 rows of softmax-shaped probabilities (up to 64 rows the
    segment reduce + scan kernels, more rows the one-workgroup-per-row kernel); algorithmic bytes
    per row = read 4V + write 4(V + 1)."""
    out = []
    g = torch.Generator(device="cuda").manual_seed(5)
    for rows in rows_list:
        z = torch.randn(rows, vocab, device="cuda", generator=g) * 3.0
        p = torch.softmax(z, dim=1).contiguous()
        nc.quantize_cdf24(p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            nc.quantize_cdf24(p)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1000.0 / reps
        gbs = rows * (8 * vocab + 4) / (us * 1e-6) / 1e9
        out.append({"rows": rows, "vocab": vocab, "us_per_call": round(us, 2),
                    "achieved_GBps": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)})
    return out


# The paper's incremental feature ladder (ablation table), on synthetic streams.
ABLATION = [
    ("A0: LLM + coder, CDF-16", dict(cdf_total=1 << 16, use_head=False, use_ngram=False,
                                     use_skip=False, use_mixer=False)),
    ("A1: + CDF-24", dict(cdf_total=1 << 24, use_head=False, use_ngram=False, use_skip=False,
                          use_mixer=False)),
    ("A2: + adaptive head", dict(cdf_total=1 << 24, use_head=True, use_ngram=False,
                                 use_skip=False, use_mixer=False)),
    ("A3: + n-gram + skip", dict(cdf_total=1 << 24, use_head=True, use_ngram=True, use_skip=True,
                                 use_mixer=False)),
    ("A4: full system", dict(cdf_total=1 << 24, use_head=True, use_ngram=True, use_skip=True,
                             use_mixer=True)),
]


def ablation(nc, wl, weights, streams, n_oracle: int):
    """Each ladder step: GPU encode + decode of the streams (bits, rate, round trip) and, on a
    prefix of the first stream, the FP64 oracle's coded bits for the same switches."""
    import synth
    from oracle import pipeline as op
    rows = []
    n_tok = int(sum(len(x) for x in streams))
    for name, over in ABLATION:
        cfg = nc.make_config(wl.shape, ngram_order=wl.ngram_order, precision=wl.precision,
                             skip=wl.skip, mix_init=wl.mix_init, warmup=wl.warmup,
                             head_lr=wl.head_lr, max_streams=len(streams), **over)
        ctx = nc.Context(cfg, synth.flat_weights(wl.shape, weights))
        t0 = time.perf_counter()
        data, bits = ctx.encode_stream(streams)
        out = ctx.decode_stream(data, [len(x) for x in streams])
        dt = time.perf_counter() - t0
        ok = all(np.array_equal(a, b) for a, b in zip(out, streams))
        st = ctx.stats()
        pre = streams[0][:n_oracle]
        _, pb = ctx.encode_stream([pre])
        ref = op.encode(op.Settings.from_workload(wl, **over), wl.shape, weights, pre)
        bpt = float(sum(bits)) / n_tok
        rows.append({"config": name, "bits_per_token": round(bpt, 5),
                     "bpb_at_4_bytes_per_token": round(bpt / 4.0, 5),
                     "tok_s_encode_decode": round(n_tok / dt, 1),
                     "skip_rate": round(st["skipped"] / max(st["tokens"], 1), 4),
                     "roundtrip_exact": bool(ok),
                     "oracle_prefix_tokens": len(pre),
                     "gpu_minus_oracle_bits_per_token_prefix":
                         round((float(pb[0]) - float(ref.n_bits)) / len(pre), 5)})
    return rows


def cpu_baseline(wl, weights, stream, n_sample: int):
    """The oracle (FP64 numpy + exact integer quantiser + Python-integer coder) on a prefix."""
    from threadpoolctl import threadpool_info
    from oracle import pipeline as op
    s = op.Settings.from_workload(wl)
    toks = stream[:n_sample]
    t0 = time.perf_counter()
    r = op.encode(s, wl.shape, weights, toks)
    t1 = time.perf_counter()
    out = op.decode(s, wl.shape, weights, r.data, len(toks))
    t2 = time.perf_counter()
    assert np.array_equal(out, toks), "oracle round trip failed"
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return r, {"value": round(len(toks) / (t2 - t0), 3), "unit": "tokens/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(toks)} tokens of stream 0, encode ({t1 - t0:.1f} s) + "
                         f"decode ({t2 - t1:.1f} s), FP64 numpy with {threads} BLAS threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="full_fp32")
    ap.add_argument("--kernel", default="attn", help="kernel class for the roofline")
    ap.add_argument("--max-len", type=int, default=None, help="truncate streams (quick runs)")
    ap.add_argument("--n-streams", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=1500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain streaming kernel of this size first (counter scaling)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="offline: turn two rocprofv3 --pmc counter files into the traffic figure")
    ap.add_argument("--traffic-command", default="", help="the counter runs' command, recorded")
    ap.add_argument("--ablation", action="store_true",
                    help="run the A0-A4 feature ladder on the workload instead of the timing")
    ap.add_argument("--oracle-prefix", type=int, default=200)
    ap.add_argument("--profile-stride", type=int, default=8,
                    help="time every n-th launch of the roofline class with HIP events")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the fixed GEMM launch-shape rule (no tuning before the warmup)")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from(*args.traffic_from, args.kernel, args.workload,
                                      args.copy_probe_mib, args.traffic_command)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (streams are "
              "independent and would be sharded by stream, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2602_19626_amd as nc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    wl = synth.WORKLOADS[args.workload]
    streams = synth.workload_streams(wl, max_len=args.max_len, n_streams=args.n_streams)
    n_tok = int(sum(len(s) for s in streams))
    weights = synth.make_weights(wl.shape, wl.weight_seed)
    cfg = nc.make_config(wl.shape, ngram_order=wl.ngram_order, precision=wl.precision,
                         skip=wl.skip, mix_init=wl.mix_init, warmup=wl.warmup,
                         head_lr=wl.head_lr, cdf_total=wl.cdf_total, ensemble=wl.ensemble,
                         max_streams=len(streams))
    if args.ablation:
        print(json.dumps({"workload": args.workload, "streams": len(streams), "tokens": n_tok,
                          "ablation": ablation(nc, wl, weights, streams, args.oracle_prefix)}),
              flush=True)
        return
    ctx = nc.Context(cfg, synth.flat_weights(wl.shape, weights))
    if wl.precision == "fp8":
        ctx.calibrate_fp8(synth.make_stream(2048, wl.shape.vocab, synth.CALIBRATION_SEED,
                                            span=wl.span))

    tune = None
    if not args.no_autotune:
        # launch shapes per (GEMM, row bucket) up to the largest pass: every stream's slide-long
        # segment at once; timed outside the measured steps
        t0 = time.perf_counter()
        table = ctx.autotune(max_rows=len(streams) * wl.shape.slide, reps=5)
        tune = {"seconds": round(time.perf_counter() - t0, 3), "entries": len(table),
                "changed": sum(e["kind"] != "rule" for e in table),
                "est_saving_us": round(sum(e["us_default"] - e["us_best"] for e in table), 1)}

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        data, bits = ctx.encode_stream(streams)
        te = time.perf_counter()
        st_enc = ctx.stats()
        out = ctx.decode_stream(data, [len(s) for s in streams])
        td = time.perf_counter()
        torch.cuda.synchronize()
        st_dec = ctx.stats()
        return data, bits, out, te - t0, td - te, st_enc, st_dec

    for _ in range(args.warmup):
        step()
    ctx.profile(args.kernel, args.profile_stride)
    t_enc = t_dec = w_enc = w_dec = 0.0
    ok = True
    for _ in range(args.steps):
        data, bits, out, te, td, st_enc, st_dec = step()
        t_enc += te
        t_dec += td
        w_enc += st_enc["wait_seconds"]
        w_dec += st_dec["wait_seconds"]
        ok = ok and all(np.array_equal(a, b) for a, b in zip(out, streams))
    prof = ctx.profile_read()
    ctx.profile(None)
    total_bits = float(sum(bits))

    # roofline of the profiled kernel class
    avg_ms = prof["ms"] / max(prof["timed"], 1)
    gemm_classes = ("qkv", "oproj", "gateup", "down", "lmhead")
    bound = "hbm"
    achieved = prof["bytes"] / max(prof["ms"], 1e-9) / 1e6           # GB/s
    peak, unit = HBM_PEAK_GBS, "GB/s"
    ai = prof["flops"] / max(prof["bytes"], 1.0)
    ridge = MFMA_PEAK_TFLOPS[wl.precision] * 1e12 / (HBM_PEAK_GBS * 1e9)
    if args.kernel in gemm_classes + ("attn",) and ai > ridge:
        bound = "mfma"
        achieved = prof["flops"] / max(prof["ms"], 1e-9) / 1e9        # TFLOP/s
        peak, unit = MFMA_PEAK_TFLOPS[wl.precision], "TFLOP/s"
    traffic = load_traffic(args.kernel, args.workload)
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": args.kernel, "launches": prof["launches"],
                "timed_launches": prof["timed"], "avg_launch_us": round(avg_ms * 1000, 3),
                "algorithmic_bytes_per_launch": round(prof["bytes"] / max(prof["timed"], 1)),
                "algorithmic_flops_per_launch": round(prof["flops"] / max(prof["timed"], 1))}

    line = {"metric": METRIC,
            "value": round(args.steps * n_tok / (t_enc + t_dec), 2),
            "unit": "tokens/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(1000 * (t_enc + t_dec) / args.steps, 2),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[wl.precision],
            "data": "synthetic: seeded Zipf(1.1) token streams with 30% copied spans, "
                    "random-init N(0, 0.02) weights of the 135M shape",
            "config": {"workload": args.workload, "streams": len(streams), "tokens": n_tok,
                       "precision": wl.precision, "ngram_order": wl.ngram_order,
                       "skip": wl.skip, "ensemble": wl.ensemble},
            "encode_tok_s": round(args.steps * n_tok / t_enc, 2),
            "decode_tok_s": round(args.steps * n_tok / t_dec, 2),
            "bits_per_token": round(total_bits / n_tok, 5),
            "skip_rate": None, "roundtrip_exact": bool(ok),
            "host_wait_frac": {"encode": round(w_enc / t_enc, 3), "decode": round(w_dec / t_dec, 3)},
            "roofline": roofline, "autotune": tune}
    line["cdf24_standalone"] = cdf24_standalone(nc, torch, wl.shape.vocab)
    dstat = ctx.stats()
    line["skip_rate"] = round(dstat["skipped"] / max(dstat["tokens"], 1), 4)
    line["gpu_ideal_bits_per_token"] = round(st_enc["ideal_bits"] / n_tok, 5)

    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample, len(streams[0]))
        ref, cb = cpu_baseline(wl, weights, streams[0], n_s)
        line["cpu_baseline"] = cb
        # gap of the GPU coder against the oracle's ideal code length, same prefix
        d, b = ctx.encode_stream([streams[0][:n_s]])
        # against the oracle's ideal code length sum -log2 p (FP64, before quantisation); it can
        # be negative: the one-count floor caps a near-zero probability's cost at log2 T bits
        line["gap_bits_per_token_sample"] = round((b[0] - ref.ideal_bits) / n_s, 5)
        line["gap_bpb_at_4_bytes_per_token"] = round(line["gap_bits_per_token_sample"] / 4.0, 5)
        # against the oracle's own coder on its quantised CDFs, and its quantised ideal length
        line["coded_bits_sample"] = {"gpu": int(b[0]), "oracle": int(ref.n_bits),
                                     "oracle_quantised_ideal": round(ref.quant_bits, 3)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
