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
KERNEL_PRIMARY_RE = {"attn": r"attention_(quad|chunk|seq)_kernel", "vocab": r"vocab_lse_kernel",
                     "ngram": r"ngram_dense_kernel"}
PROBE_RE = r"neg"   # the plain streaming probe kernel (torch.neg: reads N bytes, writes N bytes)


def log(msg: str):
    """Progress on stderr (the JSON line on stdout stays the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def stats_summary(stats_csv: str, title: str, command: str, top: int = 24) -> str:
    """Markdown table of the top kernels of a rocprofv3 --stats kernel_stats.csv."""
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    calls = sum(int(r["Calls"]) for r in rows)
    out = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```",
           command, "```", "", "| kernel | calls | total ms | avg us | % |",
           "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = r["Name"].replace("|", "/")
        name = name if len(name) <= 90 else name[:87] + "..."
        out.append(f"| `{name}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / tot:.2f} |")
    out += ["", f"Total kernel time {tot / 1e6:.1f} ms over {calls} launches", ""]
    return "\n".join(out)


def pmc_summary(paths, title: str, command: str, probe_mib: int = 0, simds: int = 1024,
                top: int = 30) -> str:
    """Per-kernel sums of rocprofv3 --pmc counter files: dispatches, counter totals, and the
    derived figures when their counters are present (MFMA busy share of the SIMD cycles; HBM
    bytes per dispatch from FETCH_SIZE / WRITE_SIZE, each scaled by the same counter's reading
    for the streaming probe of probe_mib MiB)."""
    per = {}
    for path in paths:
        for row in csv.DictReader(open(path)):
            k = per.setdefault(row["Kernel_Name"], {"ids": set()})
            k["ids"].add(row.get("Dispatch_Id", row.get("Correlation_Id", "")))
            c = row["Counter_Name"]
            k[c] = k.get(c, 0.0) + float(row["Counter_Value"])
            k["n_" + c] = k.get("n_" + c, 0) + 1
    scale = {}
    if probe_mib:
        for name, k in per.items():
            if re.search(PROBE_RE, name):
                for c in ("FETCH_SIZE", "WRITE_SIZE"):
                    if c in k:
                        scale[c] = probe_mib * 1024.0 / k[c]
    out = [f"# {title}", "", "Commands (from the repository root, on one MI355X):", "", "```",
           command, "```", ""]
    counters = sorted({c for k in per.values() for c in k if c != "ids" and not c.startswith("n_")})
    out.append("Counters: " + ", ".join(counters) + (f"; FETCH/WRITE scale from the probe: "
               + ", ".join(f"{c} x{v:.4f}" for c, v in scale.items()) if scale else ""))
    out.append("")
    hdr = "| kernel | dispatches |"
    if "SQ_VALU_MFMA_BUSY_CYCLES" in counters and "GRBM_GUI_ACTIVE" in counters:
        hdr += " MFMA busy % |"
    if "MfmaUtil" in counters:
        hdr += " MfmaUtil % (mean) |"
    if "FETCH_SIZE" in counters:
        hdr += " fetch KB / dispatch |"
    if "WRITE_SIZE" in counters:
        hdr += " write KB / dispatch |"
    out += [hdr, "|---|---:|" + "---:|" * (hdr.count("|") - 3)]
    key = next((c for c in ("GRBM_GUI_ACTIVE", "FETCH_SIZE") if c in counters), counters[0])
    for name, k in sorted(per.items(), key=lambda kv: -kv[1].get(key, 0.0))[:top]:
        n = max(len(k["ids"]), 1)
        nm = name if len(name) <= 80 else name[:77] + "..."
        line = f"| `{nm}` | {n} |"
        if "SQ_VALU_MFMA_BUSY_CYCLES" in counters and "GRBM_GUI_ACTIVE" in counters:
            line += f" {100 * k.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) / max(k['GRBM_GUI_ACTIVE'] * simds, 1):.1f} |"
        if "MfmaUtil" in counters:
            line += f" {k.get('MfmaUtil', 0) / max(k.get('n_MfmaUtil', 1), 1):.1f} |"
        if "FETCH_SIZE" in counters:
            line += f" {k.get('FETCH_SIZE', 0) * scale.get('FETCH_SIZE', 1.0) / n:.1f} |"
        if "WRITE_SIZE" in counters:
            line += f" {k.get('WRITE_SIZE', 0) * scale.get('WRITE_SIZE', 1.0) / n:.1f} |"
        out.append(line)
    return "\n".join(out) + "\n"


def cdf24_standalone(nc, torch, vocab: int, rows_list=(64, 1024, 4096), reps: int = 20):
    """nc_quantize_cdf24 alone on float32 rows of softmax-shaped probabilities (up to 64 rows the
    segment reduce + scan kernels, more rows the one-workgroup-per-row kernel); algorithmic bytes
    per row = read 4V + write 4(V + 1).  From 1,024 rows at V = 49,152 the rows and their CDFs
    (402 MB and more) exceed the 256 MB Infinity Cache.  Beside it: a plain device-to-device copy
    of the same rows (read 4V + write 4V), the streaming rate this part reaches in practice."""
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
        # the practical streaming ceiling for the same bytes: a device-to-device copy of the rows
        q = torch.empty_like(p)
        q.copy_(p)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            q.copy_(p)
        e1.record()
        torch.cuda.synchronize()
        us_copy = e0.elapsed_time(e1) * 1000.0 / reps
        gbs_copy = rows * 8 * vocab / (us_copy * 1e-6) / 1e9
        out.append({"rows": rows, "vocab": vocab, "us_per_call": round(us, 2),
                    "achieved_GBps": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                    "copy_same_bytes_GBps": round(gbs_copy, 1),
                    "frac_of_copy": round(gbs / gbs_copy, 4)})
        del q
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


def cpu_baseline(wl, weights, stream, n_sample: int, n_single: int):
    """The oracle (FP64 numpy + exact integer quantiser + Python-integer coder) on a prefix, with
    every BLAS thread, and again on a shorter prefix with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import pipeline as op
    s = op.Settings.from_workload(wl)

    def run(toks):
        t0 = time.perf_counter()
        r = op.encode(s, wl.shape, weights, toks)
        t1 = time.perf_counter()
        out = op.decode(s, wl.shape, weights, r.data, len(toks))
        t2 = time.perf_counter()
        assert np.array_equal(out, toks), "oracle round trip failed"
        return r, t1 - t0, t2 - t1

    toks = stream[:n_sample]
    r, te, td = run(toks)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    out = {"value": round(len(toks) / (te + td), 3), "unit": "tokens/s", "cores": threads,
           "kind": "oracle",
           "sample": f"first {len(toks)} tokens of stream 0 (the KV cache slides at token 2,048), "
                     f"encode ({te:.1f} s) + decode ({td:.1f} s), FP64 numpy with {threads} "
                     "BLAS threads"}
    if n_single:
        with threadpool_limits(limits=1):
            t1 = stream[:n_single]
            _, te1, td1 = run(t1)
        out["single_thread"] = {"value": round(len(t1) / (te1 + td1), 3), "unit": "tokens/s",
                                "cores": 1, "sample": f"first {len(t1)} tokens, encode "
                                f"({te1:.1f} s) + decode ({td1:.1f} s), one BLAS thread"}
    return r, out


def class_rooflines(prof: dict, precision: str) -> dict:
    """Per kernel class: average launch time and the achieved fraction of its roofline (HBM for
    byte-bound classes, MFMA for classes whose arithmetic intensity is above the ridge)."""
    ridge = MFMA_PEAK_TFLOPS[precision] * 1e12 / (HBM_PEAK_GBS * 1e9)
    out = {}
    for cls, k in prof.items():
        if not k["timed"]:
            continue
        ai = k["flops"] / max(k["bytes"], 1.0)
        mfma = cls in ("qkv", "oproj", "gateup", "down", "lmhead", "attn") and ai > ridge
        if mfma:
            ach, peak, unit = k["flops"] / k["ms"] / 1e9, MFMA_PEAK_TFLOPS[precision], "TFLOP/s"
        else:
            ach, peak, unit = k["bytes"] / k["ms"] / 1e6, HBM_PEAK_GBS, "GB/s"
        out[cls] = {"bound": "mfma" if mfma else "hbm", "achieved": round(ach, 2), "peak": peak,
                    "unit": unit, "frac": round(ach / peak, 4),
                    "avg_launch_us": round(1000 * k["ms"] / k["timed"], 3),
                    "launches": k["launches"], "timed_launches": k["timed"],
                    "est_total_ms": round(k["ms"] * k["launches"] / k["timed"], 1),
                    "algorithmic_bytes_per_launch": round(k["bytes"] / k["timed"]),
                    "algorithmic_flops_per_launch": round(k["flops"] / k["timed"])}
    return out


def batched_line(nc, synth, max_len: int, steps: int = 1):
    """The 64-stream BF16 workload (p_max skip) with every stream cut to max_len tokens:
    encode + decode tokens/s, round trip checked."""
    wl = synth.WORKLOADS["batch64_bf16"]
    streams = synth.workload_streams(wl, max_len=max_len)
    n_tok = int(sum(len(s) for s in streams))
    w = synth.make_weights(wl.shape, wl.weight_seed)
    cfg = nc.make_config(wl.shape, ngram_order=wl.ngram_order, precision=wl.precision,
                         skip=wl.skip, mix_init=wl.mix_init, warmup=wl.warmup, head_lr=wl.head_lr,
                         cdf_total=wl.cdf_total, max_streams=len(streams))
    ctx = nc.Context(cfg, synth.flat_weights(wl.shape, w))
    ctx.autotune(max_rows=len(streams) * wl.shape.slide, reps=5)
    data, _ = ctx.encode_stream(streams)              # warm-up
    ctx.decode_stream(data, [len(s) for s in streams])
    te = td = 0.0
    ok = True
    for _ in range(steps):
        t0 = time.perf_counter()
        data, bits = ctx.encode_stream(streams)
        t1 = time.perf_counter()
        out = ctx.decode_stream(data, [len(s) for s in streams])
        t2 = time.perf_counter()
        te += t1 - t0
        td += t2 - t1
        ok = ok and all(np.array_equal(a, b) for a, b in zip(out, streams))
    st = ctx.stats()
    ctx.close()
    return {"workload": f"batch64_bf16, every stream cut to {max_len} tokens",
            "streams": len(streams), "tokens": n_tok,
            "value": round(steps * n_tok / (te + td), 1),
            "encode_tok_s": round(steps * n_tok / te, 1),
            "decode_tok_s": round(steps * n_tok / td, 1),
            "bits_per_token": round(float(sum(bits)) / n_tok, 5),
            "skip_rate": round(st["skipped"] / max(st["tokens"], 1), 4),
            "roundtrip_exact": bool(ok)}


def precision_lines(nc, synth, wl, weights, stream, n: int, ref=None):
    """The precision forms on the plain configuration's stream prefix (the KV cache slides at
    token 2,048): max |logit error| and mean KL(p_llm) against the FP64 oracle at sampled
    positions (skip off, so the model runs there), and the coded length against the oracle
    coder's on the same prefix (method as specified).  Tolerances: the error model of
    tests/golden/precision_tolerances.json."""
    import dataclasses
    from oracle.transformer import Transformer
    toks = stream[:n]
    pos = [p for p in (0, 100, 500, 1000, 1500, 2046, 2047, 2048, 2049, 2100, n - 1) if p < n]
    model = Transformer(wl.shape, weights, max_block=512)
    x = np.concatenate([[0], toks[:-1]])
    z_ref = model.logits(model.append(x)[pos])
    tol = json.load(open(os.path.join(ROOT, "tests", "golden", "precision_tolerances.json")))
    calib = synth.make_stream(2048, wl.shape.vocab, synth.CALIBRATION_SEED, span=wl.span)
    out = {}
    for prec in ("fp32", "bf16", "fp8"):
        row = {}
        for skip in ("none", wl.skip):
            w2 = dataclasses.replace(wl, precision=prec, skip=skip)
            cfg = nc.make_config(w2.shape, ngram_order=w2.ngram_order, precision=prec, skip=skip,
                                 mix_init=w2.mix_init, warmup=w2.warmup, head_lr=w2.head_lr,
                                 cdf_total=w2.cdf_total, max_streams=1)
            ctx = nc.Context(cfg, synth.flat_weights(w2.shape, weights))
            if prec == "fp8":
                ctx.calibrate_fp8(calib)
            if skip == "none":
                ctx.reset(1, n + 1)
                errs, kls = [], []
                for k, i in enumerate(pos):
                    _, pr = ctx.probs_for_context(0, toks[:i], probe=True)
                    z = pr["logits"].astype(np.float64)
                    errs.append(float(np.max(np.abs(z - z_ref[k]))))
                    zr = z_ref[k] - z_ref[k].max()
                    pref = np.exp(zr) / np.exp(zr).sum()
                    q = np.exp(z - z.max())
                    q /= q.sum()
                    kls.append(float(np.sum(pref * (np.log2(pref) - np.log2(q)))))
                row.update(max_abs_logit_err=round(max(errs), 6), mean_kl_llm_bits=float(
                    f"{np.mean(kls):.4g}"), positions=pos)
                if prec != "fp32":
                    row["tolerance"] = {"max_abs_logit": round(tol[prec]["max_abs_logit"], 4),
                                        "mean_kl_bits": float(f"{tol[prec]['mean_kl_bits']:.4g}")}
            else:
                _, bits = ctx.encode_stream([toks])
                row["coded_bits"] = int(bits[0])
                if ref is not None:
                    row["oracle_coded_bits"] = int(ref.n_bits)
                    row["gap_vs_oracle_coder_bits_per_token"] = round(
                        (bits[0] - ref.n_bits) / n, 5)
                    row["gap_vs_oracle_ideal_bits_per_token"] = round(
                        (bits[0] - ref.ideal_bits) / n, 5)
                    row["gap_vs_oracle_ideal_bpb_at_4_bytes_per_token"] = round(
                        (bits[0] - ref.ideal_bits) / n / 4.0, 5)
            ctx.close()
        out[prec] = row
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="full_fp32")
    ap.add_argument("--kernel", default="auto",
                    help="kernel class for the roofline (auto: the class with the most time)")
    ap.add_argument("--max-len", type=int, default=None, help="truncate streams (quick runs)")
    ap.add_argument("--n-streams", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=2200,
                    help="oracle prefix (all BLAS threads); the default crosses the KV slide")
    ap.add_argument("--cpu-single-sample", type=int, default=256,
                    help="oracle prefix timed with one BLAS thread (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16 / FP8 lines (logit error, KL, coded length vs oracle)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain streaming kernel of this size first (counter scaling)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="offline: turn two rocprofv3 --pmc counter files into the traffic figure")
    ap.add_argument("--traffic-command", default="", help="the counter runs' command, recorded")
    ap.add_argument("--stats-summary", nargs=3, metavar=("STATS_CSV", "TITLE", "OUT_MD"),
                    help="offline: markdown summary of a rocprofv3 --stats kernel_stats.csv")
    ap.add_argument("--pmc-summary", nargs="+", metavar="ARG",
                    help="offline: TITLE OUT_MD CSV [CSV ...]: per-kernel counter summary")
    ap.add_argument("--summary-command", default="", help="the profiled command, recorded")
    ap.add_argument("--ablation", action="store_true",
                    help="run the A0-A4 feature ladder on the workload instead of the timing")
    ap.add_argument("--oracle-prefix", type=int, default=200)
    ap.add_argument("--profile-stride", type=int, default=4,
                    help="in the profiled step after the timed ones, time every n-th launch of "
                         "each kernel class with HIP events")
    ap.add_argument("--batch-len", type=int, default=2048,
                    help="also run the 64-stream BF16 workload cut to this many tokens per "
                         "stream (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the fixed GEMM launch-shape rule (no tuning before the warmup)")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from(*args.traffic_from, args.kernel, args.workload,
                                      args.copy_probe_mib, args.traffic_command)))
        return
    if args.stats_summary:
        csv_path, title, out_md = args.stats_summary
        open(out_md, "w").write(stats_summary(csv_path, title, args.summary_command))
        return
    if args.pmc_summary:
        title, out_md, *paths = args.pmc_summary
        open(out_md, "w").write(pmc_summary(paths, title, args.summary_command,
                                            args.copy_probe_mib))
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
        log("launch shapes tuned")
        tune = {"seconds": round(time.perf_counter() - t0, 3), "entries": len(table),
                "changed": sum(e["kind"] != "rule" for e in table),
                "est_saving_us": round(sum(e["us_default"] - e["us_best"] for e in table), 1)}

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        data, bits = ctx.encode_stream(streams)
        te = time.perf_counter()
        log(f"  encode {te - t0:.2f} s")
        st_enc = ctx.stats()
        out = ctx.decode_stream(data, [len(s) for s in streams])
        td = time.perf_counter()
        log(f"  decode {td - te:.2f} s")
        torch.cuda.synchronize()
        st_dec = ctx.stats()
        return data, bits, out, te - t0, td - te, st_enc, st_dec

    for k in range(args.warmup):
        step()
        log(f"warmup step {k + 1}/{args.warmup} done")
    t_enc = t_dec = w_enc = w_dec = 0.0
    ok = True
    for k in range(args.steps):
        data, bits, out, te, td, st_enc, st_dec = step()
        log(f"timed step {k + 1}/{args.steps}: encode {te:.2f} s, decode {td:.2f} s")
        t_enc += te
        t_dec += td
        w_enc += st_enc["wait_seconds"]
        w_dec += st_dec["wait_seconds"]
        ok = ok and all(np.array_equal(a, b) for a, b in zip(out, streams))
    total_bits = float(sum(bits))
    ideal_enc = st_enc["ideal_bits"]
    skip_rate = st_dec["skipped"] / max(st_dec["tokens"], 1)

    # one more step, untimed, with every kernel class bracketed by HIP events on its stream
    ctx.profile("all", args.profile_stride)
    step()
    from paper_2602_19626_amd._lib import KERNEL_CLASSES
    prof = {k: ctx.profile_read(k) for k in KERNEL_CLASSES}
    ctx.profile(None)
    log("profiled step done")
    classes = class_rooflines(prof, wl.precision)
    kern = args.kernel if args.kernel != "auto" else \
        max(classes, key=lambda k: classes[k]["est_total_ms"])
    roofline = dict(classes[kern])
    roofline["kernel"] = kern
    roofline["traffic"] = load_traffic(kern, args.workload)
    roofline = {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                         "kernel", "avg_launch_us", "launches", "timed_launches",
                                         "algorithmic_bytes_per_launch",
                                         "algorithmic_flops_per_launch")}

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
            "skip_rate": round(skip_rate, 4), "roundtrip_exact": bool(ok),
            "host_wait_frac": {"encode": round(w_enc / t_enc, 3), "decode": round(w_dec / t_dec, 3)},
            "roofline": roofline, "kernel_classes": classes, "autotune": tune}
    line["cdf24_standalone"] = cdf24_standalone(nc, torch, wl.shape.vocab)
    log("CDF-24 standalone timed")
    line["gpu_ideal_bits_per_token"] = round(ideal_enc / n_tok, 5)
    if args.batch_len and args.workload == "full_fp32":
        b = batched_line(nc, synth, args.batch_len)
        log("64-stream BF16 line done")
        b["vs_this_line_value"] = round(b["value"] / line["value"], 2)
        line["batch64_bf16"] = b

    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample, len(streams[0]))
        log(f"oracle baseline on {n_s} tokens (all threads) and "
            f"{min(args.cpu_single_sample, len(streams[0]))} tokens (one thread) ...")
        ref, cb = cpu_baseline(wl, weights, streams[0], n_s,
                               min(args.cpu_single_sample, len(streams[0])))
        log("oracle baseline done")
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
        if args.workload == "full_fp32" and not args.no_precision:
            log("precision forms against the oracle ...")
            line["precision_forms"] = precision_lines(nc, synth, wl, weights, streams[0], n_s, ref)
            log("precision forms done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
