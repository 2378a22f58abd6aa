"""Host-side logic of bench.py: the counter-file reduction behind the roofline's traffic figure
and the one-GPU rule."""
import csv
import json
import os
import subprocess
import sys

import bench


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": kib})


def test_traffic_from_scales_by_probe(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_2602_19626_amd" / "csrc")
    (tmp_path / "paper_2602_19626_amd" / "csrc" / "k_llm.hip").write_text("// src")
    probe = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>"
    gu = "void nc::gemm_split_kernel<0, 0, 2, 1>(nc::GemmArgs)"
    qkv = "void nc::gemm_split_kernel<0, 0, 3, 1>(nc::GemmArgs)"
    # the probe reads 64 MiB; the counter reports 10% more, so every reading is scaled by 1/1.1
    _write(tmp_path / "f.csv", "FETCH_SIZE",
           [(probe, 65536 * 1.1), (gu, 1100.0), (gu, 3300.0), (qkv, 99999.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(probe, 65536 * 2.0), (gu, 200.0), (gu, 200.0)])
    t = bench.traffic_from(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "gateup",
                           "full_fp32", 64, "cmd")
    assert t["launches"] == 2
    assert t["fetch_bytes_per_launch"] == round(2200 * 1024 / 1.1)
    assert t["write_bytes_per_launch"] == round(200 * 1024 / 2.0)
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    stored = json.load(open(tmp_path / "profiles" / "traffic_gateup_full_fp32.json"))
    assert stored["source_sha"] == bench.kernel_source_hash("gateup")
    # the stored figure is used only while the kernel source is unchanged
    assert bench.load_traffic("gateup", "full_fp32") == t["bytes_per_launch"]
    (tmp_path / "paper_2602_19626_amd" / "csrc" / "k_llm.hip").write_text("// changed")
    assert bench.load_traffic("gateup", "full_fp32") is None


def test_traffic_from_counts_class_launches(tmp_path, monkeypatch):
    """A class launch of several kernels (attention: quad + fold) is one launch."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_2602_19626_amd" / "csrc")
    (tmp_path / "paper_2602_19626_amd" / "csrc" / "k_llm.hip").write_text("// src")
    probe = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>"
    quad, fold = "void nc::attention_quad_kernel<0>", "void nc::attention_fold_kernel<0>"
    seq = "void nc::attention_seq_kernel<0, 0>"
    rows_f = [(probe, 65536.0), (quad, 100.0), (fold, 10.0), (quad, 300.0), (fold, 30.0), (seq, 60.0)]
    rows_w = [(probe, 65536.0), (quad, 1.0), (fold, 2.0), (quad, 1.0), (fold, 2.0), (seq, 3.0)]
    _write(tmp_path / "f.csv", "FETCH_SIZE", rows_f)
    _write(tmp_path / "w.csv", "WRITE_SIZE", rows_w)
    t = bench.traffic_from(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "attn",
                           "full_fp32", 64, "cmd")
    assert t["launches"] == 3
    assert t["fetch_bytes_per_launch"] == round(500 * 1024 / 3)
    assert t["write_bytes_per_launch"] == round(9 * 1024 / 3)


def test_more_than_one_gpu_is_refused():
    """`--gpus N` with N > 1 exits with status 2 and a message, before any device work."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
