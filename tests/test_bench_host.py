"""Host-side logic of bench.py (no GPU): the one-GPU guard and the counter
summary (copy-probe scaling, early-exit dispatches left out)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": kib})


def test_counter_summary_scaling_and_early_exits(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h")
    mib = 64
    # FETCH_SIZE reads half of a copy's bytes, WRITE_SIZE all of them
    fetch = [("void knng::k_join_split<3, 1>(knng::Views)", 4096, 1000.0),
             ("void knng::k_join_split<3, 1>(knng::Views)", 4096, 3000.0),
             ("void knng::k_join_split<3, 1>(knng::Views)", 4096, 1.0),        # early exit
             ("__amd_rocclr_copyBuffer", mib << 8, mib * 1024 / 2.0)]
    write = [("void knng::k_join_split<3, 1>(knng::Views)", 4096, 10.0),
             ("void knng::k_join_split<3, 1>(knng::Views)", 4096, 30.0),
             ("void knng::k_join_split<3, 1>(knng::Views)", 4096, 0.0),
             ("__amd_rocclr_copyBuffer", mib << 8, mib * 1024.0)]
    _write(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), mib, "cmd", "blobs4m_d3")
    out = json.load(open(tmp_path / "profiles" / "traffic_blobs4m_d3.json"))
    j = out["k_join_split"]
    assert out["_scale"]["fetch"] == pytest.approx(2.0) and out["_scale"]["write"] == pytest.approx(1.0)
    assert j["launches"] == 2 and j["early_exits"] == 1
    assert j["fetch_bytes_per_launch"] == int(2000.0 * 1024 * 2.0)
    assert j["write_bytes_per_launch"] == int(20.0 * 1024)
    assert j["source_hash"] == "h"
    assert bench.traffic_record("k_join_split", "blobs4m_d3") == j["bytes_per_launch"]
    assert bench.traffic_record("k_join_split", "image60k_d784") is None   # no headline summary here


def test_traffic_file_names():
    assert bench.traffic_path("image60k_d784").endswith(os.path.join("profiles", "traffic.json"))
    assert bench.traffic_path("blobs4m_d3").endswith(os.path.join("profiles", "traffic_blobs4m_d3.json"))


def test_join_roofline_byte_model():
    """Algorithmic join bytes: FP32 rows (4 d_pad) + 8 B sample entry per
    member gathered, 8 B per proposal; the encoding figure prices the rows the
    kernel reads (2 d_pad per split plane) plus 20 B of member metadata."""
    class K:
        PATH_VALU, PATH_MFMA, PATH_MFMA_BF16X3 = 1, 2, 4
    w = {"d": 784, "workload": "none"}
    s0 = {"path": 4, "dpad": 800, "planes": 1, "iters": 2, "proposals": [100, 50], "evals": [1000, 500]}
    stats = [{"join_ms": [0.001, 0.001]}]
    members = [10_000, 20_000]
    r = bench.join_roofline(K, w, s0, stats, members, "fp32")
    alg = 10_000 * (3200 + 8) + 800 + 20_000 * (3200 + 8) + 400
    assert r["kernel"] == "k_join_split"
    assert r["bytes_per_launch"] == alg // 2
    assert r["achieved"] == round(alg / 2e-6 / 1e9, 1)
    assert r["frac"] == round(r["achieved"] / 8000.0, 4)
    enc = 10_000 * (1600 + 20) + 800 + 20_000 * (1600 + 20) + 400
    assert r["encoding"]["bytes_per_launch"] == enc // 2 and r["encoding"]["row_bytes"] == 1600
    assert r["frac"] > 1 and "encoding" in r["note"]
    assert r["mfma"]["flops_per_launch"] == (1000 + 500) * 2 * 784 // 2
    s0["path"] = 1
    s0["dpad"] = 4
    r = bench.join_roofline(K, {"d": 3, "workload": "none"}, s0, stats, members, "fp32")
    assert r["kernel"] == "k_join_valu" and r["encoding"]["row_bytes"] == 16 and "note" not in r
