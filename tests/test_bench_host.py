"""bench.py's host-side contract without a GPU: more than one GPU is refused
with a message, and the stored HBM traffic of a kernel is reported only while
the kernel's source is the one the counters were taken on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stored_traffic_follows_the_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_1808_01829_amd" / "csrc"
    src.mkdir(parents=True)
    kernel = src / "update_mfma.hip"
    kernel.write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    sha = hashlib.sha256(kernel.read_bytes()).hexdigest()
    doc = {"kernels": {"update": {"source": "paper_1808_01829_amd/csrc/update_mfma.hip",
                                  "source_sha256": sha, "bytes_per_launch": 12345}}}
    (tmp_path / "profiles" / "traffic_c5_mixed.json").write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("c5", "mixed", "update") == 12345
    assert bench.stored_traffic("c5", "f64", "update") is None      # no summary for it
    assert bench.stored_traffic("c5", "mixed", "hop") is None       # no entry for it
    kernel.write_text("// kernel v2\n")                               # source changed
    assert bench.stored_traffic("c5", "mixed", "update") is None


def test_cpu_baseline_leg_on_a_small_workload():
    """The cpu_baseline leg (the oracle's multi-shift CG timed on the host and
    scaled to a per-vector solve) at 8^4 with a short budget: the contract's
    fields and the thread count it reports."""
    import re

    from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge
    w = dict(configs.WORKLOADS["c2"])
    r = configs.workload_coefficients("c2")
    U = random_gauge(w["dims"], w["eps"], 2000)
    B = gaussian_block(w["dims"], w["n"], 2001)
    try:
        out = bench.cpu_oracle_sample(U, B, w, r, 500, 0.2, threads=2)
    finally:
        bench.set_omp_threads(os.cpu_count() or 1)
    assert out["kind"] == "oracle" and out["unit"] == "RHS-solves/s" and out["cores"] == 2
    assert out["value"] > 0
    assert re.search(r"[0-9.]+ s/iteration", out["sample"])
    assert "scaled to the 500 iterations" in out["sample"]


def test_hop_traversal_table(tmp_path):
    """--write-hop-traversal: each row's fetch is the median FETCH_SIZE of its
    timed launches (the untimed first one skipped) scaled by the copy
    calibration, shown in MB and in block vectors beyond the links; a counter
    run with another number of hop dispatches is refused."""
    import csv as _csv
    dims, n, reps = [4, 4, 4, 4], 16, 3
    rows = [dict(prec="f64", variant=-1, cfg=[0, 0, 0, 2, 1], par=1),
            dict(prec="f32", variant=4, cfg=[8, 8, 8, 4, 1], par=0)]
    run = dict(lattice=dims, n=n, link_rows=2, reps=reps, rows=rows)
    tim = dict(run, rows=[dict(r, us=10.0) for r in rows])
    (tmp_path / "pmc.json").write_text("log line\n" + json.dumps(run) + "\n")
    (tmp_path / "time.json").write_text(json.dumps(tim) + "\n")
    vh = 4 ** 4 // 2

    def sizes(b):
        return vh * 3 * n * 2 * b, vh * 8 * 6 * 2 * b   # S, G

    def write_csv(path, vals):
        with open(path, "w", newline="") as f:
            w = _csv.writer(f)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for i, (k, v) in enumerate(vals):
                w.writerow([i, k, "FETCH_SIZE", v])
    # calibration: 1 GiB copy counted as 2^19 KiB (factor 2)
    write_csv(tmp_path / "cal.csv", [("fill", 1.0), ("copy", 524288.0)])
    S64, G64 = sizes(8)
    S32, G32 = sizes(4)
    # fetch = G + 2 S (FP64 row) and G + 3 S (FP32 row), in KiB before the factor 2
    f64_kib = (G64 + 2 * S64) / 2048.0
    f32_kib = (G32 + 3 * S32) / 2048.0
    vals = [("k_hop_q", 1e9), ("k_hop_q", f64_kib), ("k_hop_q", f64_kib * 1.5), ("k_hop_q", f64_kib),
            ("k_hop_s", 1e9), ("k_hop_s", f32_kib), ("k_hop_s", f32_kib), ("k_hop_s", 0.0)]
    write_csv(tmp_path / "fetch.csv", vals + [("k_other", 5.0)])
    out = bench.write_hop_traversal(str(tmp_path / "fetch.csv"), str(tmp_path / "pmc.json"),
                                    str(tmp_path / "time.json"), str(tmp_path / "cal.csv"),
                                    "cmd", str(tmp_path / "t.txt"))
    lines = [l for l in open(out) if l.startswith(("f64", "f32"))]
    assert len(lines) == 2
    f = lines[0].split()
    assert f[1] == "-1" and abs(float(f[-2]) - 2.0) < 1e-9
    assert abs(float(f[-3]) - (G64 + 2 * S64) / 1e6) < 0.05
    g = lines[1].split()
    assert g[1] == "4" and abs(float(g[-2]) - 3.0) < 1e-9
    write_csv(tmp_path / "fetch.csv", vals[:-1])
    import pytest
    with pytest.raises(SystemExit):
        bench.write_hop_traversal(str(tmp_path / "fetch.csv"), str(tmp_path / "pmc.json"),
                                  str(tmp_path / "time.json"), str(tmp_path / "cal.csv"),
                                  "cmd", str(tmp_path / "t.txt"))
