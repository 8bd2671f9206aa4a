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
