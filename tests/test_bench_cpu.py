"""Host-side pieces of bench.py: the one-GPU refusal, the per-image learning rate
(Eq. 6-7) it feeds the Adam step, and the traffic record lookup that the roofline
line uses (bytes only while the kernel's source is the one the counters saw)."""
import hashlib
import json
import math
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""   # no JSON line for a configuration that was not measured


def test_eq6_learning_rate_endpoints_and_log_linearity():
    eta0, etaf, ta = 1.6e-4, 1.6e-6, 30000.0
    assert bench.eq6_lr(0) == pytest.approx(eta0, rel=1e-12)
    assert bench.eq6_lr(ta) == pytest.approx(etaf, rel=1e-12)
    assert bench.eq6_lr(5 * ta) == pytest.approx(etaf, rel=1e-12)   # progress is capped at 1
    # log-linear: the midpoint is the geometric mean of the endpoints
    assert bench.eq6_lr(ta / 2) == pytest.approx(math.sqrt(eta0 * etaf), rel=1e-12)
    rates = [bench.eq6_lr(t) for t in range(0, 30001, 1000)]
    assert all(a > b for a, b in zip(rates, rates[1:]))


def test_traffic_record_matches_the_committed_source():
    for kernel in ("render_bwd", "render_fwd"):
        path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_c3.json")
        if not os.path.exists(path):
            pytest.skip("no traffic record")
        rec = json.load(open(path))
        src = os.path.join(ROOT, rec["source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        got = bench.traffic_for(kernel, "c3")
        if sha == rec["source_sha256"]:
            assert got == rec["bytes_per_launch"]
            # (each of the three is rounded to whole bytes on its own)
            assert abs(rec["bytes_per_launch"] - (rec["read_bytes"] + rec["written_bytes"])) <= 1
        else:
            assert got is None
    assert bench.traffic_for("no_such_kernel", "c3") is None


def test_traffic_is_dropped_once_the_source_changes(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "render_bwd_traffic_c3.json")))
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_2503_13086_amd" / "csrc"
    csrc.mkdir(parents=True)
    src_name = bench.KERNEL_SOURCE["render_bwd"]
    shutil.copy(os.path.join(ROOT, "paper_2503_13086_amd", "csrc", src_name), csrc / src_name)
    rec["source_sha256"] = hashlib.sha256((csrc / src_name).read_bytes()).hexdigest()
    (tmp_path / "profiles" / "render_bwd_traffic_c3.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("render_bwd", "c3") == rec["bytes_per_launch"]
    with open(csrc / src_name, "a") as f:
        f.write("\n// edited\n")
    assert bench.traffic_for("render_bwd", "c3") is None


def test_cpu_baseline_leg_reports_its_sample():
    # the oracle leg of the bench on the small 10k-Gaussian workload, with a short budget
    import scenegen
    cb = bench.cpu_baseline(scenegen.config1(), budget_s=0.3)
    assert cb["kind"] == "oracle" and cb["unit"] == "Mpix/s"
    assert cb["value"] > 0 and cb["cores"] >= 1
    assert "random pixels of view 0" in cb["sample"]
    full = cb["small_workload_full"]
    assert full["pixels"] == 128 * 128 and full["seconds"] > 0 and full["mpix_s"] > 0
