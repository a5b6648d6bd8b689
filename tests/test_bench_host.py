"""bench.py on the CPU: the one-GPU refusal, the HBM arithmetic of the bench
line, and the code hash that keys the committed counter summary."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_step_hbm_arithmetic():
    copy = {"GB_per_s": 5000.0}
    out = bench._step_hbm({"ms_per_step": 10.0}, 64, 1000, copy)
    # 4 N_r P bytes per update: f read and written by the sweep, then by stage 2
    assert out["algorithmic_bytes_per_step"] == 32 * 1000
    assert out["achieved"] == pytest.approx(32 * 1000 / 1e-2 / 1e9)
    assert out["frac"] == pytest.approx(out["achieved"] / 8000.0)
    assert out["frac_of_copy"] == pytest.approx(out["achieved"] / 5000.0)
    assert bench._step_hbm({"ms_per_step": 10.0}, 32, 1000, copy)["algorithmic_bytes_per_step"] == 16 * 1000


def test_code_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// header\nint f(int x) {  /* a */ return x + 1; }\n")
    monkeypatch.setattr(bench, "SWEEP_SRC", str(src))
    h0 = bench._source_hash()
    src.write_text("// another header\n\nint f(int x) {\n  return x + 1;  // same code\n}\n")
    assert bench._source_hash() == h0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert bench._source_hash() != h0


def test_committed_counter_summary_matches_the_sweep_code():
    # the counters in profiles/ were taken on the sweep as it is now
    assert bench._traffic(64) is not None and bench._traffic(32) is not None
    assert bench._step_traffic(64) is not None
