"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the
device-code hash that ties profile summaries to the code they measured, and the
lookup of profiled HBM traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_source_hash_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2405_04253_amd" / "csrc"
    csrc.mkdir(parents=True)
    code = "int f(int x) {\n    return x + 1;\n}\n"
    (csrc / "fnt_device.hpp").write_text(code)
    (csrc / "fnt_kernels.hip").write_text(code)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    (csrc / "fnt_kernels.hip").write_text("// a comment\n/* a block\n comment */\n\nint f(int x) {  // trailing\n"
                                          "    return x + 1;\n}\n")
    assert bench.kernel_source_hash() == h0
    (csrc / "fnt_kernels.hip").write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_lookup_exact_scaled_and_stale(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    entry = {"source_hash": "h1", "aeq_blocks": 1000, "bytes_per_launch": 5.0e6}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"batched": {"k (lead)": entry}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    b, why = bench.load_traffic("k (lead)", "batched", 1000)
    assert b == 5.0e6 and "this launch" in why
    b, why = bench.load_traffic("k (lead)", "batched", 3000, per_block=True)
    assert b == pytest.approx(1.5e7) and "per block" in why
    assert bench.load_traffic("k (lead)", "batched", 3000)[0] is None
    assert bench.load_traffic("other", "batched", 1000)[0] is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h2")
    b, why = bench.load_traffic("k (lead)", "batched", 1000)
    assert b is None and "current kernel source" in why

