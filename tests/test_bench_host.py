"""Host-side logic of bench.py (no GPU): the algorithmic flop count it
prices the roofline with, the staleness check of the recorded HBM
counters, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2308_12698_amd import inputs as I  # noqa: E402


def test_flop_count_is_the_reference_operation_count(oracle):
    sw = I.config2(n=8, n_steps=10)
    ops = oracle.count_ops(sw.types[0], sw.glob, 1, sw.dt)
    assert ops["flops"] == bench.FLOPS_PER_AGENT_STEP
    assert (ops["add"], ops["mul"], ops["div"], ops["sqrt"]) == (390, 506, 58, 8)


def test_source_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // add one\n}\n/* block\n comment */\n")
    b.write_text("int f(int x)\n{\n\treturn x + 1;\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a)])
    h1 = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(b)])
    assert bench.kernel_source_hash() == h1
    b.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h1


def test_traffic_is_reported_only_for_the_current_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fused") is None                    # no file
    f.write_text(json.dumps({"fused": {"source_hash": "0" * 16, "bytes_per_launch": 123}}))
    assert bench.measured_traffic("fused") is None                    # stale counters
    f.write_text(json.dumps({"fused": {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 123}}))
    assert bench.measured_traffic("fused") == 123
    assert bench.measured_traffic("plain") is None                    # not recorded


@pytest.mark.timeout(120)
def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=100)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_host_cpu_is_described():
    text = bench.host_cpu()
    assert "logical CPUs" in text and text.split(",")[0].strip()


def test_alu_roofline_prices_the_flop_count():
    r = bench.alu_roofline(1e11)
    assert r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP32_TFLOPS
    assert abs(r["achieved"] - 96.2) < 1e-9 and abs(r["frac"] - round(96.2 / 157.3, 4)) < 1e-12
