"""The bench.py output contract, on the CPU (the GPU run is in test_gpu_bench_line.py)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_schema_on_the_tiny_case():
    from synth import make_case

    out = bench.cpu_baseline(make_case("tiny"), 6, 2)
    assert out["kind"] == "oracle" and out["unit"] == "GUPS" and out["value"] > 0
    assert isinstance(out["cores"], int) and out["cores"] >= 1
    assert "6 of 120 views" in out["sample"]
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    json.dumps(out)


def test_kernel_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int f(int a) { return a + 1; }  // one\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("k.hip",))
    h0 = bench.kernel_source_hash()
    src.write_text("/* header */\nint f(int a)\n{\n    return a + 1;   // two\n}\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("int f(int a) { return a + 2; }\n")
    assert bench.kernel_source_hash() != h0
