"""Host-side parts of the benchmark contract (no GPU): the one-GPU refusal,
and the rule that a committed HBM-traffic record is used only while the
kernel source it was measured on is unchanged (comments aside)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_code_only_ignores_comments_and_blank_space():
    b = _bench()
    a = "int x = 1; // one\n/* block\n comment */\n\n  int y = 2;\n"
    assert b._code_only(a) == b._code_only("int x = 1;\nint y = 2;")
    assert b._code_only(a) != b._code_only("int x = 1;\nint y = 3;")


def test_traffic_record_needs_matching_source(tmp_path, monkeypatch):
    b = _bench()
    sha = b.source_sha("butterfly.hip")
    assert sha and len(sha) == 64
    rec = {"kernel": "void sht::k_bf_level<4, double>(...)", "source": "butterfly.hip", "source_sha256": sha,
           "L": 4095, "nside": 2048, "nmaps": 4, "bytes_per_launch": 123}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"records": [rec]}))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.measured_traffic("void sht::k_bf_level<4, double>", 4095, 2048, 4) == 123
    assert b.measured_traffic("void sht::k_bf_level<4, double>", 2047, 1024, 4) is None  # other workload
    rec["source_sha256"] = "0" * 64  # measured on other code
    f.write_text(json.dumps({"records": [rec]}))
    assert b.measured_traffic("void sht::k_bf_level<4, double>", 4095, 2048, 4) is None
