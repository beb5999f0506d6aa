"""Host-side logic of bench.py (no GPU): the one-GPU contract, form parsing
and the lookup of the committed HBM-traffic counters."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_parse_form():
    b = _bench()
    assert b.parse_form("fp32") == ("fp32", 0, False)
    assert b.parse_form("fp16x3+lanczos") == ("fp16x3", 1, False)
    assert b.parse_form("fp64+lanczos+az") == ("fp64", 1, True)


def test_traffic_lookup_follows_the_kernel_source(tmp_path, monkeypatch):
    """The counters count only for the kernel source they were taken on."""
    import hashlib
    import json
    b = _bench()
    (tmp_path / "paper_2301_04642_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = b"// kernel source\n"
    (tmp_path / "paper_2301_04642_amd" / "csrc" / "k_symprod.hip").write_bytes(src)
    sha = hashlib.sha256(src).hexdigest()[:16]
    rec = {"source_sha256_16": sha, "traffic_bytes_per_launch": {"fp32": 123}}
    prof = tmp_path / "profiles" / "k_symprod_bands_n4000_traffic.md"
    prof.write_text("# summary\n\nmachine-readable: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("fp32") == 123
    assert b.measured_traffic("fp64") is None
    (tmp_path / "paper_2301_04642_amd" / "csrc" / "k_symprod.hip").write_bytes(src + b"//\n")
    assert b.measured_traffic("fp32") is None
