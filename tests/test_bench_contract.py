"""Host-side pieces of bench.py (no GPU): the one-GPU refusal, the stored
counter lookup and the step-kernel code hash it is keyed by."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stored_traffic_matches_the_current_code():
    entries = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["entries"]
    sha = bench.kernel_source_hash()
    assert all(e["kernel_sha"] == sha for e in entries), "profiles/traffic.json was taken on other kernel code"
    for e in entries:
        assert bench.stored_traffic(e["storage"], e["n_sites"], e["order"]) == e["bytes_per_launch"]
        assert bench.stored_traffic(e["storage"], e["n_sites"], "morton") is None
    assert bench.stored_traffic("f64", 12345, "bands7") is None


def test_code_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = os.path.join(ROOT, "paper_2202_11770_amd", "csrc")
    root = tmp_path / "r"
    (root / "paper_2202_11770_amd" / "csrc").mkdir(parents=True)
    for name in ("hlb_device.h", "hlb_kernels.hip", "hlb_internal.h"):
        (root / "paper_2202_11770_amd" / "csrc" / name).write_text(open(os.path.join(csrc, name)).read())
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.kernel_source_hash()
    k = root / "paper_2202_11770_amd" / "csrc" / "hlb_kernels.hip"
    k.write_text(k.read_text() + "\n// a comment\n/* and a\n block */\n")
    assert bench.kernel_source_hash() == h0
    k.write_text(k.read_text() + "\nstatic int extra_code = 1;\n")
    assert bench.kernel_source_hash() != h0
