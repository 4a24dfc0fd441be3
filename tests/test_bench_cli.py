"""Host-side behaviour of bench.py: one GPU only, and stored HBM traffic reported
only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_stored_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "k_x_kagome432_L6F64_bf16_1x_hbm_traffic.md"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abcd")
    assert bench.stored_traffic("kagome432_L6F64", "bf16_1x", "k_x") is None          # no summary
    f.write_text("traffic_bytes_per_launch: 123\nsource_sha256_16: abcd\n")
    assert bench.stored_traffic("kagome432_L6F64", "bf16_1x", "k_x") == 123
    f.write_text("traffic_bytes_per_launch: 123\nsource_sha256_16: ffff\n")           # sources changed
    assert bench.stored_traffic("kagome432_L6F64", "bf16_1x", "k_x") is None

