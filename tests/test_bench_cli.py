"""bench.py's host-side contract on the CPU: a request for more than one GPU is refused
with a JSON message and a non-zero status (the path runs on one GPU), and the
kernel-source hash that guards the stored HBM-traffic figure ignores layout but not
tokens."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_kernel_source_hash_ignores_layout(tmp_path, monkeypatch):
    sys.path.insert(0, str(ROOT))
    import bench

    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n  return x + 1;\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["a.hip"])
    h1 = bench.kernel_source_hash()
    a.write_text("int f(int x)\n{\n    return x + 1;  \n}\n\n")
    assert bench.kernel_source_hash() == h1
    a.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_hash() != h1
