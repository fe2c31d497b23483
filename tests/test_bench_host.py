"""Host logic of bench.py that needs no GPU."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_only_for_the_source_the_counters_were_taken_on(tmp_path, monkeypatch):
    """`traffic` comes from the committed FETCH_SIZE / WRITE_SIZE summary only
    while the kernel source has the hash recorded with it; after any change
    of that source it is null (the counters no longer describe the kernel)."""
    import bench
    src = tmp_path / "paper_2203_01120_amd" / "csrc" / "plane.hip"
    src.parent.mkdir(parents=True)
    src.write_bytes(b"// kernels\n")
    (tmp_path / "profiles").mkdir()
    rec = {"source": "paper_2203_01120_amd/csrc/plane.hip",
           "source_sha256_16": hashlib.sha256(src.read_bytes()).hexdigest()[:16],
           "kernels": {"k_apply_w": {"bytes": 124379123456.7}}}
    (tmp_path / "profiles" / "hexslab_48x48x180_hbm_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_apply_w") == 124379000000.0
    assert bench.measured_traffic("k_density_w") is None          # not profiled
    src.write_bytes(b"// kernels, changed\n")
    assert bench.measured_traffic("k_apply_w") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
