"""bench.py command line on the CPU: one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""



def test_committed_counters_apply_only_to_the_kernel_they_were_taken_on(tmp_path, monkeypatch):
    # The roofline's measured HBM traffic and VALU count come from committed
    # rocprofv3 summaries that carry a hash of the fused kernel's sources;
    # they must go stale when any of those files changes.
    import json
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    for rel in bench.FUSED_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    rec = {"sources": bench.FUSED_SOURCES, "sources_sha256": bench.kernel_sources_sha256(bench.FUSED_SOURCES)}
    json.dump(dict(rec, traffic_bytes_per_launch=4.1e6), open(tmp_path / "profiles/fused_c2_traffic.json", "w"))
    json.dump(dict(rec, sq_insts_valu_per_launch=1.4e8), open(tmp_path / "profiles/fused_c2_valu.json", "w"))
    assert bench.measured_traffic("c2") == 4.1e6
    assert bench.measured_valu("c2") == 1.4e8
    assert bench.measured_traffic("c4") is None
    with open(tmp_path / "paper_2109_13030_amd/csrc/am_device.h", "a") as f:
        f.write("\n")
    assert bench.measured_traffic("c2") is None
    assert bench.measured_valu("c2") is None
