"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that a committed HBM
traffic figure is reported only for the kernel source and kernel it was measured on."""
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_reported_only_for_the_measured_source_and_kernel(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2102_12663_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("aq_kernels.hip", "aq_device.h"):
        shutil.copy(os.path.join(ROOT, "paper_2102_12663_amd", "csrc", f), csrc / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_source_hash()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "kernel_traffic.json").write_text(json.dumps(
        {"eye64x32s0/f64": {"kernel": "step2_kernel<0, false, false, 8>", "bytes_per_launch": 1234, "kernel_hash": h}}))
    assert bench.measured_traffic("eye64x32s0/f64", "step2_kernel<0, false, false, 8> (two time steps per launch)") == 1234
    assert bench.measured_traffic("eye64x32s0/f64", "step_kernel<0, false, false, false>") is None
    assert bench.measured_traffic("eye64x32s0/f64", "step2_kernel<0, false, false, 4>") is None
    assert bench.measured_traffic("eye64x32s1/f64", "step2_kernel<0, false, false, 8>") is None
    with open(csrc / "aq_device.h", "a") as f:
        f.write("\n// changed\n")
    assert bench.kernel_source_hash() != h
    assert bench.measured_traffic("eye64x32s0/f64", "step2_kernel<0, false, false, 8>") is None
