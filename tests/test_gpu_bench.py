"""bench.py's JSON line on the GPU: the contract fields, a positive throughput, and a roofline
object for the dominant kernel whose fraction is priced on the bytes a launch must move (at
most the peak), for a short run (2 timed check intervals of the 512-instance batch, the
sweep stopped after 20 s, legs beyond the headline dropped)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[bench] short run: --steps 2 --warmup 1 --quick --no-cpu-baseline", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--quick", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f32" and d["config"]["workload"] and d["config"]["instances"] > 500
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0 < rf["frac"] <= 1.0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["kernel"].startswith("batch_step2_kernel<1,") and "traffic" in rf
    # algorithmic bytes per time step over the wall clock of a step stay below the peak too
    per_step_bytes = rf["bytes_per_active_node_launch"] * d["config"]["active_nodes"] / 2 * 100
    assert per_step_bytes / (d["ms_per_step"] * 1e-3) / 1e9 <= 8000.0
    assert d["sweep512"]["solves_per_s"] >= 0


def test_copy_bandwidth_is_physical():
    """The plain copy kernel over 1 GiB (2 GiB of traffic per pass, far past the 256 MB
    last-level cache) reports a positive rate below the 8 TB/s HBM peak."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    g = aq.copy_bandwidth(1 << 30, 3)
    print(f"[bench] copy kernel {g:.0f} GB/s", flush=True)
    assert 1000.0 < g < 8000.0
