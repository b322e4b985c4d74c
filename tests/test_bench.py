"""The benchmark's command-line contract: one JSON line with the metric,
the roofline of the fused kernel and the oracle baseline (GPU), and a clear
refusal of more than one GPU (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_json_line():
    """A short default-workload run (20 timed steps, a 2 s oracle sample): the
    warm-closure wake at 4096 x 1024 in FP64, with the FP32 and FP16-deviation
    variants and their errors against FP64."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "2",
                        "--cpu-budget", "2"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["value"] > 0
    assert d["config"]["workload"] == "wake2d_warmc" and d["dtype"] == "f64"
    pv = d["precision_variants"]
    for st in ("fp32", "fp16dev"):
        err = pv[st]["rel_l2_vs_fp64"]
        assert set(err) == {"n-1", "mz", "mx", "ez"}
        # measured at 400 steps: FP32 <= 2e-6, FP16 deviations <= 1e-3
        assert max(err.values()) <= (1e-4 if st == "fp32" else 1e-2), (st, err)
        assert pv[st]["speedup_vs_fp64"] > 1.0
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9
    assert d["cpu_baseline"]["kind"] == "oracle" and d["cpu_baseline"]["cores"] >= 1
