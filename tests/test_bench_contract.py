"""The bench's command-line contract: one JSON line with the fields the
throughput report needs (GPU run on a small grid), and a clear refusal of
several GPUs (CPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_several_gpus_are_refused():
    r = _bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


@pytest.mark.gpu
def test_json_line_fields():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, steps, warmup = 128, 20, 2
    print(f"case: bench.py --n {n} --steps {steps} --warmup {warmup}", flush=True)
    r = _bench("--n", str(n), "--steps", str(steps), "--warmup", str(warmup), "--cpu-budget", "1",
               "--compare-steps", "10", "--tune-iter", "4", "--tune-rep", "1")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert isinstance(d["metric"], str) and d["metric"]
    assert d["unit"] == "Gpt/s" and d["value"] > 0
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["ms_per_step"] > 0 and d["higher_is_better"] is True and d["scaling"] == "weak"
    assert d["dtype"] == "f32" and d["data"] == "synthetic" and "vs_baseline" in d
    assert isinstance(d["config"]["workload"], str) and d["config"]["workload"]
    # value = points per step / time per step.
    assert abs(d["value"] - n ** 3 / (d["ms_per_step"] * 1e-3) / 1e9) <= 1e-3 * d["value"] + 1e-3
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    if d["config"]["tune"].get("mode", "one-step") == "one-step":
        assert abs(rf["achieved"] - 16 * n ** 3 / (d["ms_per_step"] * 1e-3) / 1e9) <= 1e-3 * rf["achieved"] + 0.1
    assert rf["traffic"] is None or rf["traffic"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == "Gpt/s"
    assert isinstance(cb["sample"], str) and cb["sample"]
