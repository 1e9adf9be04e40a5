"""bench.py end to end on a small state: the one JSON line and its contract (metric, value,
steps, roofline with bound / achieved / peak / fraction, per-precision figures, serving
statistics), with the same code path as the 16-qubit benchmark but 11 qubits, 4 layers and a
40-request stream, so it runs in about a minute."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_contract():
    print("[gpu-case] bench.py n=11 layers=4 serve=40", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "11", "--layers", "4", "--steps", "1",
           "--warmup", "1", "--width", "2", "--no-cpu-baseline", "--serve-requests", "40", "--plain-budget-s", "2"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=280)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1  # exactly one JSON line on stdout
    d = json.loads(lines[0])
    assert d["metric"] == "16-qubit DM superop applies/s" and d["unit"] == "applies/s"
    assert d["value"] > 0 and d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["dtype"] == "f64" and d["data"] == "synthetic"
    assert d["config"]["n_qubits"] == 11 and d["config"]["layers"] == 4 and "workload" in d["config"]
    assert abs(d["ms_per_step"] * d["value"] / 1e3 - d["config"]["fused_applies_per_step"]) <= 1e-2 * d["config"]["fused_applies_per_step"]
    rl = d["roofline"]
    assert rl["bound"] in ("hbm", "mfma") and rl["achieved"] > 0 and rl["peak"] > 0
    assert rl["unit"] == ("GB/s" if rl["bound"] == "hbm" else "TFLOP/s")
    assert rl["frac"] == pytest.approx(rl["achieved"] / rl["peak"], abs=2e-4)
    assert rl["traffic"] is None  # the committed counter summary is for 16 qubits
    for prec in ("f64", "f32"):
        x = d[prec]
        assert x["applies_per_s"] > 0 and x["fused_applies"] > 0
        assert 0.99 < x["trace"] < 1.01
        if "mfma_flops_executed" in x["roofline"]:
            assert x["roofline"]["mfma_measured_TFLOPs"] > 0
        assert x["hbm"]["stream_GBs"] > 0
    assert "f32_vs_f64" in d and d["f32_vs_f64"]["max_abs_dprob"] < 1e-5
    s = d["serving"]
    assert s["batched_f32"]["completed"] == 40 and s["batched_f32"]["circuits_per_s"] > 0
    assert s["plain_f64"]["completed"] >= 1
    assert "cpu_baseline" not in d or d["cpu_baseline"] is None
