"""The benchmark's host-side arithmetic and contract, no GPU needed: the roofline of a pass and
of a single apply (bound, achieved rate, fraction), the copy-calibrated traffic lookup and its
invalidation when kernel sources change, and the one-GPU guard.

The expected values are written out from the definitions (bytes = one read and one write of
4^n elements; a pass executes 6 flops per complex multiply-add in 3M form, 16 x 16 per
16-element group per superoperator; datasheet peaks 8 TB/s, 78.6 and 157.3 TFLOP/s)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_pass_roofline_is_mfma_bound_at_four_superoperators():
    n, secs, m = 16, 0.037487, 3.749
    rl = bench.roofline_pass("f64", n, secs, m, alg_flops=2.0e12)
    executed = m * 6 * 16 * 4.0 ** 16
    assert rl["bound"] == "mfma" and rl["unit"] == "TFLOP/s" and rl["peak"] == 78.6
    assert rl["achieved"] == pytest.approx(executed / secs / 1e12, abs=0.01)
    assert rl["frac"] == pytest.approx(executed / secs / 78.6e12, abs=1e-4)
    assert rl["frac"] == pytest.approx(0.5246, abs=1e-4)  # the FP64 headline figure of one run
    assert rl["algorithmic_bytes"] == 2 * 4 ** 16 * 16
    assert rl["effective_frac_algorithmic"] == pytest.approx(2.0e12 / secs / 78.6e12, abs=1e-4)
    assert rl["hbm_frac"] == pytest.approx(2 * 4 ** 16 * 16 / secs / 8e12, abs=1e-4)


def test_pass_roofline_is_hbm_bound_at_two_superoperators():
    # 2 superoperators: 10.5 ms of executed flops at peak against 17.2 ms of bytes
    rl = bench.roofline_pass("f64", 16, 0.029, 2.0, alg_flops=1.1e12)
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["achieved"] == pytest.approx(2 * 4 ** 16 * 16 / 0.029 / 1e9, abs=0.1)
    # FP32: half the bytes, twice the peak
    rl = bench.roofline_pass("f32", 16, 0.0205, 4.09, alg_flops=2.2e12)
    assert rl["bound"] == "mfma" and rl["peak"] == 157.3
    assert rl["frac"] == pytest.approx(4.09 * 96 * 4.0 ** 16 / 0.0205 / 157.3e12, abs=1e-4)
    assert rl["algorithmic_bytes"] == 2 * 4 ** 16 * 8


def test_single_apply_roofline():
    k2 = bench.roofline("f64", 2, 16, 0.0267)
    assert k2["bound"] == "hbm" and k2["achieved"] == pytest.approx(2 * 4 ** 16 * 16 / 0.0267 / 1e9, abs=0.1)
    k3 = bench.roofline("f64", 3, 16, 0.0332)
    alg = 8.0 * 64 * 4.0 ** 16
    assert k3["bound"] == "mfma" and k3["frac"] == pytest.approx(alg / 0.0332 / 78.6e12, abs=1e-4)
    assert k3["mfma_flops_executed"] == pytest.approx(0.75 * alg)  # 3M: three real products of four


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    name = "apply_pass_kernel<double, 12, 512>"
    good = tmp_path / "good.txt"
    good.write_text("# summary\nsource_hash %s\nkernel %s 6.0e10 7.0e10 1 1 1.0 5\n"
                    % (bench.kernel_source_hash(), name.replace(" ", "")))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic(name) == pytest.approx(1.3e11)
    assert bench.measured_traffic("some_other_kernel<float>") is None
    stale = tmp_path / "stale.txt"
    stale.write_text("source_hash 0000000000000000\nkernel %s 6.0e10 7.0e10 1 1 1.0 5\n" % name.replace(" ", ""))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic(name) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic(name, 16) == pytest.approx(1.3e11)
    assert bench.measured_traffic(name, 12) is None  # the summary's bytes are for 16 qubits
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic(name) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
