"""bench.py pieces that run without a GPU: the refusal of several GPUs, the
roofline arithmetic of the JSON line, and the CPU baseline's fields."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "one GPU" in r.stdout
    assert r.stdout.strip() == ""   # no JSON line


class _FakeGabi:
    FP64, FP32_PAIR, SCHEME_SYMMETRIC = 0, 1, 1

    @staticmethod
    def tune_get(precision, bucket):
        return (1, 1, 1, 0)


def test_roofline_arithmetic():
    n = 20480
    products = 30
    avg_ms = 0.25
    res = {"timed_products_fp32": products, "timed_products_fp64": 3,
           "kernel_total_ms": {"fp32": products * avg_ms, "fp64": 3 * 0.5},
           "timed_pass_ms_per_step": 10.0, "event_solves": 2}
    r = bench.roofline(res, "fp32", n, "no-such-workload", _FakeGabi)
    flop = bench.FLOP_PER_PAIR * n * (n - 1)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["peak"] == bench.PEAK_TFLOPS["fp32"] == 157.3
    assert r["flop_per_launch"] == flop
    assert r["achieved"] == pytest.approx(flop / (avg_ms * 1e-3) / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3, rel=1e-3)
    assert r["avg_launch_ms"] == pytest.approx(avg_ms)
    assert r["traffic"] is None and r["hw_valu"] is None   # no profile for this workload
    assert r["executed_frac"] is None
    assert r["kernel"] == "gabi::sym_pair_kernel<true>"
    r64 = bench.roofline(res, "fp64", n, "no-such-workload", _FakeGabi)
    assert r64["peak"] == 78.6 and r64["kernel"] == "gabi::sym_pair_kernel<false>"
    assert bench.roofline({"timed_products_fp32": 0}, "fp32", n, "x", _FakeGabi) is None


def test_cpu_baseline_fields():
    from paper_1301_5885_amd.synth import config_problem
    p = config_problem("kirkwood", nu=4)           # N = 320
    small = config_problem("born")
    out = bench.cpu_baseline(p, 0.4, 30, small)
    assert out["kind"] == "oracle" and out["unit"] == "Gpair-kernels/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "-march=native" in out["build"]
    assert "random rows" in out["sample"]
    assert out["one_core"]["value"] > 0
    assert out["default_build"]["value"] > 0
    assert out["solve"]["kind"] == "extrapolated" and out["solve"]["products"] == 30
    assert out["solve"]["seconds_per_solve"] > 0
    assert out["small_solve"]["kind"] == "measured" and out["small_solve"]["products"] > 0
    import oracle
    assert oracle.num_threads() == out["cores"]      # thread count restored
    # the calls after the timing use the default build again
    assert oracle._lib._name.endswith("liboracle.so")


def test_potential_errors_over_samples_and_full_vector(tmp_path):
    import numpy as np
    n = 50
    rng = np.random.default_rng(0)
    ref_u = rng.normal(size=2 * n)
    idx = np.array([1, 5, 9])
    ref = {"samples": {"seed": 1, "index": idx.tolist(), "phi": ref_u[idx].tolist(),
                       "psi": ref_u[n + idx].tolist()}}
    u = ref_u.copy()
    u[5] *= 1 + 1e-6
    e = bench.potential_errors(u, ref, n)
    assert e["psi_rel_err"] == 0.0 and 0 < e["phi_rel_err"] < 1e-6
    assert bench.potential_errors(u, None, n) is None
